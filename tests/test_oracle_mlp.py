"""Pins of the MLP oracle and of the order-projection oracle."""
import math

import numpy as np
import pytest

from dg_inputs import band_limited_state
from oracle import SphereDG, mlp, project_order

torch = pytest.importorskip("torch")


def small_params(seed, n_in=7, n_hid=9, n_out=5):
    return mlp.init_params(seed, n_in, n_hid, n_out)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-8, 8, 4000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 65504.0, 3.4e38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)
    assert mlp.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0            # tie to even
    assert mlp.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6


def test_gelu_and_derivative_match_torch():
    z = np.linspace(-6, 6, 241)
    zt = torch.from_numpy(z).requires_grad_(True)
    y = torch.nn.functional.gelu(zt, approximate="none")
    y.sum().backward()
    np.testing.assert_allclose(mlp.gelu(z), y.detach().numpy(), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(mlp.gelu_grad(z), zt.grad.numpy(), rtol=1e-13, atol=1e-15)


def test_backward_matches_central_differences():
    """Exact (unrounded) gradients against central differences in FP64."""
    p = small_params(3)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((11, 7))
    T = rng.standard_normal((11, 5))
    mask = np.array([0.0, 1.0, 1.0, 1.0, 1.0])
    Y, cache = mlp.forward(p, X, exact=True)
    g = mlp.backward(p, cache, Y, T, mask, exact=True)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(mlp.forward(p, X, exact=True)[0], T, mask)
            flat[idx] = old - h
            lm = mlp.loss(mlp.forward(p, X, exact=True)[0], T, mask)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (k, idx, fd, an)


def test_backward_matches_torch_autograd():
    """Exact gradients equal torch autograd of the same network (library)."""
    p = small_params(5)
    rng = np.random.default_rng(6)
    X = rng.standard_normal((13, 7))
    T = rng.standard_normal((13, 5))
    mask = np.ones(5)
    Y, cache = mlp.forward(p, X, exact=True)
    g = mlp.backward(p, cache, Y, T, mask, exact=True)
    tp = {k: torch.from_numpy(v.copy()).requires_grad_(True) for k, v in p.items()}
    Xt = torch.from_numpy(X)
    a = torch.nn.functional.gelu(Xt @ tp["W1"] + tp["b1"])
    a = torch.nn.functional.gelu(a @ tp["W2"] + tp["b2"])
    out = a @ tp["W3"] + tp["b3"]
    ((out - torch.from_numpy(T)) ** 2).mean().backward()
    for k in p:
        np.testing.assert_allclose(g[k], tp[k].grad.numpy(), rtol=1e-11, atol=1e-14)


def test_adam_matches_torch():
    p = small_params(7)
    tp = {k: torch.from_numpy(v.copy()).requires_grad_(True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    state = {}
    rng = np.random.default_rng(8)
    for _ in range(4):
        g = {k: rng.standard_normal(v.shape) for k, v in p.items()}
        mlp.adam(p, g, state)
        opt.zero_grad()
        for k in tp:
            tp[k].grad = torch.from_numpy(g[k].copy())
        opt.step()
    for k in p:
        np.testing.assert_allclose(p[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15)


def test_stencil_features_brute_force():
    n_lon, n_lat = 5, 4
    q = np.arange(n_lon * n_lat * 12, dtype=np.float64).reshape(n_lon * n_lat, 3, 4)
    X = mlp.stencil_features(q, n_lon, n_lat)
    for j in range(n_lat):
        for i in range(n_lon):
            e = j * n_lon + i
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    jj = min(max(j + dj, 0), n_lat - 1)
                    ii = (i + di) % n_lon
                    k = ((dj + 1) * 3 + (di + 1)) * 12
                    np.testing.assert_array_equal(X[e, k:k + 12], q[jj * n_lon + ii].reshape(12))


def test_projection_reproduces_lower_order_and_conserves_mass():
    """P_1 of a state that is already of degree 1 returns it; P_1 keeps the
    cos-weighted integral of every variable (constants are in the target space)."""
    n_lon, n_lat = 12, 6
    m1, m4 = SphereDG(n_lon, n_lat, 1), SphereDG(n_lon, n_lat, 4)
    q1, _ = band_limited_state(n_lon, n_lat, 1, 4, 3)
    # embed q1 into the r = 4 basis: modes with a, b <= 1 copied
    q4 = np.zeros((m4.E, 3, m4.N))
    for b in range(2):
        for a in range(2):
            q4[:, :, b * 5 + a] = q1[:, :, b * 2 + a]
    np.testing.assert_allclose(project_order(q4, m4, m1), q1, rtol=0, atol=1e-10 * np.abs(q1).max())
    q4r, _ = band_limited_state(n_lon, n_lat, 4, 6, 5)
    p1 = project_order(q4r, m4, m1)
    np.testing.assert_allclose(m1.mass(p1), m4.mass(q4r), rtol=1e-12)


@pytest.mark.parametrize("src,dst", [(4, 0), (4, 2), (5, 3), (3, 2)])
def test_projection_any_order_is_the_cos_weighted_orthogonal_projection(src, dst):
    """project_order onto orders other than 1 (the plain runs of the
    equal-error comparison start from it): a field already of the target
    degree is returned; the residual q - P q is orthogonal, in the
    cos-weighted inner product of the mass matrix, to every target basis
    function (checked with the source's own mass matrix, a different
    computation); projections nest, P_k P_m = P_k for k < m; mass is kept."""
    n_lon, n_lat = 10, 5
    ms, md = SphereDG(n_lon, n_lat, src), SphereDG(n_lon, n_lat, dst)
    ns, nd = src + 1, dst + 1

    def embed(q, n_lo, n_hi):
        out = np.zeros((q.shape[0], 3, n_hi * n_hi))
        for b in range(n_lo):
            out[:, :, b * n_hi:b * n_hi + n_lo] = q[:, :, b * n_lo:(b + 1) * n_lo]
        return out

    qd, _ = band_limited_state(n_lon, n_lat, dst, 4, 8)
    np.testing.assert_allclose(project_order(embed(qd, nd, ns), ms, md), qd, rtol=0,
                               atol=1e-10 * np.abs(qd).max())
    q, _ = band_limited_state(n_lon, n_lat, src, 6, 9)
    p = project_order(q, ms, md)
    r = ms.grid(q - embed(p, nd, ns))                       # residual in the source basis
    for b in range(nd):
        for a in range(nd):
            # <phi_(a,b), r>_M: row (b, a) of the source mass matrix against r
            row = b * ns + a
            ip = np.einsum("jn,jivn->jiv", ms.M[:, row, :], r)
            assert np.abs(ip).max() <= 1e-10 * np.abs(np.einsum("jn,jivn->jiv", np.abs(ms.M[:, row, :]),
                                                                 np.abs(ms.grid(q)))).max()
    if dst > 0:
        mid = SphereDG(n_lon, n_lat, dst - 1)
        np.testing.assert_allclose(project_order(p, md, mid), project_order(q, ms, mid), rtol=0,
                                   atol=1e-10 * np.abs(q).max())
    np.testing.assert_allclose(md.mass(p), ms.mass(q), rtol=1e-12)
