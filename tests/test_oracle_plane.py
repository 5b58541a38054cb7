"""Pins of the planar oracle (the f-plane scheme of section 4.2) against
facts that do not come from the oracle itself: the r = 0 case is a textbook
first-order finite-volume scheme, a lake at rest stays at rest, the exact
momentum budget of the Coriolis force on a periodic domain, the x <-> y
mirror symmetry, translation equivariance, and consistency of the operator
on steady geostrophic jets (exact steady states of the planar equations)."""
import numpy as np
import pytest

from oracle import PlaneDG

G, F = 9.81, 1.0e-4
LX, LY = 1.0e7, 0.8e7


def random_state(m, seed, h0=1000.0, dh=5.0, vel=2.0):
    """Smooth random fields projected onto the basis (a few Fourier modes)."""
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, 6)

    def fun(x, y):
        kx, ky = 2 * np.pi / m.lx, 2 * np.pi / m.ly
        h = h0 + dh * (np.sin(kx * x + ph[0]) * np.cos(ky * y + ph[1]) + 0.5 * np.cos(2 * kx * x + ph[2]))
        u = vel * (0.7 + np.cos(ky * y + ph[3]) * np.sin(kx * x + ph[4]))
        v = vel * (-0.4 + np.sin(2 * ky * y + ph[5]))
        return np.stack([h, h * u, h * v])

    return m.project(fun)


# ---------------------------------------------------------------- r = 0 is first-order finite volume
def _fv_rhs(Q, dx, dy, alpha=None):
    """First-order finite volume with the local Lax-Friedrichs flux on a
    doubly periodic grid of cell averages Q[j, i, v]:
    dQ/dt = -(F_E - F_W)/dx - (G_N - G_S)/dy + (0, f hv, -f hu).
    alpha given: the global Lax-Friedrichs flux with that fixed speed."""
    ny, nx, _ = Q.shape
    out = np.zeros_like(Q)

    def fx(q):
        h, hu, hv = q
        return np.array([hu, hu * hu / h + G * h * h / 2, hu * hv / h])

    def fy(q):
        h, hu, hv = q
        return np.array([hv, hu * hv / h, hv * hv / h + G * h * h / 2])

    def llf(ql, qr, fl, c):
        a = max(abs(ql[c] / ql[0]) + np.sqrt(G * ql[0]), abs(qr[c] / qr[0]) + np.sqrt(G * qr[0]))
        a = a if alpha is None else alpha
        return 0.5 * (fl(ql) + fl(qr)) - 0.5 * a * (qr - ql)

    for j in range(ny):
        for i in range(nx):
            q = Q[j, i]
            FE = llf(q, Q[j, (i + 1) % nx], fx, 1)
            FW = llf(Q[j, (i - 1) % nx], q, fx, 1)
            GN = llf(q, Q[(j + 1) % ny, i], fy, 2)
            GS = llf(Q[(j - 1) % ny, i], q, fy, 2)
            S = np.array([0.0, F * q[2], -F * q[1]])
            out[j, i] = -(FE - FW) / dx - (GN - GS) / dy + S
    return out


def test_plane_r0_equals_first_order_finite_volume():
    nx, ny = 9, 7
    rng = np.random.default_rng(3)
    Q = np.empty((ny, nx, 3))
    Q[..., 0] = 1000 + 5 * rng.standard_normal((ny, nx))
    Q[..., 1] = Q[..., 0] * 2 * rng.standard_normal((ny, nx))
    Q[..., 2] = Q[..., 0] * 2 * rng.standard_normal((ny, nx))
    m = PlaneDG(nx, ny, 0, LX, LY, gravity=G, f=F)
    got = m.rhs((2.0 * Q).reshape(m.E, 3, 1)).reshape(ny, nx, 3) / 2.0
    ref = _fv_rhs(Q, LX / nx, LY / ny)
    scale = np.abs(ref).max(axis=(0, 1))
    assert np.all(np.abs(got - ref).max(axis=(0, 1)) <= 1e-13 * scale)


def test_plane_r0_global_alpha_equals_global_lax_friedrichs():
    """The fixed-speed Rusanov branch of the plane at r = 0: first-order
    finite volume with the global Lax-Friedrichs flux."""
    nx, ny, alpha = 9, 7, 130.0
    rng = np.random.default_rng(4)
    Q = np.empty((ny, nx, 3))
    Q[..., 0] = 1000 + 5 * rng.standard_normal((ny, nx))
    Q[..., 1] = Q[..., 0] * 2 * rng.standard_normal((ny, nx))
    Q[..., 2] = Q[..., 0] * 2 * rng.standard_normal((ny, nx))
    m = PlaneDG(nx, ny, 0, LX, LY, gravity=G, f=F, alpha_mode="global", alpha=alpha)
    got = m.rhs((2.0 * Q).reshape(m.E, 3, 1)).reshape(ny, nx, 3) / 2.0
    ref = _fv_rhs(Q, LX / nx, LY / ny, alpha=alpha)
    scale = np.abs(ref).max(axis=(0, 1))
    assert np.all(np.abs(got - ref).max(axis=(0, 1)) <= 1e-13 * scale)
    assert np.abs(_fv_rhs(Q, LX / nx, LY / ny) - ref).max() > 1e-6 * np.abs(ref).max()


@pytest.mark.parametrize("order", [0, 1, 2, 3, 5])
def test_plane_lake_at_rest(order):
    m = PlaneDG(6, 5, order, LX, LY, gravity=G, f=F)
    q = np.zeros((m.E, 3, m.N))
    q[:, 0, 0] = 2.0 * 1000.0
    d = m.rhs(q)
    # size of the cancelling pressure terms: g h^2/2 times the derivative
    # tables (2/dx) P~' (up to about (r+1)^2) per unit mass
    scale = G * 1000.0 ** 2 / 2 / min(m.dx, m.dy) * (order + 1) ** 2
    assert np.abs(d).max() <= 1e-14 * scale


@pytest.mark.parametrize("order", [1, 2, 4])
def test_plane_momentum_budget(order):
    """On a periodic domain the fluxes telescope: d/dt int h = 0,
    d/dt int hu = f int hv, d/dt int hv = -f int hu, exactly for the
    discrete operator (the source integral of mode 00 is exact)."""
    m = PlaneDG(8, 6, order, LX, LY, gravity=G, f=F)
    q = random_state(m, 10 + order)
    d = m.rhs(q)
    md, mq = m.mass(d), m.mass(q)
    ref = np.array([0.0, F * mq[2], -F * mq[1]])
    scale = F * np.abs(mq).max() + 1e-300
    assert np.all(np.abs(md - ref) <= 1e-10 * scale + 1e-13 * np.abs(ref)), (md, ref)
    # and the budget is not trivially zero
    assert abs(ref[1]) > 1e-3 * scale or abs(ref[2]) > 1e-3 * scale


@pytest.mark.parametrize("order", [1, 3])
def test_plane_transpose_symmetry(order):
    """Mirroring x <-> y maps the system to itself with hu <-> hv, modes
    (a, b) -> (b, a) and f -> -f (the mirror reverses orientation)."""
    nx, ny = 7, 5
    m = PlaneDG(nx, ny, order, LX, LY, gravity=G, f=F)
    mt = PlaneDG(ny, nx, order, LY, LX, gravity=G, f=-F)
    n = order + 1
    q = random_state(m, 7)

    def transpose(qq, nx_, ny_):
        g = qq.reshape(ny_, nx_, 3, n, n)                    # [j, i, v, b, a]
        g = g.transpose(1, 0, 2, 4, 3)[:, :, [0, 2, 1]]      # [i, j, v', a, b]
        return np.ascontiguousarray(g).reshape(nx_ * ny_, 3, n * n)

    d = m.rhs(q)
    dt = mt.rhs(transpose(q, nx, ny))
    ref = transpose(d, nx, ny)
    assert np.abs(dt - ref).max() <= 1e-12 * np.abs(ref).max()


def test_plane_translation_equivariance():
    m = PlaneDG(8, 6, 2, LX, LY, gravity=G, f=F)
    q = random_state(m, 5)
    d = m.rhs(q).reshape(6, 8, 3, -1)
    for sj, si in [(0, 3), (2, 0), (4, 5)]:
        qs = np.roll(q.reshape(6, 8, 3, -1), (sj, si), axis=(0, 1)).reshape(m.E, 3, -1)
        ds = m.rhs(qs).reshape(6, 8, 3, -1)
        assert np.abs(ds - np.roll(d, (sj, si), axis=(0, 1))).max() <= 1e-12 * np.abs(d).max()


def _jet(m, along_x):
    """Steady geostrophic jet: u = U sin(k y), h = h0 + (f U / (g k)) cos(k y)
    (along x), or v = U sin(k x), h = h0 - (f U / (g k)) cos(k x)."""
    U, h0 = 20.0, 1000.0

    def fun(x, y):
        if along_x:
            k = 2 * np.pi / m.ly
            h = h0 + F * U / (G * k) * np.cos(k * y)
            return np.stack([h, h * U * np.sin(k * y), 0 * h])
        k = 2 * np.pi / m.lx
        h = h0 - F * U / (G * k) * np.cos(k * x)
        return np.stack([h, 0 * h, h * U * np.sin(k * x)])

    return fun


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("along_x", [True, False])
def test_plane_geostrophic_jet_consistency(order, along_x):
    """The jets are exact steady states, so the DG operator on their
    projection goes to zero with the mesh width at about order r; a wrong
    sign of f or of a flux derivative leaves an O(1) residual."""
    errs = []
    for n in (6, 12, 24):
        m = PlaneDG(n, n, order, LX, LY, gravity=G, f=F)
        q = m.project(_jet(m, along_x))
        d = m.rhs(q)
        scale = F * 20.0 * 1000.0                 # size of the balanced terms f h u
        errs.append(np.abs(d[:, 1:]).max() / scale)
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert errs[-1] < [0.3, 0.05, 0.02][order - 1], errs
    assert rates[-1] > order - 0.75, (errs, rates)
