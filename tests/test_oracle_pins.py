"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: quadrature exactness, closed
forms, library routines used as an independent evaluation, a textbook
first-order finite-volume scheme (the r = 0 case of the method), a literal
quadrature sum of the weak form over each element's four faces (the form of
the Rusanov functor listing of section 3.1), physical invariants (lake at
rest, conservation, symmetries), consistency of the operator on smooth
fields, and the Butcher tableaux printed in the paper.
"""
import json
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from scipy import integrate

from oracle import SphereDG, butcher_step, gauss_legendre, legendre, ssp_rk3
from dg_inputs import band_limited_state, lake_at_rest_state

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
R, G, OM = 6.371e6, 9.80616, 7.292e-5


# ---------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8, 12, 32])
def test_gauss_legendre_exactness(n):
    """An n-point Gauss rule integrates x^k exactly for k <= 2n-1 and not
    for k = 2n (which fixes n)."""
    x, w = gauss_legendre(n)
    for k in range(2 * n):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14 * max(1.0, n), (n, k)
    # x^(2n): the error is the Gauss-Legendre remainder constant
    # 2^(2n+1) (n!)^4 / ((2n+1) ((2n)!)^2), which is nonzero
    from math import factorial
    k = 2 * n
    exact = 2.0 / (k + 1)
    remainder = 2.0 ** (k + 1) * factorial(n) ** 4 / ((k + 1) * factorial(k) ** 2)
    if remainder > 1e-12:
        assert abs((exact - np.sum(w * x ** k)) - remainder) <= 1e-7 * remainder + 1e-15


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 9, 32])
def test_gauss_legendre_matches_library(n):
    x, w = gauss_legendre(n)
    xr, wr = npleg.leggauss(n)
    np.testing.assert_allclose(x, xr, rtol=0, atol=2e-15)
    np.testing.assert_allclose(w, wr, rtol=0, atol=2e-15)


# ---------------------------------------------------------------- basis
@pytest.mark.parametrize("order", [0, 1, 3, 5, 7])
def test_legendre_orthonormal_exact(order):
    """Exact polynomial integration with numpy's Legendre series objects."""
    x = np.linspace(-1, 1, 7)
    P, dP = legendre(order, x)
    for a in range(order + 1):
        ca = np.zeros(a + 1)
        ca[a] = np.sqrt((2 * a + 1) / 2.0)
        pa = npleg.Legendre(ca)
        np.testing.assert_allclose(P[:, a], pa(x), atol=1e-13)
        np.testing.assert_allclose(dP[:, a], pa.deriv()(x), atol=1e-12)
        for b in range(order + 1):
            cb = np.zeros(b + 1)
            cb[b] = np.sqrt((2 * b + 1) / 2.0)
            prod = (pa * npleg.Legendre(cb)).integ()
            val = prod(1.0) - prod(-1.0)
            assert abs(val - (a == b)) < 1e-13


@pytest.mark.parametrize("order", [0, 2, 5])
def test_legendre_orthonormal_brute_force(order):
    """Brute-force orthonormality of the 2-D tensor basis on a 40-point rule."""
    xq, wq = npleg.leggauss(40)
    P, _ = legendre(order, xq)
    n = order + 1
    phi = np.einsum("pa,sb->psba", P, P).reshape(40 * 40, n * n)
    wt = np.outer(wq, wq).ravel()
    gram = (phi.T * wt) @ phi
    np.testing.assert_allclose(gram, np.eye(n * n), atol=1e-13)


def test_legendre_endpoint_closed_form():
    P, _ = legendre(7, np.array([-1.0, 1.0]))
    a = np.arange(8)
    np.testing.assert_allclose(P[1], np.sqrt((2 * a + 1) / 2.0), rtol=1e-15)
    np.testing.assert_allclose(P[0], (-1.0) ** a * np.sqrt((2 * a + 1) / 2.0), rtol=1e-15)


# ---------------------------------------------------------------- mass
def test_mass_r0_closed_form():
    """r = 0: M_00 = (dlam/4)(sin theta_t - sin theta_b) (phi_00 = 1/2)."""
    m = SphereDG(12, 7, 0)
    th = m.theta_edge
    expect = 0.25 * m.dlam * (np.sin(th[1:]) - np.sin(th[:-1]))
    np.testing.assert_allclose(m.M[:, 0, 0], expect, rtol=1e-14)


@pytest.mark.parametrize("order", [0, 1, 3, 5])
def test_mass_sphere_area(order):
    """Mass of h = 1 is the sphere's area 4 pi R^2."""
    m = SphereDG(10, 6, order)
    q = np.zeros((m.E, 3, m.N))
    q[:, :, 0] = 2.0
    np.testing.assert_allclose(m.mass(q), 4 * np.pi * R ** 2, rtol=1e-13)


def test_mass_longitude_blocks_and_dblquad():
    """M is diagonal in the longitude degree a; entries agree with SciPy's
    adaptive dblquad of phi_m phi_m' cos(theta) over a pole-row element."""
    m = SphereDG(8, 6, 2)
    n = m.n
    for j in (0, 2):
        M = m.M[j]
        for i1 in range(m.N):
            for i2 in range(m.N):
                if i1 % n != i2 % n:
                    assert abs(M[i1, i2]) < 1e-14 * np.abs(M).max()
    j = 0
    lam0, th0 = 0.0, m.theta_edge[j]

    def phi(mm, xi, eta):
        a, b = mm % n, mm // n
        ca = np.zeros(a + 1); ca[a] = np.sqrt((2 * a + 1) / 2)
        cb = np.zeros(b + 1); cb[b] = np.sqrt((2 * b + 1) / 2)
        return npleg.legval(xi, ca) * npleg.legval(eta, cb)

    for (i1, i2) in [(0, 0), (0, 6), (3, 3), (4, 7), (8, 2)]:
        f = lambda th, lam: (phi(i1, 2 * (lam - lam0) / m.dlam - 1, 2 * (th - th0) / m.dth - 1)
                             * phi(i2, 2 * (lam - lam0) / m.dlam - 1, 2 * (th - th0) / m.dth - 1)
                             * np.cos(th))
        val, _ = integrate.dblquad(f, lam0, lam0 + m.dlam, th0, th0 + m.dth, epsabs=1e-15, epsrel=1e-13)
        assert abs(val - m.M[j, i1, i2]) < 1e-12 * max(abs(val), 1e-3), (i1, i2, val, m.M[j, i1, i2])


# ---------------------------------------------------------------- r = 0 is first-order finite volume
def _fv_rhs(Q, n_lon, n_lat, balanced=True, alpha=None):
    """Textbook first-order finite volume on the lat-lon grid with the local
    Lax-Friedrichs flux, written for cell values Q[j, i, v]:
    dlam (sin t - sin b) dQ/dt = -dth (F_E - F_W) - dlam (G_N - G_S) + dlam dth S(centre).
    alpha given: the global Lax-Friedrichs flux, one fixed speed at every face."""
    dl, dt_ = 2 * np.pi / n_lon, np.pi / n_lat
    out = np.zeros_like(Q)
    for j in range(n_lat):
        tb = -np.pi / 2 + j * dt_
        tt = tb + dt_
        tc = tb + dt_ / 2
        cb = 0.0 if j == 0 else np.cos(tb)
        ct = 0.0 if j == n_lat - 1 else np.cos(tt)
        for i in range(n_lon):
            def fl(q):
                h, hu, hv = q
                return np.array([hu, hu * hu / h + G * h * h / 2, hu * hv / h]) / R

            def gl(q, c):
                h, hu, hv = q
                return c * np.array([hv, hu * hv / h, hv * hv / h + G * h * h / 2]) / R

            def llf_lam(ql, qr):
                a = max(abs(ql[1] / ql[0]) + np.sqrt(G * ql[0]), abs(qr[1] / qr[0]) + np.sqrt(G * qr[0]))
                a = a if alpha is None else alpha
                return 0.5 * (fl(ql) + fl(qr)) - 0.5 * a / R * (qr - ql)

            def llf_th(qs, qn, c):
                a = max(abs(qs[2] / qs[0]) + np.sqrt(G * qs[0]), abs(qn[2] / qn[0]) + np.sqrt(G * qn[0]))
                a = a if alpha is None else alpha
                return 0.5 * (gl(qs, c) + gl(qn, c)) - 0.5 * a * c / R * (qn - qs)

            q = Q[j, i]
            FE = llf_lam(q, Q[j, (i + 1) % n_lon])
            FW = llf_lam(Q[j, (i - 1) % n_lon], q)
            GN = np.zeros(3) if j == n_lat - 1 else llf_th(q, Q[j + 1, i], ct)
            GS = np.zeros(3) if j == 0 else llf_th(Q[j - 1, i], q, cb)
            h, hu, hv = q
            u = hu / h
            sfac = (cb - ct) / dt_ if balanced else np.sin(tc)
            cor = 2 * OM * np.sin(tc) * np.cos(tc) + u * np.sin(tc) / R
            S = np.array([0.0, cor * hv, -G * h * h / 2 * sfac / R - cor * hu])
            out[j, i] = (-dt_ * (FE - FW) - dl * (GN - GS) + dl * dt_ * S) / (dl * (np.sin(tt) - np.sin(tb)))
    return out


@pytest.mark.parametrize("metric", ["balanced", "pointwise"])
def test_r0_equals_first_order_finite_volume(metric):
    n_lon, n_lat = 12, 7
    rng = np.random.default_rng(11)
    Q = np.empty((n_lat, n_lon, 3))
    Q[..., 0] = 1e4 + 100 * rng.standard_normal((n_lat, n_lon))
    Q[..., 1] = Q[..., 0] * 20 * rng.standard_normal((n_lat, n_lon))
    Q[..., 2] = Q[..., 0] * 20 * rng.standard_normal((n_lat, n_lon))
    m = SphereDG(n_lon, n_lat, 0, metric=metric)
    q = (2.0 * Q).reshape(m.E, 3, 1)                 # phi_00 = 1/2
    got = m.rhs(q).reshape(n_lat, n_lon, 3) / 2.0
    ref = _fv_rhs(Q, n_lon, n_lat, balanced=(metric == "balanced"))
    scale = np.abs(ref).max(axis=(0, 1))
    assert np.all(np.abs(got - ref).max(axis=(0, 1)) <= 1e-13 * scale), (np.abs(got - ref).max(axis=(0, 1)), scale)


@pytest.mark.parametrize("alpha", [150.0, 420.0])
def test_r0_global_alpha_equals_global_lax_friedrichs(alpha):
    """The fixed-speed ("global") branch of the Rusanov flux: at r = 0 the
    method is first-order finite volume with the global Lax-Friedrichs flux,
    F^ = (F- + F+)/2 - (alpha/2R)(q+ - q-) on longitude faces and
    (alpha cos/2R)(q+ - q-) on latitude faces.  Two speeds, one below the
    local wave speed (~330 m/s) and one above, so the dissipation term is
    pinned with a coefficient that differs from the local one."""
    n_lon, n_lat = 12, 7
    rng = np.random.default_rng(12)
    Q = np.empty((n_lat, n_lon, 3))
    Q[..., 0] = 1e4 + 100 * rng.standard_normal((n_lat, n_lon))
    Q[..., 1] = Q[..., 0] * 20 * rng.standard_normal((n_lat, n_lon))
    Q[..., 2] = Q[..., 0] * 20 * rng.standard_normal((n_lat, n_lon))
    m = SphereDG(n_lon, n_lat, 0, alpha_mode="global", alpha=alpha)
    got = m.rhs((2.0 * Q).reshape(m.E, 3, 1)).reshape(n_lat, n_lon, 3) / 2.0
    ref = _fv_rhs(Q, n_lon, n_lat, alpha=alpha)
    scale = np.abs(ref).max(axis=(0, 1))
    assert np.all(np.abs(got - ref).max(axis=(0, 1)) <= 1e-13 * scale), (np.abs(got - ref).max(axis=(0, 1)), scale)
    # and it is not the local flux (the branch is taken)
    loc = _fv_rhs(Q, n_lon, n_lat)
    assert np.abs(loc - ref).max() > 1e-6 * np.abs(ref).max()


# ---------------------------------------------------------------- weak form, literal per face
def _weak_form_by_faces(q, n_lon, n_lat, order, alpha=None):
    """h(q) as the literal quadrature of equation "dg_parts" per element:
    volume term - sum over the four faces of (f* . n) phi, with the Rusanov
    flux written from each element's own side (own trace, opposite trace,
    outward normal), in physical (lambda, theta) coordinates, basis from
    numpy's legval.  alpha given: a fixed speed in place of the local
    eigenvalue estimate.  Pure Python loops: tiny meshes only."""
    n = order + 1
    xq, wq = npleg.leggauss(n)
    dl, dt_ = 2 * np.pi / n_lon, np.pi / n_lat
    Q = q.reshape(n_lat, n_lon, 3, n, n)              # [j, i, v, b, a]

    def leg(a, x, d=0):
        c = np.zeros(a + 1); c[a] = np.sqrt((2 * a + 1) / 2)
        return npleg.legval(x, npleg.legder(c, d) if d else c)

    def value(j, i, xi, eta):
        return np.array([sum(Q[j, i, v, b, a] * leg(a, xi) * leg(b, eta)
                             for a in range(n) for b in range(n)) for v in range(3)])

    def F(u):
        h, hu, hv = u
        return np.array([hu, hu * hu / h + G * h * h / 2, hu * hv / h]) / R

    def Gf(u, c):
        h, hu, hv = u
        return c * np.array([hv, hu * hv / h, hv * hv / h + G * h * h / 2]) / R

    def lat(j, eta):
        return -np.pi / 2 + j * dt_ + (1 + eta) * dt_ / 2

    out = np.zeros((n_lat, n_lon, 3, n, n))
    for j in range(n_lat):
        for i in range(n_lon):
            # volume: F dphi/dlam + G dphi/dtheta + S phi, Jacobian dl dt / 4
            for p in range(n):
                for s in range(n):
                    th = lat(j, xq[s])
                    u = value(j, i, xq[p], xq[s])
                    h, hu, hv = u
                    c, sn = np.cos(th), np.sin(th)
                    cor = 2 * OM * sn * c + hu / h * sn / R
                    S = np.array([0.0, cor * hv, -G * h * h / 2 * sn / R - cor * hu])
                    Fv, Gv = F(u), Gf(u, c)
                    for a in range(n):
                        for b in range(n):
                            dphil = (2 / dl) * leg(a, xq[p], 1) * leg(b, xq[s])
                            dphit = (2 / dt_) * leg(a, xq[p]) * leg(b, xq[s], 1)
                            phi = leg(a, xq[p]) * leg(b, xq[s])
                            out[j, i, :, b, a] += (dl * dt_ / 4) * wq[p] * wq[s] * (
                                Fv * dphil + Gv * dphit + S * phi)
            # faces: (xi or eta fixed, normal, neighbour, neighbour's coordinate)
            faces = [("E", (1, 0)), ("W", (-1, 0)), ("N", (0, 1)), ("S", (0, -1))]
            for name, nrm in faces:
                for k in range(n):
                    if name in "EW":
                        xs = 1.0 if name == "E" else -1.0
                        own = value(j, i, xs, xq[k])
                        inb = (i + nrm[0]) % n_lon
                        opp = value(j, inb, -xs, xq[k])
                        th = lat(j, xq[k])
                        c = np.cos(th)
                        spd = max(abs(own[1] / own[0]) + np.sqrt(G * own[0]),
                                  abs(opp[1] / opp[0]) + np.sqrt(G * opp[0]))
                        a_ = (spd if alpha is None else alpha) / (R * c)
                        Uo, Un = own * c, opp * c
                        fstar_n = 0.5 * (F(own) + F(opp)) * nrm[0] - 0.5 * a_ * (Un - Uo)
                        jac = dt_ / 2
                        xi_f, eta_f = xs, xq[k]
                    else:
                        ys = 1.0 if name == "N" else -1.0
                        jn = j + nrm[1]
                        if jn < 0 or jn >= n_lat:
                            continue                                  # pole: zero flux
                        own = value(j, i, xq[k], ys)
                        opp = value(jn, i, xq[k], -ys)
                        c = np.cos(-np.pi / 2 + (j + (1 if name == "N" else 0)) * dt_)
                        spd = max(abs(own[2] / own[0]) + np.sqrt(G * own[0]),
                                  abs(opp[2] / opp[0]) + np.sqrt(G * opp[0]))
                        a_ = (spd if alpha is None else alpha) / R
                        Uo, Un = own * c, opp * c
                        fstar_n = 0.5 * (Gf(own, c) + Gf(opp, c)) * nrm[1] - 0.5 * a_ * (Un - Uo)
                        jac = dl / 2
                        xi_f, eta_f = xq[k], ys
                    for a in range(n):
                        for b in range(n):
                            out[j, i, :, b, a] -= jac * wq[k] * fstar_n * leg(a, xi_f) * leg(b, eta_f)
    return out.reshape(n_lat, n_lon, 3, n * n)


@pytest.mark.parametrize("order", [1, 2])
def test_residual_equals_literal_weak_form(order):
    n_lon, n_lat = 5, 4
    q, _ = band_limited_state(n_lon, n_lat, order, 3, seed=5)
    m = SphereDG(n_lon, n_lat, order, metric="pointwise")
    got = m.residual(q)
    ref = _weak_form_by_faces(q, n_lon, n_lat, order)
    scale = np.abs(ref).max(axis=(0, 1, 3))
    err = np.abs(got - ref).max(axis=(0, 1, 3))
    assert np.all(err <= 1e-12 * scale), (err, scale)


def test_residual_global_alpha_equals_literal_weak_form():
    """The global-speed Rusanov branch at r = 2 against the same literal
    per-face quadrature with the fixed speed put into its flux."""
    n_lon, n_lat, order, alpha = 5, 4, 2, 400.0
    q, _ = band_limited_state(n_lon, n_lat, order, 3, seed=6)
    m = SphereDG(n_lon, n_lat, order, metric="pointwise", alpha_mode="global", alpha=alpha)
    got = m.residual(q)
    ref = _weak_form_by_faces(q, n_lon, n_lat, order, alpha=alpha)
    scale = np.abs(ref).max(axis=(0, 1, 3))
    err = np.abs(got - ref).max(axis=(0, 1, 3))
    assert np.all(err <= 1e-12 * scale), (err, scale)


# ---------------------------------------------------------------- Rusanov
def test_rusanov_consistency_and_antisymmetry():
    """f*(q, q) = f(q); the dissipative part is antisymmetric in the two sides."""
    m = SphereDG(6, 4, 2)
    rng = np.random.default_rng(3)
    q = np.empty((5, 3, 3))
    q[:, 0] = 1e4 + 50 * rng.standard_normal((5, 3))
    q[:, 1:] = 1e4 * 15 * rng.standard_normal((5, 2, 3))
    c = np.cos(0.3 + 0.1 * np.arange(3))[None, None, :]
    np.testing.assert_allclose(m.rusanov_lambda(q, q, c), m._flux_lambda(q), rtol=1e-15)
    np.testing.assert_allclose(m.rusanov_theta(q, q, 0.7), m._flux_theta(q, 0.7), rtol=1e-15)
    q2 = q[::-1].copy()
    for fn, flux in ((lambda a, b: m.rusanov_lambda(a, b, c), m._flux_lambda),
                     (lambda a, b: m.rusanov_theta(a, b, 0.7), lambda x: m._flux_theta(x, 0.7))):
        d1 = fn(q, q2) - 0.5 * (flux(q) + flux(q2))
        d2 = fn(q2, q) - 0.5 * (flux(q) + flux(q2))
        np.testing.assert_allclose(d1, -d2, rtol=1e-13, atol=1e-20)


# ---------------------------------------------------------------- lake at rest
@pytest.mark.parametrize("order,n_lon,n_lat", [(0, 16, 8), (1, 32, 16), (2, 12, 9), (3, 20, 10), (4, 8, 5), (5, 16, 8)])
def test_lake_at_rest_balanced(order, n_lon, n_lat):
    """Constant depth and zero velocity: the balanced reading gives a zero
    right-hand side to roundoff.  The scale is that of the cancelling terms,
    the pressure's divergence alone: M^-1 (vol - surf) of g h^2/2."""
    m = SphereDG(n_lon, n_lat, order)
    q = lake_at_rest_state(n_lon, n_lat, order)
    d = m.rhs(q)
    scale = (2.0 / min(m.dlam, m.dth)) * 0.5 * G * 1e8 / R * order ** 2 + 0.5 * G * 1e8 / R
    assert np.abs(d).max() <= 1e-13 * scale * (order + 1) ** 2, np.abs(d).max() / scale


@pytest.mark.parametrize("order", [1, 2, 3])
def test_lake_at_rest_pointwise_defect(order):
    """Pointwise reading: h and hu residuals vanish; the hv residual is the
    Gauss-Legendre defect of the discrete integration by parts of the
    pressure-metric term, which is derived here from the continuous system:
    (dlam/2) (g H^2 / 2R) sqrt(2) delta_a0 [beta_b - (dth/2) sum_s w_s sin_s P~_b(eta_s)],
    beta_b = sum_s w_s cos_s P~'_b(eta_s) - (c_t P~_b(1) - c_b P~_b(-1))."""
    n_lon, n_lat = 10, 6
    H = 1e4
    m = SphereDG(n_lon, n_lat, order, metric="pointwise")
    res = m.residual(lake_at_rest_state(n_lon, n_lat, order, H))
    n = order + 1
    x, w = npleg.leggauss(n)
    scale = 0.5 * G * H * H / R * max(m.dlam, m.dth)    # size of the cancelling terms
    assert np.abs(res[..., 0, :]).max() == 0.0
    assert np.abs(res[..., 1, :]).max() <= 1e-12 * scale
    for j in range(n_lat):
        tb = -np.pi / 2 + j * m.dth
        tt = tb + m.dth
        th = tb + (1 + x) * m.dth / 2
        cb = 0.0 if j == 0 else np.cos(tb)
        ct = 0.0 if j == n_lat - 1 else np.cos(tt)
        for b in range(n):
            c = np.zeros(b + 1); c[b] = np.sqrt((2 * b + 1) / 2)
            beta = np.sum(w * np.cos(th) * npleg.legval(x, npleg.legder(c))) - (
                ct * npleg.legval(1.0, c) - cb * npleg.legval(-1.0, c))
            src = 0.5 * m.dth * np.sum(w * np.sin(th) * npleg.legval(x, c))
            expect = 0.5 * m.dlam * (G * H * H / (2 * R)) * np.sqrt(2) * (beta - src)
            got = res[j, :, 2, b * n]                       # a = 0
            np.testing.assert_allclose(got, expect, rtol=1e-9, atol=1e-13 * scale)
            for a in range(1, n):
                assert np.abs(res[j, :, 2, b * n + a]).max() <= 1e-12 * scale


# ---------------------------------------------------------------- conservation
@pytest.mark.parametrize("order", [0, 1, 3])
def test_mass_conservation_rhs(order):
    """d/dt of the total h-mass is a telescoping sum of edge fluxes plus zero
    pole fluxes: it vanishes to roundoff."""
    m = SphereDG(16, 8, order)
    q, _ = band_limited_state(16, 8, order, 6, seed=7)
    res = m.residual(q)
    tot = res[..., 0, 0].sum()
    assert abs(tot) <= 1e-14 * np.abs(res[..., 0, 0]).sum()


def test_mass_conservation_rk3_c1():
    """32 x 16, r = 1, 100 SSP-RK3 steps at CFL 0.1: relative h-mass drift at roundoff."""
    m = SphereDG(32, 16, 1)
    q, info = band_limited_state(32, 16, 1, 6, seed=1)
    dt = m.cfl_time_step(info.cmax, 0.1)
    m0 = m.mass(q)[0]
    for _ in range(100):
        q = m.ssp_rk3_step(q, dt)
    assert abs(m.mass(q)[0] - m0) <= 1e-13 * abs(m0)
    assert np.all(np.isfinite(q))


# ---------------------------------------------------------------- symmetries
def test_longitude_shift_equivariance():
    m = SphereDG(12, 6, 2)
    q, _ = band_limited_state(12, 6, 2, 5, seed=9)
    d = m.grid(m.rhs(q))
    qs = np.roll(m.grid(q), 5, axis=1).reshape(q.shape)
    ds = m.grid(m.rhs(qs))
    np.testing.assert_allclose(ds, np.roll(d, 5, axis=1), rtol=0, atol=1e-11 * np.abs(d).max())


def _mirror(mesh, q):
    n = mesh.n
    g = mesh.grid(q)[::-1].copy()
    b = np.arange(mesh.N) // n
    g *= ((-1.0) ** b)[None, None, None, :]
    g[:, :, 2] *= -1.0
    return g.reshape(q.shape)


@pytest.mark.parametrize("metric", ["balanced", "pointwise"])
def test_equator_mirror_equivariance(metric):
    """theta -> -theta: rows reversed, odd latitude degrees change sign and
    hv changes sign; the right-hand side maps the same way."""
    m = SphereDG(10, 7, 3, metric=metric)
    q, _ = band_limited_state(10, 7, 3, 5, seed=13)
    d = m.rhs(q)
    d2 = m.rhs(_mirror(m, q))
    np.testing.assert_allclose(d2, _mirror(m, d), rtol=0, atol=1e-11 * np.abs(d).max())


# ---------------------------------------------------------------- consistency on smooth fields
H0 = 1e4


def _fields(lam, th):
    h = H0 + 100 * np.cos(th) ** 2 * np.sin(lam) + 50 * np.sin(th) * np.cos(th)
    u = 20 * np.cos(th) + 5 * np.sin(2 * lam) * np.cos(th) ** 2
    v = 8 * np.cos(lam) * np.cos(th) ** 2 * np.sin(th)
    return h, u, v


def _q_exact(lam, th):
    h, u, v = _fields(lam, th)
    return np.array([h, h * u, h * v])


def _dUdt(lam, th):
    """-dF/dlam - dG/dtheta + S of the smooth fields, the derivatives by the
    complex-step method (exact to roundoff for analytic functions)."""
    eps = 1e-30

    def FG(l, t):
        h, u, v = _fields(l, t)
        p = 0.5 * G * h * h
        return (np.array([h * u, h * u * u + p, h * u * v]) / R,
                np.cos(t) * np.array([h * v, h * u * v, h * v * v + p]) / R)

    dF = FG(lam + 1j * eps, th + 0j)[0].imag / eps
    dG = FG(lam + 0j, th + 1j * eps)[1].imag / eps
    h, u, v = _fields(lam, th)
    p = 0.5 * G * h * h
    cor = 2 * OM * np.sin(th) * np.cos(th) + u * np.sin(th) / R
    S = np.array([0 * h, cor * h * v, -p * np.sin(th) / R - cor * h * u])
    return -dF - dG + S


@pytest.mark.parametrize("order", [1, 2, 3])
def test_operator_consistency_converges(order):
    """On the projection of a smooth state the DG operator approaches the
    projection of the exact time derivative, with order about r in the
    maximum modal norm.  A wrong or missing term leaves an O(1) error."""
    errs = []
    for n_lon, n_lat in [(16, 8), (32, 16), (64, 32)]:
        m = SphereDG(n_lon, n_lat, order)
        d = m.rhs(m.project(_q_exact))
        ex = m.weak_forcing(_dUdt)
        errs.append(np.abs(d - ex).max(axis=(0, 2)) / np.abs(ex).max(axis=(0, 2)))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert np.all(errs[-1] < [0.05, 0.05, 0.02][order - 1]), errs
    assert np.all(rates[-1] > order - 0.75), rates


def _h_l2_error(m, q, ref):
    """Cos-weighted L2 norm of the h error, relative to that of ref (both
    modal; the norm uses the mass matrix, which is exact)."""
    d = m.grid(q - ref)[:, :, 0]
    r = m.grid(ref)[:, :, 0]
    return np.sqrt(np.einsum("jim,jmn,jin->", d, m.M, d) / np.einsum("jim,jmn,jin->", r, m.M, r))


@pytest.mark.parametrize("order", [1, 2])
def test_manufactured_solution_time_integrated_rate(order):
    """Convergence order r + 1 of the whole method in time (the rates of the
    paper's section 4 convergence tables, 2.00 / 3.00 for p = 1, 2): the
    smooth state U* is made steady by the forcing dF/dlam + dG/dtheta - S of
    U*, the oracle runs SSP-RK3 from the projection of U* for one simulated
    hour, and the cos-weighted L2 error of h decays like h^(r+1) between
    16 x 8 and 32 x 16 elements.  The time step is CFL 0.2 against the
    smallest element width (it shrinks like h^2, so the RK3 error is
    negligible); a dropped or wrong term leaves an error that does not
    converge, and a first-order flux or metric mistake lowers the rate."""
    errs = []
    cmax = 20.0 + np.sqrt(G * (H0 + 150.0)) + 10.0
    for n_lat in (4, 8, 16):
        m = SphereDG(2 * n_lat, n_lat, order)
        q0 = m.project(_q_exact)
        m.forcing = -m.weak_forcing(_dUdt)
        dt = m.cfl_time_step(cmax, 0.2)
        steps = int(np.ceil(3600.0 / dt))
        q = q0.copy()
        for _ in range(steps):
            q = m.ssp_rk3_step(q, 3600.0 / steps)
        errs.append(_h_l2_error(m, q, q0))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    print("oracle mms", order, errs, rates)
    assert abs(rates[-1] - (order + 1)) < 0.3, (errs, rates)
    assert rates[0] > order, (errs, rates)


# ---------------------------------------------------------------- time integration
def _tableaux():
    with open(os.path.join(GOLDEN, "butcher_tableaux.json")) as f:
        return json.load(f)


def test_ssp_rk3_equals_printed_tableau():
    """The Shu-Osher form used by both paths equals Table 'Butcher''s third
    tableau applied literally, on the DG system itself."""
    tab = _tableaux()["RK3"]
    m = SphereDG(16, 8, 2)
    q, info = band_limited_state(16, 8, 2, 5, seed=4)
    dt = m.cfl_time_step(info.cmax, 0.2)
    a = ssp_rk3(m.rhs, q, dt)
    b = butcher_step(m.rhs, q, dt, tab["A"], tab["b"])
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * np.abs(q).max())


@pytest.mark.parametrize("name,order", [("RK1", 1), ("RK2", 2), ("RK3", 3), ("RK4", 4)])
def test_printed_tableaux_stability_polynomials(name, order):
    """On y' = lambda y each printed tableau of order p gives the truncated
    exponential sum_{k<=p} z^k/k!, and the Shu-Osher SSP-RK3 gives the
    cubic one."""
    tab = _tableaux()[name]
    for z in (-0.3, 0.5 + 0.2j, -1.7):
        L = lambda y: z * y
        got = butcher_step(L, np.array([1.0 + 0j]), 1.0, tab["A"], tab["b"])[0]
        expect = sum(z ** k / np.prod(range(1, k + 1)) for k in range(order + 1))
        assert abs(got - expect) < 1e-14
        if name == "RK3":
            assert abs(ssp_rk3(L, np.array([1.0 + 0j]), 1.0)[0] - expect) < 1e-14


# ---------------------------------------------------------------- tolerance scale
@pytest.mark.parametrize("order,n_lon,n_lat", [(1, 32, 16), (3, 40, 20)])
def test_rhs_scale_bounds_rhs_and_rounding(order, n_lon, n_lat):
    """The componentwise scale bounds |rhs| (triangle inequality), and a
    one-ulp random change of the input moves rhs by a few eps of it."""
    m = SphereDG(n_lon, n_lat, order)
    q, _ = band_limited_state(n_lon, n_lat, order, 8, seed=21)
    ref = m.rhs(q)
    sc = m.rhs_scale(q)
    assert np.all(np.abs(ref) <= sc * (1 + 1e-12))
    rng = np.random.default_rng(0)
    qp = q * (1 + 1.1e-16 * rng.choice([-1.0, 1.0], size=q.shape))
    assert (np.abs(m.rhs(qp) - ref) / sc).max() < 1e-14
