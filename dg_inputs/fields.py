"""Random band-limited shallow-water states on the latitude-longitude mesh.

Recipe (the same for every workload):

* Height: h = h0 + dh, dh a sum of real spherical harmonics of degree
  1 <= l <= L with independent N(0, 1) coefficients (flat spectrum), scaled
  so that max |dh| over the sampling points equals ``dh_amp``.
* Velocity from a random streamfunction psi (same spectrum, independent
  coefficients): u = -(1/R) d psi / d theta, v = (1/(R cos theta)) d psi /
  d lambda, a smooth non-divergent field on the sphere, scaled so that the
  largest speed over the sampling points equals ``vmax``.
* (h, hu, hv) are sampled at a tensor grid of Gauss-Legendre points inside
  each element and turned into coefficients of the orthonormal Legendre
  tensor basis by the unweighted L2 projection on the reference square
  (numpy's Legendre routines).  This is input synthesis only: any smooth
  state is a valid input to the operator.

The planar Gaussian bump (``gaussian_bump_plane``) follows the same
projection on the periodic rectangle.

Layout: q[e][v][m], e = j*n_lon + i (j = 0 southernmost row, i = 0 at
longitude 0), v in (h, hu, hv), m = b*n + a (a: longitude degree,
b: latitude degree).
"""
from dataclasses import dataclass

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import sph_legendre_p


@dataclass
class StateInfo:
    cmax: float        # largest |v| + sqrt(g h) over the sampling points
    hmin: float
    hmax: float
    vmax: float


def _orthonormal_vander(order, x):
    V = npleg.legvander(x, order)
    return V * np.sqrt((2.0 * np.arange(order + 1) + 1.0) / 2.0)


def _harmonic_tables(L, colat):
    """Normalised associated Legendre values and colatitude derivatives,
    [l, m, point] for 0 <= m <= l <= L."""
    P = np.zeros((L + 1, L + 1, colat.size))
    dP = np.zeros_like(P)
    for l in range(1, L + 1):
        for m in range(0, l + 1):
            val = sph_legendre_p(l, m, colat, diff_n=1)
            P[l, m], dP[l, m] = val[0], val[1]
    return P, dP


def band_limited_state(n_lon, n_lat, order, L, seed, h0=1.0e4, dh_amp=100.0,
                       vmax=20.0, radius=6.371e6, gravity=9.80616, nq=None):
    """Seeded band-limited (h, hu, hv) state as float64 q[E][3][N]."""
    n = order + 1
    nq = nq or (n + 3)
    rng = np.random.default_rng(seed)
    a_h = rng.standard_normal((2, L + 1, L + 1))
    a_p = rng.standard_normal((2, L + 1, L + 1))
    ll, mm = np.meshgrid(np.arange(L + 1), np.arange(L + 1), indexing="ij")
    mask = (mm <= ll) & (ll >= 1)
    for a in (a_h, a_p):
        a[:, ~mask] = 0.0
        a[1, :, 0] = 0.0                      # sin(0 lambda) carries nothing

    x, w = npleg.leggauss(nq)
    dlam, dth = 2.0 * np.pi / n_lon, np.pi / n_lat
    lam = (np.arange(n_lon)[:, None] * dlam + (1.0 + x[None, :]) * 0.5 * dlam).ravel()
    th = (-0.5 * np.pi + np.arange(n_lat)[:, None] * dth + (1.0 + x[None, :]) * 0.5 * dth).ravel()
    colat = 0.5 * np.pi - th

    P, dP = _harmonic_tables(L, colat)        # [l, m, lat]
    mvec = np.arange(L + 1)
    cosm = np.cos(np.outer(mvec, lam))        # [m, lon]
    sinm = np.sin(np.outer(mvec, lam))

    def synth(coef, table):
        Ac = np.einsum("lm,lmt->tm", coef[0], table)
        As = np.einsum("lm,lmt->tm", coef[1], table)
        return Ac, As

    Ac, As = synth(a_h, P)
    dh = Ac @ cosm + As @ sinm                                   # [lat, lon]
    # psi and its derivatives
    Pc, Ps = synth(a_p, dP)
    dpsi_dcolat = Pc @ cosm + Ps @ sinm
    Qc, Qs = synth(a_p, P)
    dpsi_dlam = (Qc * mvec) @ (-sinm) + (Qs * mvec) @ cosm
    u = dpsi_dcolat / radius                   # -(1/R) d/dtheta = (1/R) d/dcolat
    v = dpsi_dlam / (radius * np.cos(th))[:, None]

    dh *= dh_amp / np.abs(dh).max()
    speed = np.sqrt(u * u + v * v)
    s = vmax / speed.max()
    u *= s
    v *= s
    h = h0 + dh
    fields = np.stack([h, h * u, h * v])                         # [v, lat, lon]

    Vx = _orthonormal_vander(order, x)                            # [point, a]
    f = fields.reshape(3, n_lat, nq, n_lon, nq)                   # [v, j, s, i, p]
    q = np.einsum("vjsip,s,p,pa,sb->jivba", f, w, w, Vx, Vx)
    q = np.ascontiguousarray(q.reshape(n_lat * n_lon, 3, n * n))
    info = StateInfo(cmax=float((np.sqrt(u * u + v * v) + np.sqrt(gravity * h)).max()),
                     hmin=float(h.min()), hmax=float(h.max()),
                     vmax=float(np.sqrt(u * u + v * v).max()))
    return q, info


def lake_at_rest_state(n_lon, n_lat, order, h0=1.0e4):
    """Constant depth h0, zero velocity: only the (h, mode 0) coefficient,
    2 h0 since the first basis function is 1/2."""
    n = order + 1
    q = np.zeros((n_lon * n_lat, 3, n * n))
    q[:, 0, 0] = 2.0 * h0
    return q


def ensemble_members(n_members=64, seed=4, orders=(2, 3, 4), n_lats=(45, 90, 135, 180)):
    """Uneven ensemble: order r and latitude count drawn uniformly by seed,
    n_lon = 2 n_lat.  Returns a list of dicts (n_lon, n_lat, order, seed),
    member k's fields seeded with seed * 1000 + k."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_members):
        r = int(rng.choice(orders))
        nt = int(rng.choice(n_lats))
        out.append({"n_lon": 2 * nt, "n_lat": nt, "order": r, "seed": seed * 1000 + k})
    return out


def gaussian_bump_plane(nx, ny, order, lx, ly, h0=1000.0, h1=5.0, sigma_frac=1.0 / 20.0, nq=None):
    """Fluid at rest on the periodic rectangle [0, lx] x [0, ly] with a
    Gaussian bump h0 + h1 exp(-r^2 / (2 sigma^2)) at the centre, sigma =
    sigma_frac lx: the geostrophic-adjustment start of section 4.2
    (h0 = 1000 m, h1 = 5 m, sigma = L/20).  Projected unweighted onto the
    orthonormal basis like the sphere states; layout q[e][v][m] with
    e = j nx + i (i along x)."""
    n = order + 1
    nq = nq or (n + 6)
    x, w = npleg.leggauss(nq)
    dx, dy = lx / nx, ly / ny
    xs = (np.arange(nx)[:, None] + 0.5 * (1.0 + x[None, :])) * dx      # [i, p]
    ys = (np.arange(ny)[:, None] + 0.5 * (1.0 + x[None, :])) * dy      # [j, s]
    sig = sigma_frac * lx
    r2 = (xs.ravel()[None, :] - 0.5 * lx) ** 2 + (ys.ravel()[:, None] - 0.5 * ly) ** 2
    h = (h0 + h1 * np.exp(-r2 / (2.0 * sig * sig))).reshape(ny, nq, nx, nq)   # [j, s, i, p]
    Vx = _orthonormal_vander(order, x)
    qh = np.einsum("jsip,s,p,pa,sb->jiba", h, w, w, Vx, Vx).reshape(ny * nx, n * n)
    q = np.zeros((ny * nx, 3, n * n))
    q[:, 0] = qh
    return q


def random_plane_state(nx, ny, order, lx, ly, seed, h0=1000.0, dh=5.0, vel=2.0, kmax=3, nq=None):
    """Seeded smooth state on the periodic rectangle: h = h0 + a random sum of
    Fourier modes |kx|, |ky| <= kmax scaled to max |dh| = dh, and (u, v) a
    mean flow plus random modes scaled to max speed vel; projected like
    ``gaussian_bump_plane``."""
    rng = np.random.default_rng(seed)
    n = order + 1
    nq = nq or (n + 6)
    x, w = npleg.leggauss(nq)
    dx, dy = lx / nx, ly / ny
    X = ((np.arange(nx)[:, None] + 0.5 * (1.0 + x[None, :])) * dx).ravel()
    Y = ((np.arange(ny)[:, None] + 0.5 * (1.0 + x[None, :])) * dy).ravel()
    XX, YY = np.meshgrid(X, Y)                     # [y, x]

    def field():
        out = np.zeros_like(XX)
        for kx in range(-kmax, kmax + 1):
            for ky in range(0, kmax + 1):
                if kx == 0 and ky == 0:
                    continue
                a, ph = rng.standard_normal(), rng.uniform(0, 2 * np.pi)
                out += a * np.cos(2 * np.pi * (kx * XX / lx + ky * YY / ly) + ph)
        return out / np.abs(out).max()

    h = h0 + dh * field()
    u = 0.5 + field()
    v = -0.3 + field()
    s_ = vel / np.sqrt(u * u + v * v).max()
    u, v = u * s_, v * s_
    f = np.stack([h, h * u, h * v]).reshape(3, ny, nq, nx, nq)
    Vx = _orthonormal_vander(order, x)
    q = np.einsum("vjsip,s,p,pa,sb->jivba", f, w, w, Vx, Vx)
    return np.ascontiguousarray(q.reshape(ny * nx, 3, n * n))


def sine_square(k, order):
    """u0 = sin(2 pi x) sin(2 pi y) on the unit square with k x k elements
    (section 4.1's initial condition), projected unweighted onto the
    orthonormal basis; layout u[e][m], e = j k + i, m = b (r+1) + a."""
    n = order + 1
    x, w = npleg.leggauss(n + 6)
    xs = (np.arange(k)[:, None] + 0.5 * (1.0 + x[None, :])) / k       # [i, p]
    Vx = _orthonormal_vander(order, x)
    s = np.sin(2 * np.pi * xs)                                          # [i, p]
    c = np.einsum("ip,p,pa->ia", s, w, Vx)                              # 1-D coefficients
    return np.ascontiguousarray(np.einsum("jb,ia->jiba", c, c).reshape(k * k, n * n))

