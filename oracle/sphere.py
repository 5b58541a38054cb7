"""Plain FP64 oracle of the modal DG right-hand side of the shallow-water
equations on the latitude-longitude rectangle, and of its SSP Runge-Kutta loop.

Test infrastructure only (see ``oracle/__init__.py``).  Written from the
paper's statement of the method; every array operation is a dense
per-element matrix product in the form the paper's volume-integral stencil
uses (section 3.2, "DG solver: stencils": ``phi @ u_modal`` to get nodal
values, ``phi_grad.T @ (f * w)`` to integrate), vectorised over elements.

What is followed, by passage:

* Conserved variables, fluxes and source (section 2, the system that follows
  the component-wise equations "sph3"):
  U = (h, hu, hv) cos(theta),  F = (1/R)(hu, hu^2 + g h^2/2, huv),
  G = (cos(theta)/R)(hv, huv, hv^2 + g h^2/2),
  S = (0, (f cos + u sin / R) hv, -g h^2 sin / (2R) - (f cos + u sin / R) hu),
  f = 2 Omega sin(theta).
* Boundary conditions (section 2 after "sph3", and section 4.4): periodic in
  longitude, zero flux through the two pole edges.
* Weak form after integration by parts (section 2, equation "dg_parts"),
  Rusanov flux (equation "rusanov") with the outward normal, modal basis
  (equation "basis_expansion"), semi-discrete ODE M dq/dt = h(q) (equation
  "ode"), and the local mass matrix with cos(theta) absorbed, so that the
  unknowns are h, hu, hv (section 2, the cos-weighted mass matrix).
* SSP-RK3 (Table "Butcher", third tableau), in Shu-Osher form.

Readings taken where the paper is silent (the same readings bind the GPU
path):

* orthonormal Legendre basis P~_a = sqrt((2a+1)/2) P_a; mode m = b*n + a with
  a the longitude degree and b the latitude degree; element e = j*n_lon + i
  with j = 0 the southernmost row and i = 0 starting at longitude 0;
* (r+1) x (r+1) Gauss-Legendre nodes for the volume terms and r+1 per edge;
  nonlinear fluxes are evaluated at those nodes;
* the mass matrix is integrated exactly (to roundoff) with a 32-point rule in
  latitude; it depends only on the latitude row;
* the Rusanov jump acts on the conserved U = q cos(theta), with alpha the
  largest local eigenvalue of dF/dU (resp. dG/dU) over both sides of the
  edge point ("local"), or a fixed speed ("global");
* "balanced" metric: the pressure-metric source uses s~ instead of
  sin(theta), where s~ is the polynomial of degree r in eta that makes the
  discrete integration by parts of the pressure term exact, so that a lake
  at rest has a zero right-hand side.  "pointwise" keeps sin(theta).
"""
import numpy as np

from .basis import gauss_legendre, legendre
from .timestep import ssp_rk3


class SphereDG:
    """Mesh, basis tables and the DG operator on n_lon x n_lat elements."""

    def __init__(self, n_lon, n_lat, order, radius=6.371e6, gravity=9.80616,
                 omega=7.292e-5, metric="balanced", alpha_mode="local",
                 alpha=0.0):
        if metric not in ("balanced", "pointwise"):
            raise ValueError(metric)
        if alpha_mode not in ("local", "global"):
            raise ValueError(alpha_mode)
        self.n_lon, self.n_lat, self.order = int(n_lon), int(n_lat), int(order)
        self.R, self.g, self.omega = float(radius), float(gravity), float(omega)
        self.metric, self.alpha_mode, self.alpha = metric, alpha_mode, float(alpha)
        n = self.order + 1
        self.n, self.N = n, n * n
        self.E = self.n_lon * self.n_lat
        self.dlam = 2.0 * np.pi / self.n_lon
        self.dth = np.pi / self.n_lat

        xi, w = gauss_legendre(n)
        P, dP = legendre(self.order, xi)                     # P[p, a]
        Pe, _ = legendre(self.order, np.array([-1.0, 1.0]))
        Pm, Pp = Pe[0], Pe[1]                                # P~_a(-1), P~_a(+1)
        self.xi, self.w = xi, w

        # node k = s*n + p (p: longitude node, s: latitude node); mode m = b*n + a
        pk, sk = np.tile(np.arange(n), n), np.repeat(np.arange(n), n)
        am, bm = pk, sk
        self.pk, self.sk = pk, sk
        self.V = P[pk][:, am] * P[sk][:, bm]                 # phi_m at node k
        self.DX = dP[pk][:, am] * P[sk][:, bm]               # d phi_m / d xi
        self.DY = P[pk][:, am] * dP[sk][:, bm]               # d phi_m / d eta
        self.Wq = w[pk] * w[sk]
        # traces on the four edges, rows = edge node
        self.EE = Pp[am][None, :] * P[:, bm]                 # xi = +1, node s
        self.EW = Pm[am][None, :] * P[:, bm]                 # xi = -1, node s
        self.EN = P[:, am] * Pp[bm][None, :]                 # eta = +1, node p
        self.ES = P[:, am] * Pm[bm][None, :]                 # eta = -1, node p

        # latitude geometry
        j = np.arange(self.n_lat + 1)
        self.theta_edge = -0.5 * np.pi + j * self.dth
        cos_e = np.cos(self.theta_edge)
        cos_e[0] = 0.0
        cos_e[-1] = 0.0                                      # the poles, exactly
        self.cos_edge = cos_e
        self.theta_node = (self.theta_edge[:-1, None]
                           + (1.0 + xi[None, :]) * 0.5 * self.dth)   # [j, s]
        self.cos_node = np.cos(self.theta_node)
        self.sin_node = np.sin(self.theta_node)

        # cos-weighted mass matrix per latitude row, dense N x N
        nq = max(32, 2 * n + 8)
        eta_q, w_q = gauss_legendre(nq)
        Pq, _ = legendre(self.order, eta_q)
        Vm = (P[:, None, :, None] * Pq[None, :, None, :]).reshape(n * nq, n, n)
        Vm = Vm.transpose(0, 2, 1).reshape(n * nq, self.N)   # column m = b*n + a
        wx = np.repeat(w, nq)
        self.M = np.empty((self.n_lat, self.N, self.N))
        for jj in range(self.n_lat):
            th_q = self.theta_edge[jj] + (1.0 + eta_q) * 0.5 * self.dth
            wt = wx * np.tile(w_q * np.cos(th_q), n)
            self.M[jj] = (self.dlam * self.dth / 4.0) * (Vm.T * wt) @ Vm

        # the latitude factor of the pressure-metric source, per row and node
        if metric == "balanced":
            beta = (np.einsum("s,js,sb->jb", w, self.cos_node, dP)
                    - (cos_e[1:, None] * Pp[None, :] - cos_e[:-1, None] * Pm[None, :]))
            self.stilde = (2.0 / self.dth) * np.einsum("sb,jb->js", P, beta)
        else:
            self.stilde = self.sin_node.copy()
        self.forcing = None

    # ------------------------------------------------------------ helpers
    def grid(self, q):
        """(E, 3, N) -> (n_lat, n_lon, 3, N) view."""
        return np.asarray(q, dtype=np.float64).reshape(self.n_lat, self.n_lon, 3, self.N)

    def _flux_lambda(self, q):
        h, hu, hv = q[..., 0, :], q[..., 1, :], q[..., 2, :]
        return np.stack([hu, hu * hu / h + 0.5 * self.g * h * h, hu * hv / h], axis=-2) / self.R

    def _flux_theta(self, q, c):
        h, hu, hv = q[..., 0, :], q[..., 1, :], q[..., 2, :]
        return c * np.stack([hv, hu * hv / h, hv * hv / h + 0.5 * self.g * h * h], axis=-2) / self.R

    def rusanov_lambda(self, qm, qp, c):
        """Flux through a constant-longitude edge, minus = west side.

        qm, qp: (..., 3, n) traces of (h, hu, hv); c: cos(theta) at the edge
        nodes, broadcastable to (..., 1, n).  Written on U = q cos(theta):
        F^ = (F(U-) + F(U+))/2 - (alpha/2)(U+ - U-), alpha = largest
        eigenvalue of dF/dU = (|u| + sqrt(g h)) / (R cos(theta)).
        """
        Fm, Fp = self._flux_lambda(qm), self._flux_lambda(qp)
        Um, Up = qm * c, qp * c
        if self.alpha_mode == "local":
            sm = np.abs(qm[..., 1, :] / qm[..., 0, :]) + np.sqrt(self.g * qm[..., 0, :])
            sp = np.abs(qp[..., 1, :] / qp[..., 0, :]) + np.sqrt(self.g * qp[..., 0, :])
            speed = np.maximum(sm, sp)[..., None, :]
        else:
            speed = self.alpha
        a = speed / (self.R * c)
        return 0.5 * (Fm + Fp) - 0.5 * a * (Up - Um)

    def rusanov_theta(self, qm, qp, c):
        """Flux through a constant-latitude edge, minus = south side.

        alpha = largest eigenvalue of dG/dU = (|v| + sqrt(g h)) / R.
        """
        Gm, Gp = self._flux_theta(qm, c), self._flux_theta(qp, c)
        Um, Up = qm * c, qp * c
        if self.alpha_mode == "local":
            sm = np.abs(qm[..., 2, :] / qm[..., 0, :]) + np.sqrt(self.g * qm[..., 0, :])
            sp = np.abs(qp[..., 2, :] / qp[..., 0, :]) + np.sqrt(self.g * qp[..., 0, :])
            speed = np.maximum(sm, sp)[..., None, :]
        else:
            speed = self.alpha
        a = speed / self.R
        return 0.5 * (Gm + Gp) - 0.5 * a * (Up - Um)

    # ------------------------------------------------------------ operator
    def residual(self, q):
        """h(q) of the semi-discrete ODE M dq/dt = h(q), shape (n_lat, n_lon, 3, N)."""
        q = self.grid(q)
        R, g = self.R, self.g
        Q = np.einsum("km,jivm->jivk", self.V, q)            # nodal values
        h, hu, hv = Q[:, :, 0], Q[:, :, 1], Q[:, :, 2]
        cosk = self.cos_node[:, self.sk][:, None, :]
        sink = self.sin_node[:, self.sk][:, None, :]
        stk = self.stilde[:, self.sk][:, None, :]
        u, v = hu / h, hv / h
        pres = 0.5 * g * h * h
        F = np.stack([hu, hu * u + pres, hu * v], axis=2) / R
        G = cosk[:, :, None] * np.stack([hv, hu * v, hv * v + pres], axis=2) / R
        cor = 2.0 * self.omega * sink * cosk + u * sink / R
        S = np.stack([np.zeros_like(h), cor * hv, -pres * stk / R - cor * hu], axis=2)
        W = self.Wq
        vol = (0.5 * self.dth * np.einsum("km,jivk->jivm", self.DX, W * F)
               + 0.5 * self.dlam * np.einsum("km,jivk->jivm", self.DY, W * G)
               + 0.25 * self.dlam * self.dth * np.einsum("km,jivk->jivm", self.V, W * S))

        qE = np.einsum("sm,jivm->jivs", self.EE, q)
        qW = np.einsum("sm,jivm->jivs", self.EW, q)
        qN = np.einsum("pm,jivm->jivp", self.EN, q)
        qS = np.einsum("pm,jivm->jivp", self.ES, q)
        # constant-longitude edges: edge i is east of element i (periodic)
        c_lam = self.cos_node[:, None, None, :]
        F_E = self.rusanov_lambda(qE, np.roll(qW, -1, axis=1), c_lam)
        F_W = np.roll(F_E, 1, axis=1)
        # constant-latitude edges: 0 and n_lat are the poles, zero flux
        G_edge = np.zeros((self.n_lat + 1, self.n_lon, 3, self.n))
        if self.n_lat > 1:
            G_edge[1:-1] = self.rusanov_theta(qN[:-1], qS[1:],
                                              self.cos_edge[1:-1, None, None, None])
        G_N, G_S = G_edge[1:], G_edge[:-1]
        w = self.w
        surf = (0.5 * self.dth * (np.einsum("sm,jivs->jivm", self.EE, w * F_E)
                                  - np.einsum("sm,jivs->jivm", self.EW, w * F_W))
                + 0.5 * self.dlam * (np.einsum("pm,jivp->jivm", self.EN, w * G_N)
                                     - np.einsum("pm,jivp->jivm", self.ES, w * G_S)))
        return vol - surf

    def rhs_scale(self, q):
        """Size of the terms that are summed into each entry of rhs(q): the
        same computation with every term replaced by its absolute value
        (nodal fluxes and sources, both Rusanov halves and the dissipation,
        |M^-1|).  Rounding in any evaluation order is a small multiple of
        eps times this, entry by entry, so it is the scale of a
        componentwise comparison of two floating-point evaluations.  It is
        large where terms cancel: near the poles the longitude-flux
        difference is divided by the small cos(theta)-weighted element area.
        """
        q = self.grid(q)
        R, g = self.R, self.g
        Q = np.einsum("km,jivm->jivk", np.abs(self.V), np.abs(q))
        Qs = np.einsum("km,jivm->jivk", self.V, q)
        h, hu, hv = np.abs(Qs[:, :, 0]), np.abs(Qs[:, :, 1]), np.abs(Qs[:, :, 2])
        hmag = Q[:, :, 0]
        cosk = self.cos_node[:, self.sk][:, None, :]
        sink = np.abs(self.sin_node[:, self.sk])[:, None, :]
        stk = np.abs(self.stilde[:, self.sk])[:, None, :]
        u, v = hu / h, hv / h
        pres = 0.5 * g * hmag * hmag
        F = np.stack([Q[:, :, 1], hu * u + pres, hu * v], axis=2) / R
        G = cosk[:, :, None] * np.stack([Q[:, :, 2], hu * v, hv * v + pres], axis=2) / R
        cor = 2.0 * abs(self.omega) * sink * cosk + u * sink / R
        S = np.stack([np.zeros_like(h), cor * hv, pres * stk / R + cor * hu], axis=2)
        W = self.Wq
        vol = (0.5 * self.dth * np.einsum("km,jivk->jivm", np.abs(self.DX), W * F)
               + 0.5 * self.dlam * np.einsum("km,jivk->jivm", np.abs(self.DY), W * G)
               + 0.25 * self.dlam * self.dth * np.einsum("km,jivk->jivm", np.abs(self.V), W * S))
        tr = {k: np.einsum("sm,jivm->jivs", getattr(self, k), q) for k in ("EE", "EW", "EN", "ES")}
        trm = {k: np.einsum("sm,jivm->jivs", np.abs(getattr(self, k)), np.abs(q))
               for k in ("EE", "EW", "EN", "ES")}

        def half(qt, qmag, lam):
            # one side's share of |F^|: half its flux (pressure from the
            # term magnitude of h) plus half the dissipation alpha |q|
            hh = np.abs(qt[..., 0, :])
            mu, mv = np.abs(qt[..., 1, :]), np.abs(qt[..., 2, :])
            p = 0.5 * g * qmag[..., 0, :] ** 2
            speed = (mu if lam else mv) / hh + np.sqrt(g * hh)
            if lam:
                f = np.stack([qmag[..., 1, :], mu * mu / hh + p, mu * mv / hh], axis=-2)
            else:
                f = np.stack([qmag[..., 2, :], mu * mv / hh, mv * mv / hh + p], axis=-2)
            return 0.5 * f + 0.5 * speed[..., None, :] * qmag

        F_E = (half(tr["EE"], trm["EE"], True)
               + half(np.roll(tr["EW"], -1, axis=1), np.roll(trm["EW"], -1, axis=1), True)) / R
        F_W = np.roll(F_E, 1, axis=1)
        G_edge = np.zeros((self.n_lat + 1, self.n_lon, 3, self.n))
        if self.n_lat > 1:
            ce = self.cos_edge[1:-1, None, None, None]
            G_edge[1:-1] = ce * (half(tr["EN"][:-1], trm["EN"][:-1], False)
                                 + half(tr["ES"][1:], trm["ES"][1:], False)) / R
        G_N, G_S = G_edge[1:], G_edge[:-1]
        w = self.w
        surf = (0.5 * self.dth * (np.einsum("sm,jivs->jivm", np.abs(self.EE), w * F_E)
                                  + np.einsum("sm,jivs->jivm", np.abs(self.EW), w * F_W))
                + 0.5 * self.dlam * (np.einsum("pm,jivp->jivm", np.abs(self.EN), w * G_N)
                                     + np.einsum("pm,jivp->jivm", np.abs(self.ES), w * G_S)))
        tot = vol + surf
        out = np.empty_like(tot)
        for j in range(self.n_lat):
            Mi = np.abs(np.linalg.inv(self.M[j]))
            out[j] = np.einsum("mn,ivn->ivm", Mi, tot[j])
        return out.reshape(self.E, 3, self.N)

    def rhs(self, q):
        """dq/dt = M^-1 h(q) (+ the optional modal forcing), shape (E, 3, N)."""
        res = self.residual(q)
        out = np.empty_like(res)
        for j in range(self.n_lat):
            b = res[j].reshape(-1, self.N).T
            out[j] = np.linalg.solve(self.M[j], b).T.reshape(self.n_lon, 3, self.N)
        out = out.reshape(self.E, 3, self.N)
        if self.forcing is not None:
            out = out + self.forcing
        return out

    def mass(self, q):
        """R^2 * integral of (h, hu, hv) cos(theta) dlambda dtheta.

        phi_00 = 1/2, so the integral over an element is 2 (M q)_00.
        """
        q = self.grid(q)
        Mq = np.einsum("jmn,jivn->jivm", self.M, q)
        return self.R ** 2 * 2.0 * Mq[..., 0].sum(axis=(0, 1))

    # ------------------------------------------------------------ time
    def ssp_rk3_step(self, q, dt):
        """One SSP-RK3 step (Shu-Osher form of the third tableau of Table
        "Butcher")."""
        return ssp_rk3(self.rhs, np.asarray(q, dtype=np.float64), dt)

    def cfl_time_step(self, cmax, cfl):
        """dt = cfl * H / (max(r,1) c): the DG Courant number p c dt / H of
        section 2.  H is the smallest element width, read as the longitude
        width at the latitude quadrature node nearest a pole (the width at
        the centre of the pole row gives unstable runs at cfl 0.1 for r >= 3)."""
        H = self.R * min(self.dth, self.dlam * self.cos_node.min())
        return cfl * H / (max(self.order, 1) * cmax)

    # ------------------------------------------------------------ projection
    def project(self, fun, extra=9):
        """Cos-weighted L2 projection q = M^-1 int f phi cos(theta).

        fun(lam, th) -> array (3, ...) of (h, hu, hv) at the given points.
        Uses an (r+extra)-point Gauss-Legendre rule per direction.
        """
        nq = self.n + extra
        xq, wq = gauss_legendre(nq)
        Pq, _ = legendre(self.order, xq)                      # [q, a]
        lam = (np.arange(self.n_lon)[:, None] * self.dlam
               + (1.0 + xq[None, :]) * 0.5 * self.dlam)       # [i, p]
        th = (self.theta_edge[:-1, None] + (1.0 + xq[None, :]) * 0.5 * self.dth)  # [j, s]
        LAM, TH = np.meshgrid(lam.ravel(), th.ravel())
        vals = np.asarray(fun(LAM, TH), dtype=np.float64)
        vals = vals.reshape(3, self.n_lat, nq, self.n_lon, nq)   # [v, j, s, i, p]
        wc = (wq[None, :] * np.cos(th))                        # [j, s]
        b = np.einsum("vjsip,js,p,pa,sb->jivba", vals, wc, wq, Pq, Pq)
        b = 0.25 * self.dlam * self.dth * b.reshape(self.n_lat, self.n_lon, 3, self.N)
        out = np.empty_like(b)
        for j in range(self.n_lat):
            out[j] = np.linalg.solve(self.M[j], b[j].reshape(-1, self.N).T).T.reshape(
                self.n_lon, 3, self.N)
        return out.reshape(self.E, 3, self.N)

    def weak_forcing(self, fun, extra=9):
        """M^-1 int s phi dlambda dtheta for a given source density s(lam, th)
        (3 components, no cos weight): the modal form of a forcing term
        added to the right-hand side of the conservative system."""
        return self.project(lambda lam, th: np.asarray(fun(lam, th)) / np.cos(th), extra)


def project_order(q_src, src, dst, extra=9):
    """Cos-weighted L2 projection of a modal state on mesh `src` onto the
    basis of `dst` (same mesh, another order): q_dst = M_dst^-1 int q_src
    phi_dst cos(theta), by Gauss-Legendre quadrature exact for the product
    of the two polynomial degrees times cos over one latitude row."""
    assert (src.n_lon, src.n_lat) == (dst.n_lon, dst.n_lat)
    nq = src.n + dst.n + extra
    xq, wq = gauss_legendre(nq)
    Ps, _ = legendre(src.order, xq)                     # [q, a]
    Pd, _ = legendre(dst.order, xq)
    # phi at the 2-D points: [point (s, p), mode (b, a)]
    phis = np.einsum("pa,sb->spba", Ps, Ps).reshape(nq * nq, src.N)
    phid = np.einsum("pa,sb->spba", Pd, Pd).reshape(nq * nq, dst.N)
    q = src.grid(q_src)
    out = np.empty((dst.n_lat, dst.n_lon, 3, dst.N))
    for j in range(dst.n_lat):
        th = dst.theta_edge[j] + (1.0 + xq) * 0.5 * dst.dth
        wt = (np.outer(wq * np.cos(th), wq)).reshape(-1)   # [s, p]
        C = 0.25 * dst.dlam * dst.dth * (phid.T * wt) @ phis   # [m_dst, m_src]
        b = np.einsum("mn,ivn->ivm", C, q[j])
        out[j] = np.linalg.solve(dst.M[j], b.reshape(-1, dst.N).T).T.reshape(dst.n_lon, 3, dst.N)
    return out.reshape(dst.E, 3, dst.N)
