"""Plain FP64 oracle of the modal DG right-hand side of the planar
shallow-water equations on a doubly periodic rectangle (the f-plane).

Test infrastructure only (see ``oracle/__init__.py``).  Section 4.2 runs the
paper's DG scheme on the planar system: conserved U = (h, hu, hv),
F = (hu, hu^2/h + g h^2/2, hu hv/h), G = (hv, hu hv/h, hv^2/h + g h^2/2),
Coriolis source S = (0, f hv, -f hu) with constant f, periodic boundaries.
The discretisation is that of section 2 without the spherical metric: the
weak form of equation "dg_parts" on x = x_i + (1 + xi) dx/2,
y = y_j + (1 + eta) dy/2, the Rusanov flux of equation "rusanov" with the
local largest eigenvalue |u_n| + sqrt(g h), the modal orthonormal Legendre
basis of equation "basis_expansion" and the ODE M dq/dt = h(q) of equation
"ode" with M = int phi_i phi_j dx dy.

Dense per-element matrices, as in the sphere oracle: nodal values by
``V @ q``, integrals by ``D.T @ (w * F)``; edges handled with explicit
``np.roll`` in both directions.  Same readings as on the sphere for the
basis, the ordering (mode m = b n + a, a along x; element e = j nx + i, i
along x) and the quadrature ((r+1) Gauss-Legendre points per direction for
volume and edges).
"""
import numpy as np

from .basis import gauss_legendre, legendre


class PlaneDG:
    """nx x ny elements on [0, lx] x [0, ly], periodic in x and y."""

    def __init__(self, nx, ny, order, lx, ly, gravity=9.81, f=1.0e-4,
                 alpha_mode="local", alpha=0.0):
        if alpha_mode not in ("local", "global"):
            raise ValueError(alpha_mode)
        self.nx, self.ny, self.order = int(nx), int(ny), int(order)
        self.lx, self.ly = float(lx), float(ly)
        self.g, self.f = float(gravity), float(f)
        self.alpha_mode, self.alpha = alpha_mode, float(alpha)
        n = self.order + 1
        self.n, self.N = n, n * n
        self.E = self.nx * self.ny
        self.dx, self.dy = self.lx / self.nx, self.ly / self.ny

        xi, w = gauss_legendre(n)
        P, dP = legendre(self.order, xi)
        Pe, _ = legendre(self.order, np.array([-1.0, 1.0]))
        Pm, Pp = Pe[0], Pe[1]
        self.xi, self.w = xi, w
        # node k = s n + p (p along x), mode m = b n + a (a along x)
        pk, sk = np.tile(np.arange(n), n), np.repeat(np.arange(n), n)
        self.pk, self.sk = pk, sk
        self.V = P[pk][:, pk] * P[sk][:, sk]
        self.DX = dP[pk][:, pk] * P[sk][:, sk]
        self.DY = P[pk][:, pk] * dP[sk][:, sk]
        self.Wq = w[pk] * w[sk]
        self.EE = Pp[pk][None, :] * P[:, sk]        # x edge at xi = +1, rows: node s
        self.EW = Pm[pk][None, :] * P[:, sk]
        self.EN = P[:, pk] * Pp[sk][None, :]        # y edge at eta = +1, rows: node p
        self.ES = P[:, pk] * Pm[sk][None, :]
        # mass matrix int phi_i phi_j dx dy by the tensor rule (exact: degree 2r)
        self.M = 0.25 * self.dx * self.dy * (self.V.T * self.Wq) @ self.V
        self.forcing = None

    def grid(self, q):
        return np.asarray(q, dtype=np.float64).reshape(self.ny, self.nx, 3, self.N)

    def _speed(self, q, comp):
        return np.abs(q[..., comp, :] / q[..., 0, :]) + np.sqrt(self.g * q[..., 0, :])

    def flux_x(self, q):
        h, hu, hv = q[..., 0, :], q[..., 1, :], q[..., 2, :]
        return np.stack([hu, hu * hu / h + 0.5 * self.g * h * h, hu * hv / h], axis=-2)

    def flux_y(self, q):
        h, hu, hv = q[..., 0, :], q[..., 1, :], q[..., 2, :]
        return np.stack([hv, hu * hv / h, hv * hv / h + 0.5 * self.g * h * h], axis=-2)

    def rusanov(self, qm, qp, comp):
        """Numerical flux through an edge normal to x (comp = 1) or y
        (comp = 2), minus side west / south: the mean of the two physical
        fluxes minus alpha/2 times the jump, alpha the larger local
        eigenvalue |u_n| + sqrt(g h) of the two sides (or a fixed speed)."""
        fl = self.flux_x if comp == 1 else self.flux_y
        if self.alpha_mode == "local":
            a = np.maximum(self._speed(qm, comp), self._speed(qp, comp))[..., None, :]
        else:
            a = self.alpha
        return 0.5 * (fl(qm) + fl(qp)) - 0.5 * a * (qp - qm)

    def residual(self, q):
        """h(q) of M dq/dt = h(q), shape (ny, nx, 3, N)."""
        q = self.grid(q)
        Q = np.einsum("km,jivm->jivk", self.V, q)
        h, hu, hv = Q[:, :, 0], Q[:, :, 1], Q[:, :, 2]
        F = self.flux_x(Q)
        G = self.flux_y(Q)
        S = np.stack([np.zeros_like(h), self.f * hv, -self.f * hu], axis=2)
        W = self.Wq
        vol = (0.5 * self.dy * np.einsum("km,jivk->jivm", self.DX, W * F)
               + 0.5 * self.dx * np.einsum("km,jivk->jivm", self.DY, W * G)
               + 0.25 * self.dx * self.dy * np.einsum("km,jivk->jivm", self.V, W * S))
        qE = np.einsum("sm,jivm->jivs", self.EE, q)
        qW = np.einsum("sm,jivm->jivs", self.EW, q)
        qN = np.einsum("pm,jivm->jivp", self.EN, q)
        qS = np.einsum("pm,jivm->jivp", self.ES, q)
        # edge east of element i sees element i+1's west trace (periodic in x)
        FE = self.rusanov(qE, np.roll(qW, -1, axis=1), 1)
        FW = np.roll(FE, 1, axis=1)
        # edge north of row j sees row j+1's south trace (periodic in y)
        GN = self.rusanov(qN, np.roll(qS, -1, axis=0), 2)
        GS = np.roll(GN, 1, axis=0)
        w = self.w
        surf = (0.5 * self.dy * (np.einsum("sm,jivs->jivm", self.EE, w * FE)
                                 - np.einsum("sm,jivs->jivm", self.EW, w * FW))
                + 0.5 * self.dx * (np.einsum("pm,jivp->jivm", self.EN, w * GN)
                                   - np.einsum("pm,jivp->jivm", self.ES, w * GS)))
        return vol - surf

    def rhs(self, q):
        """dq/dt = M^-1 h(q) (+ optional modal forcing), shape (E, 3, N)."""
        res = self.residual(q).reshape(-1, self.N)
        out = np.linalg.solve(self.M, res.T).T.reshape(self.E, 3, self.N)
        if self.forcing is not None:
            out = out + self.forcing
        return out

    def rhs_scale(self, q):
        """Componentwise scale of rhs(q): every term replaced by its absolute
        value (the rounding of any evaluation order is a small multiple of
        eps times this, entry by entry)."""
        q = self.grid(q)
        g = self.g
        Qm = np.einsum("km,jivm->jivk", np.abs(self.V), np.abs(q))
        Qs = np.einsum("km,jivm->jivk", self.V, q)
        h, hu, hv = np.abs(Qs[:, :, 0]), np.abs(Qs[:, :, 1]), np.abs(Qs[:, :, 2])
        pres = 0.5 * g * Qm[:, :, 0] ** 2
        F = np.stack([Qm[:, :, 1], hu * hu / h + pres, hu * hv / h], axis=2)
        G = np.stack([Qm[:, :, 2], hu * hv / h, hv * hv / h + pres], axis=2)
        S = np.stack([np.zeros_like(h), abs(self.f) * hv, abs(self.f) * hu], axis=2)
        W = self.Wq
        vol = (0.5 * self.dy * np.einsum("km,jivk->jivm", np.abs(self.DX), W * F)
               + 0.5 * self.dx * np.einsum("km,jivk->jivm", np.abs(self.DY), W * G)
               + 0.25 * self.dx * self.dy * np.einsum("km,jivk->jivm", np.abs(self.V), W * S))
        tr = {k: np.einsum("sm,jivm->jivs", getattr(self, k), q) for k in ("EE", "EW", "EN", "ES")}
        trm = {k: np.einsum("sm,jivm->jivs", np.abs(getattr(self, k)), np.abs(q))
               for k in ("EE", "EW", "EN", "ES")}

        def half(qt, qmag, comp):
            hh = np.abs(qt[..., 0, :])
            mu, mv = np.abs(qt[..., 1, :]), np.abs(qt[..., 2, :])
            p = 0.5 * g * qmag[..., 0, :] ** 2
            speed = (mu if comp == 1 else mv) / hh + np.sqrt(g * hh)
            if comp == 1:
                fl = np.stack([qmag[..., 1, :], mu * mu / hh + p, mu * mv / hh], axis=-2)
            else:
                fl = np.stack([qmag[..., 2, :], mu * mv / hh, mv * mv / hh + p], axis=-2)
            return 0.5 * fl + 0.5 * speed[..., None, :] * qmag

        FE = half(tr["EE"], trm["EE"], 1) + half(np.roll(tr["EW"], -1, 1), np.roll(trm["EW"], -1, 1), 1)
        FW = np.roll(FE, 1, axis=1)
        GN = half(tr["EN"], trm["EN"], 2) + half(np.roll(tr["ES"], -1, 0), np.roll(trm["ES"], -1, 0), 2)
        GS = np.roll(GN, 1, axis=0)
        w = self.w
        surf = (0.5 * self.dy * (np.einsum("sm,jivs->jivm", np.abs(self.EE), w * FE)
                                 + np.einsum("sm,jivs->jivm", np.abs(self.EW), w * FW))
                + 0.5 * self.dx * (np.einsum("pm,jivp->jivm", np.abs(self.EN), w * GN)
                                   + np.einsum("pm,jivp->jivm", np.abs(self.ES), w * GS)))
        Mi = np.abs(np.linalg.inv(self.M))
        return np.einsum("mn,jivn->jivm", Mi, vol + surf).reshape(self.E, 3, self.N)

    def mass(self, q):
        """Integral of (h, hu, hv) over the rectangle: 2 (M q)_00 per element
        (phi_00 = 1/2)."""
        q = self.grid(q)
        Mq = np.einsum("mn,jivn->jivm", self.M, q)
        return 2.0 * Mq[..., 0].sum(axis=(0, 1))

    def cfl_time_step(self, cmax, cfl):
        """dt = cfl min(dx, dy) / (max(r, 1) c_max) (section 2's Courant number)."""
        return cfl * min(self.dx, self.dy) / (max(self.order, 1) * cmax)

    def project(self, fun, extra=9):
        """L2 projection of fun(x, y) -> (3, ...) values onto the basis, by an
        (r + 1 + extra)-point Gauss-Legendre rule per direction."""
        nq = self.n + extra
        xq, wq = gauss_legendre(nq)
        Pq, _ = legendre(self.order, xq)
        x = (np.arange(self.nx)[:, None] + 0.5 * (1.0 + xq[None, :])) * self.dx     # [i, p]
        y = (np.arange(self.ny)[:, None] + 0.5 * (1.0 + xq[None, :])) * self.dy     # [j, s]
        X, Y = np.meshgrid(x.ravel(), y.ravel())
        vals = np.asarray(fun(X, Y), dtype=np.float64).reshape(3, self.ny, nq, self.nx, nq)
        b = np.einsum("vjsip,s,p,pa,sb->jivba", vals, wq, wq, Pq, Pq)
        b = 0.25 * self.dx * self.dy * b.reshape(-1, self.N)
        return np.linalg.solve(self.M, b.T).T.reshape(self.E, 3, self.N)

