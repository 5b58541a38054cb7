"""Plain FP64 oracle of the modal DG discretisation of planar linear advection
(section 4.1 and the advection form of section 3.2's stencil listing).

Test infrastructure only (see ``oracle/__init__.py``).  Equation "lin_adv":
du/dt + div(beta u) = 0 on the periodic rectangle [0, lx] x [0, ly] with a
constant velocity beta.  The same discretisation as the shallow-water oracles:
orthonormal Legendre tensor basis of degree r per direction, (r+1)-point
Gauss-Legendre rules for the volume and the edges, the weak form of equation
"dg_parts" with the Rusanov flux of equation "rusanov" (for a linear flux the
largest eigenvalue is |beta . n| and the Rusanov flux is the upwind flux), and
the exact mass matrix (dx dy / 4) I.  Dense per-element matrices, explicit
``np.roll`` for the periodic neighbours.
"""
import numpy as np

from .basis import gauss_legendre, legendre


class AdvectionDG:
    """nx x ny elements on [0, lx] x [0, ly], periodic, velocity (bx, by)."""

    def __init__(self, nx, ny, order, lx=1.0, ly=1.0, beta=(1.0, 1.0)):
        self.nx, self.ny, self.order = int(nx), int(ny), int(order)
        self.lx, self.ly = float(lx), float(ly)
        self.bx, self.by = float(beta[0]), float(beta[1])
        n = self.order + 1
        self.n, self.N = n, n * n
        self.E = self.nx * self.ny
        self.dx, self.dy = self.lx / self.nx, self.ly / self.ny
        xi, w = gauss_legendre(n)
        P, dP = legendre(self.order, xi)
        Pe, _ = legendre(self.order, np.array([-1.0, 1.0]))
        Pm, Pp = Pe[0], Pe[1]
        self.xi, self.w = xi, w
        pk, sk = np.tile(np.arange(n), n), np.repeat(np.arange(n), n)
        self.V = P[pk][:, pk] * P[sk][:, sk]           # [node, mode]
        self.DX = dP[pk][:, pk] * P[sk][:, sk]
        self.DY = P[pk][:, pk] * dP[sk][:, sk]
        self.Wq = w[pk] * w[sk]
        self.EE = Pp[pk][None, :] * P[:, sk]           # [edge node s, mode]
        self.EW = Pm[pk][None, :] * P[:, sk]
        self.EN = P[:, pk] * Pp[sk][None, :]           # [edge node p, mode]
        self.ES = P[:, pk] * Pm[sk][None, :]
        self.M = 0.25 * self.dx * self.dy * (self.V.T * self.Wq) @ self.V

    def grid(self, q):
        return np.asarray(q, dtype=np.float64).reshape(self.ny, self.nx, self.N)

    def upwind(self, um, up, b):
        """Rusanov flux of f(u) = b u through an edge, minus side west/south:
        (f(u-) + f(u+))/2 - |b|/2 (u+ - u-), the upwind value for this f."""
        return 0.5 * b * (um + up) - 0.5 * abs(b) * (up - um)

    def residual(self, q):
        q = self.grid(q)
        U = np.einsum("km,jim->jik", self.V, q)
        W = self.Wq
        vol = (0.5 * self.dy * np.einsum("km,jik->jim", self.DX, W * self.bx * U)
               + 0.5 * self.dx * np.einsum("km,jik->jim", self.DY, W * self.by * U))
        uE = np.einsum("sm,jim->jis", self.EE, q)
        uW = np.einsum("sm,jim->jis", self.EW, q)
        uN = np.einsum("pm,jim->jip", self.EN, q)
        uS = np.einsum("pm,jim->jip", self.ES, q)
        FE = self.upwind(uE, np.roll(uW, -1, axis=1), self.bx)
        FW = np.roll(FE, 1, axis=1)
        GN = self.upwind(uN, np.roll(uS, -1, axis=0), self.by)
        GS = np.roll(GN, 1, axis=0)
        w = self.w
        surf = (0.5 * self.dy * (np.einsum("sm,jis->jim", self.EE, w * FE)
                                 - np.einsum("sm,jis->jim", self.EW, w * FW))
                + 0.5 * self.dx * (np.einsum("pm,jip->jim", self.EN, w * GN)
                                   - np.einsum("pm,jip->jim", self.ES, w * GS)))
        return vol - surf

    def rhs(self, q):
        res = self.residual(q).reshape(-1, self.N)
        return np.linalg.solve(self.M, res.T).T.reshape(self.E, self.N)

    def project(self, fun, extra=9):
        """L2 projection of fun(x, y) onto the basis ((r+1+extra)^2 points)."""
        nq = self.n + extra
        xq, wq = gauss_legendre(nq)
        Pq, _ = legendre(self.order, xq)
        x = (np.arange(self.nx)[:, None] + 0.5 * (1.0 + xq[None, :])) * self.dx
        y = (np.arange(self.ny)[:, None] + 0.5 * (1.0 + xq[None, :])) * self.dy
        X, Y = np.meshgrid(x.ravel(), y.ravel())
        vals = np.asarray(fun(X, Y), dtype=np.float64).reshape(self.ny, nq, self.nx, nq)
        b = 0.25 * self.dx * self.dy * np.einsum("jsip,s,p,pa,sb->jiba", vals, wq, wq, Pq, Pq)
        return np.linalg.solve(self.M, b.reshape(-1, self.N).T).T.reshape(self.E, self.N)

    def l2_error(self, q, fun, extra=9):
        """L2 norm over the domain of (u_h - fun), by an (r+1+extra)-point
        Gauss-Legendre rule per direction per element."""
        nq = self.n + extra
        xq, wq = gauss_legendre(nq)
        Pq, _ = legendre(self.order, xq)
        x = (np.arange(self.nx)[:, None] + 0.5 * (1.0 + xq[None, :])) * self.dx
        y = (np.arange(self.ny)[:, None] + 0.5 * (1.0 + xq[None, :])) * self.dy
        X, Y = np.meshgrid(x.ravel(), y.ravel())
        ex = np.asarray(fun(X, Y), dtype=np.float64).reshape(self.ny, nq, self.nx, nq)
        g = self.grid(q).reshape(self.ny, self.nx, self.n, self.n)        # [j, i, b, a]
        uh = np.einsum("jiba,pa,sb->jsip", g, Pq, Pq)
        d2 = np.einsum("jsip,s,p->", (uh - ex) ** 2, wq, wq) * 0.25 * self.dx * self.dy
        return float(np.sqrt(d2))
