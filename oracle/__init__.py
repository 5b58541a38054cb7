"""FP64 CPU oracle of the modal DG shallow-water right-hand side on the sphere.

TEST INFRASTRUCTURE.  This package is a plain, slow, dense NumPy
implementation written directly from the paper's equations (section 2).  It
exists to check the HIP path: only the tests, the smoke check and the CPU
baseline leg of the benchmark may import it.  The product path (the C-ABI
library and its Python binding) never imports, calls or falls back to it,
and this package imports nothing from the product.

``plane`` is the same scheme on the doubly periodic f-plane of section 4.2
(the planar shallow-water system, no metric terms).

``advection`` is the same discretisation of planar linear advection (section
4.1's convergence test), pinned by the paper's printed errors.

``mlp`` is the oracle of the learned right-hand-side correction, an addition
to the paper's method (a small network that corrects the r = 1 right-hand
side towards the projection of higher-order runs); it is pinned by finite
differences and library routines.

Every function here is pinned by tests against facts that do not come from
the oracle itself (quadrature exactness, closed forms, a textbook first-order
finite-volume scheme at r = 0, lake at rest, conservation, symmetries,
convergence of the operator on smooth fields, Runge-Kutta stability
polynomials and the paper's printed Butcher tableaux).
"""
from .basis import gauss_legendre, legendre
from .sphere import SphereDG, project_order
from .plane import PlaneDG
from .advection import AdvectionDG
from . import mlp
from .timestep import ssp_rk3, butcher_step

__all__ = ["gauss_legendre", "legendre", "SphereDG", "PlaneDG", "AdvectionDG", "project_order",
           "ssp_rk3", "butcher_step", "mlp"]
