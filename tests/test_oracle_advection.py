"""Pins of the planar linear-advection oracle (section 4.1's convergence test)
against the paper's printed errors and rates, a first-order upwind finite-
volume scheme at r = 0, conservation and the x <-> y mirror."""
import json
import os

import numpy as np
import pytest

from oracle import butcher_step
from oracle.advection import AdvectionDG

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TAB = json.load(open(os.path.join(GOLDEN, "butcher_tableaux.json")))["RK4"]
PAPER = json.load(open(os.path.join(GOLDEN, "linear_advection_errors.json")))


def u0(x, y):
    return np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)


def run_to_one(k, p):
    """RK4 to T = 1 (one period) with a step small enough that the time error
    is far below the spatial one; returns the L2 error against u0."""
    m = AdvectionDG(k, k, p)
    q = m.project(u0)
    n = int(np.ceil(1.0 / (0.1 * m.dx / ((2 * p + 1) * 2.0))))
    for _ in range(n):
        q = butcher_step(m.rhs, q, 1.0 / n, TAB["A"], TAB["b"])
    return m.l2_error(q, u0)


def test_p3_error_matches_paper():
    """r = 3 on 20 x 20 elements: the paper's two implementations print
    2.030e-6 and 2.061e-6; the oracle's error agrees within 2 %."""
    e = run_to_one(20, 3)
    assert abs(e / PAPER["GT4Py"]["3"]["20"] - 1) < 0.02, e
    assert abs(e / PAPER["G4GT"]["3"]["20"] - 1) < 0.03, e


@pytest.mark.parametrize("p,k1,lo,hi", [(1, 20, 1.9, 2.4), (2, 10, 2.8, 3.2), (3, 10, 3.8, 4.3)])
def test_convergence_rates_match_paper(p, k1, lo, hi):
    """Rates between k1 and 2 k1 elements per direction: about p + 1, as in
    the paper's tables (2.00-2.22, 2.98-3.00, 3.96-4.22)."""
    rate = np.log2(run_to_one(k1, p) / run_to_one(2 * k1, p))
    assert lo < rate < hi, rate


def test_r0_is_first_order_upwind():
    nx, ny = 7, 5
    rng = np.random.default_rng(4)
    U = rng.standard_normal((ny, nx))
    bx, by = 0.7, -1.3
    m = AdvectionDG(nx, ny, 0, lx=2.0, ly=1.5, beta=(bx, by))
    got = m.rhs((2.0 * U).reshape(-1, 1)).reshape(ny, nx) / 2.0
    dx, dy = 2.0 / nx, 1.5 / ny
    up_x = U if bx > 0 else np.roll(U, -1, axis=1)            # value carried through the east edge
    FE = bx * up_x
    up_y = U if by > 0 else np.roll(U, -1, axis=0)
    GN = by * up_y
    ref = -(FE - np.roll(FE, 1, axis=1)) / dx - (GN - np.roll(GN, 1, axis=0)) / dy
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_conservation_and_mirror(p):
    m = AdvectionDG(6, 5, p, lx=1.0, ly=0.8, beta=(1.0, 0.6))
    q = m.project(lambda x, y: 1.0 + np.cos(2 * np.pi * x + 0.3) * np.sin(2 * np.pi * y / 0.8) ** 2)
    d = m.rhs(q)
    # d/dt of the integral: the mode-00 coefficients sum to zero
    assert abs(d[:, 0].sum()) <= 1e-12 * np.abs(d).max() * m.E
    # x <-> y mirror with beta swapped maps the operator onto itself
    mt = AdvectionDG(5, 6, p, lx=0.8, ly=1.0, beta=(0.6, 1.0))
    n = p + 1

    def tr(a, nx, ny):
        return np.ascontiguousarray(a.reshape(ny, nx, n, n).transpose(1, 0, 3, 2)).reshape(nx * ny, n * n)

    assert np.abs(mt.rhs(tr(q, 6, 5)) - tr(d, 6, 5)).max() <= 1e-12 * np.abs(d).max()
