"""Comparison helpers of the parity tests.

The bar is componentwise: |gpu - oracle| <= tol * scale, entry by entry,
where scale (SphereDG.rhs_scale) is the size of the terms summed into that
entry.  Beside it the normwise error ||d||_inf / ||ref||_inf per variable is
bounded by a multiple of the oracle's own one-ulp sensitivity: the normwise
change of the FP64 oracle's output when every input value is moved by one
unit in the last place of the compared precision (random sign).  Near the
poles that sensitivity is dominated by cancellation that no evaluation
order avoids (about 1e-9 for h at 180 x 90, r = 3, in FP64), so it, not
1e-12, is the scale a normwise comparison can be held to.
"""
import numpy as np

TOL = {"f64": 1e-12, "f32": 1e-5}
# normwise error <= NORM_K * (one-ulp sensitivity of the oracle) per variable
NORM_K = 16.0


def errors(got, ref, scale):
    got = np.asarray(got, dtype=np.float64).reshape(ref.shape)
    d = np.abs(got - ref)
    comp = (d / np.maximum(scale, np.finfo(np.float64).tiny)).max(axis=(0, 2))
    norm = d.max(axis=(0, 2)) / np.maximum(np.abs(ref).max(axis=(0, 2)), np.finfo(np.float64).tiny)
    return comp, norm


def norm_bound(sens, dtype):
    """Normwise bar: NORM_K times the one-ulp sensitivity, and never below a
    few units of roundoff of the compared precision."""
    eps = np.finfo(np.float64 if dtype == "f64" else np.float32).eps
    return NORM_K * np.asarray(sens) + 4.0 * eps


def ulp_sensitivity(rhs, q, ref, dtype, seed=0):
    """Normwise relative change of rhs(q) per variable when each entry of q
    (already rounded to `dtype`) moves by one ulp of `dtype` up or down at
    random.  rhs is the oracle's FP64 right-hand side."""
    rng = np.random.default_rng(seed)
    up = rng.integers(0, 2, size=q.shape).astype(bool)
    if dtype == "f32":
        q32 = np.asarray(q, dtype=np.float32)
        qp = np.where(up, np.nextafter(q32, np.float32(np.inf)),
                      np.nextafter(q32, np.float32(-np.inf))).astype(np.float64)
    else:
        q64 = np.asarray(q, dtype=np.float64)
        qp = np.where(up, np.nextafter(q64, np.inf), np.nextafter(q64, -np.inf))
    d = np.abs(rhs(qp) - ref)
    return d.max(axis=(0, 2)) / np.maximum(np.abs(ref).max(axis=(0, 2)), np.finfo(np.float64).tiny)
