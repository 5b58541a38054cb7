"""Comparison helpers of the parity tests.

The bar is componentwise: |gpu - oracle| <= tol * scale, entry by entry,
where scale (SphereDG.rhs_scale) is the size of the terms summed into that
entry.  A normwise ||d||_inf / ||ref||_inf is reported beside it; near the
poles it is dominated by cancellation that no evaluation order avoids (a
one-ulp change of the input moves the FP64 oracle itself by ~1e-9 there at
180 x 90, r = 3).
"""
import numpy as np

TOL = {"f64": 1e-12, "f32": 1e-5}


def errors(got, ref, scale):
    got = np.asarray(got, dtype=np.float64).reshape(ref.shape)
    d = np.abs(got - ref)
    comp = (d / np.maximum(scale, np.finfo(np.float64).tiny)).max(axis=(0, 2))
    norm = d.max(axis=(0, 2)) / np.maximum(np.abs(ref).max(axis=(0, 2)), np.finfo(np.float64).tiny)
    return comp, norm
