"""NumPy oracle of the learned right-hand-side correction (not in the paper:
an addition to the method, see the header of ``oracle/__init__.py``).

Test infrastructure only.  FP64 arithmetic with the same BF16 rounding
points as the GPU kernels (round to nearest even of the FP32 value): the
GEMM inputs (features, hidden activations, weights, back-propagated
gradients) are rounded to BF16; accumulation, biases, GELU and the loss are
exact.  ``exact=True`` switches every rounding off, for finite-difference
checks.

Network: 108 -> 256 -> 256 -> 12, GELU (erf form) after the two hidden
layers.  Loss: mean squared error over the unmasked outputs.
"""
import math

import numpy as np
from scipy.special import erf

N_IN, N_HID, N_OUT = 108, 256, 12


def bf16(x):
    """Round to BF16 (nearest even) via FP32, returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    u = ((u + rounding) >> 16) << 16
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out[nan] = np.nan
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def init_params(seed, n_in=N_IN, n_hid=N_HID, n_out=N_OUT):
    """He-normal weights (std sqrt(2/fan_in)), zero biases; W[k] is (in, out)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((n_in, n_hid)) * math.sqrt(2.0 / n_in)
    W2 = rng.standard_normal((n_hid, n_hid)) * math.sqrt(2.0 / n_hid)
    W3 = rng.standard_normal((n_hid, n_out)) * math.sqrt(2.0 / n_hid)
    return {"W1": W1, "b1": np.zeros(n_hid), "W2": W2, "b2": np.zeros(n_hid),
            "W3": W3, "b3": np.zeros(n_out)}


def forward(p, X, exact=False):
    r = (lambda a: a) if exact else bf16
    Xb = r(X)
    Z1 = Xb @ r(p["W1"]) + p["b1"]
    H1 = r(gelu(Z1))
    Z2 = H1 @ r(p["W2"]) + p["b2"]
    H2 = r(gelu(Z2))
    Y = H2 @ r(p["W3"]) + p["b3"]
    return Y, {"X": Xb, "Z1": Z1, "H1": H1, "Z2": Z2, "H2": H2}


def loss(Y, T, mask):
    """Mean squared error over the unmasked outputs (mask: 0/1 per output)."""
    n = Y.shape[0] * mask.sum()
    return float(((Y - T) ** 2 * mask).sum() / n)


def backward(p, cache, Y, T, mask, exact=False):
    r = (lambda a: a) if exact else bf16
    n = Y.shape[0] * mask.sum()
    dY = 2.0 * (Y - T) * mask / n
    dYb = r(dY)
    g = {"W3": cache["H2"].T @ dYb, "b3": dY.sum(axis=0)}
    dZ2 = (dYb @ r(p["W3"]).T) * gelu_grad(cache["Z2"])
    dZ2b = r(dZ2)
    g["W2"] = cache["H1"].T @ dZ2b
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2b @ r(p["W2"]).T) * gelu_grad(cache["Z1"])
    dZ1b = r(dZ1)
    g["W1"] = cache["X"].T @ dZ1b
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place; state holds m, v per parameter and the step t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m" + k, np.zeros_like(p[k]))
        v = state.setdefault("v" + k, np.zeros_like(p[k]))
        m *= b1
        m += (1 - b1) * g[k]
        v *= b2
        v += (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] -= lr * mh / (np.sqrt(vh) + eps)
    return p


# ----------------------------------------------------------------- features
def stencil_features(q1, n_lon, n_lat):
    """3x3 element stencil of an r = 1 state q1[E][3][4] -> X[E][108].

    Feature index ((dj+1)*3 + (di+1))*12 + v*4 + m for the neighbour at
    longitude offset di (periodic) and latitude offset dj (clamped at the
    poles: the pole row stands in for the missing row)."""
    g = np.asarray(q1).reshape(n_lat, n_lon, 12)
    out = np.empty((n_lat, n_lon, 9, 12))
    for dj in (-1, 0, 1):
        rows = np.clip(np.arange(n_lat) + dj, 0, n_lat - 1)
        for di in (-1, 0, 1):
            out[:, :, (dj + 1) * 3 + (di + 1)] = np.roll(g[rows], -di, axis=1)
    return out.reshape(n_lat * n_lon, 108)
