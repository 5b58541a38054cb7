"""Gauss-Legendre quadrature and the orthonormal Legendre basis, in FP64.

Test infrastructure only (see ``oracle/__init__.py``).

The modal basis of the paper (section 2, "Modal DG approach", basis expansion
equation) is a tensor product of Legendre polynomials on the reference square
[-1, 1]^2.  The paper only says "bivariate Legendre polynomials"; the reading
used here is the orthonormal one, P~_a(x) = sqrt((2a+1)/2) P_a(x), so that the
reference mass matrix is the identity.

The quadrature nodes and weights are precomputed on the CPU (section 3.2,
"DG solver: precomputation").  They are computed here by the Golub-Welsch
method: the nodes are the eigenvalues of the symmetric Jacobi matrix of the
Legendre three-term recurrence and the weights are twice the squared first
components of the normalised eigenvectors.
"""
import numpy as np


def gauss_legendre(n):
    """n-point Gauss-Legendre rule on [-1, 1]; nodes ascending.

    Golub-Welsch: J is tridiagonal with off-diagonal k / sqrt(4k^2 - 1),
    k = 1..n-1 (monic Legendre recurrence); x = eig(J), w = 2 * v0^2.
    """
    if n < 1:
        raise ValueError("n >= 1")
    if n == 1:
        return np.array([0.0]), np.array([2.0])
    k = np.arange(1, n, dtype=np.float64)
    beta = k / np.sqrt(4.0 * k * k - 1.0)
    jac = np.diag(beta, 1) + np.diag(beta, -1)
    x, vec = np.linalg.eigh(jac)
    w = 2.0 * vec[0, :] ** 2
    # symmetric rule: enforce exact symmetry of the nodes and weights
    x = 0.5 * (x - x[::-1])
    w = 0.5 * (w + w[::-1])
    return x, w


def legendre(nmax, x):
    """Values and derivatives of the orthonormal Legendre polynomials.

    Returns (P, dP) with shape (len(x), nmax+1): P[:, a] = P~_a(x).
    Bonnet's recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1} and
    P'_{k+1} = P'_{k-1} + (2k+1) P_k, then scaling by sqrt((2a+1)/2).
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    P = np.zeros((x.size, nmax + 1))
    dP = np.zeros((x.size, nmax + 1))
    P[:, 0] = 1.0
    if nmax >= 1:
        P[:, 1] = x
        dP[:, 1] = 1.0
    for k in range(1, nmax):
        P[:, k + 1] = ((2 * k + 1) * x * P[:, k] - k * P[:, k - 1]) / (k + 1)
        dP[:, k + 1] = dP[:, k - 1] + (2 * k + 1) * P[:, k]
    scale = np.sqrt((2.0 * np.arange(nmax + 1) + 1.0) / 2.0)
    return P * scale, dP * scale
