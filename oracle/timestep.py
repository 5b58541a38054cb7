"""Explicit Runge-Kutta steps of the method of lines (section 2, Table
"Butcher").  Test infrastructure only (see ``oracle/__init__.py``).

``ssp_rk3`` is the Shu-Osher form of the third tableau, the form the GPU path
also uses; ``butcher_step`` applies any explicit tableau literally (stages
k_i = L(q + dt sum_j a_ij k_j), q + dt sum_i b_i k_i) and serves to check it.
"""
import numpy as np


def ssp_rk3(L, q, dt):
    q0 = np.asarray(q)
    q1 = q0 + dt * L(q0)
    q2 = 0.75 * q0 + 0.25 * (q1 + dt * L(q1))
    return (1.0 / 3.0) * q0 + (2.0 / 3.0) * (q2 + dt * L(q2))


def butcher_step(L, q, dt, A, b):
    q0 = np.asarray(q)
    A = np.asarray(A, dtype=np.float64)
    k = []
    for i in range(len(b)):
        qi = q0 + dt * sum(A[i, j] * k[j] for j in range(i)) if i else q0
        k.append(L(qi))
    return q0 + dt * sum(bi * ki for bi, ki in zip(b, k))
