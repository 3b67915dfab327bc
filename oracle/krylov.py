"""Rank-m Krylov subspace approximation of the kernel acting on the residual.

Paper, Methods section 6: with the identity as preconditioner (K0 = I,
eq. 33) the kernel K = J^-1 (eqs. 15-16) acting on the residual
W0 = D0[X] S - X is approximated by sum_ij V_i M_ij <W_j, W0> (eq. 34), with
the Frobenius inner product <A, B> = Tr[A^T B].  The paper leaves the
construction of V_i, M and W_i to its ref. [16]; this oracle takes the reading
that makes eq. 34 the least-squares (pseudo-inverse) solution of J Y = W0 over
a Krylov space of J:

  V_1 = W0 / ||W0||;
  W_k = J V_k = D1[V_k] - V_k, the directional derivative of the residual along
        V_k, D1 from the canonical response (eq. 36);
  V_{k+1} = W_k orthogonalised twice against V_1..V_k (classical Gram-Schmidt,
        applied twice), then normalised;
  O_ij = <W_i, W_j>, M = O^-1, Y = sum_ij V_i M_ij <W_j, W0>.

A direction whose orthogonalised norm falls below 1e-12 of the norm it came
from ends the space early (breakdown; reported as a smaller rank).  With
rank equal to the grade of the Krylov space, Y is exactly J^-1 W0.
"""

from __future__ import annotations

import numpy as np


def inner(A: np.ndarray, B: np.ndarray) -> float:
    """Frobenius inner product Tr[A^T B]."""
    return float(np.sum(A * B))


def krylov_kernel(X: np.ndarray, P0: np.ndarray, jacobian_apply, m: int, tol: float = 0.0,
                  breakdown: float = 1e-12):
    """Return (Y, rank_used, rel_resid) with Y ~ J^-1 (P0 - X) (eq. 34).

    ``jacobian_apply(V)`` must return J V = P1[V] - V, the directional
    derivative of the residual along V."""
    W0 = np.asarray(P0, dtype=np.float64) - np.asarray(X, dtype=np.float64)
    nW0 = np.sqrt(inner(W0, W0))
    Y = np.zeros_like(W0)
    if nW0 == 0.0 or m <= 0:
        return Y, 0, 0.0
    Vs, Ws = [], []
    src = W0
    rel = 1.0
    for _ in range(m):
        v = src.copy()
        for _sweep in range(2):
            for vj in Vs:
                v = v - inner(vj, v) * vj
        nv = np.sqrt(inner(v, v))
        if nv <= breakdown * np.sqrt(inner(src, src)):
            break
        v = v / nv
        w = jacobian_apply(v)
        Vs.append(v)
        Ws.append(w)
        k = len(Vs)
        O = np.array([[inner(Ws[i], Ws[j]) for j in range(k)] for i in range(k)])
        rhs = np.array([inner(Ws[j], W0) for j in range(k)])
        c = np.linalg.solve(O, rhs)
        Y = sum(c[i] * Vs[i] for i in range(k))
        r = sum(c[i] * Ws[i] for i in range(k)) - W0
        rel = np.sqrt(inner(r, r)) / nW0
        if rel < tol:
            break
        src = w
    return Y, len(Vs), rel
