"""Eigenvectors of an upper-triangular matrix (TREVC, Sec. 5) -- TEST
INFRASTRUCTURE ONLY.

For an upper-triangular T with distinct diagonal entries, T X = X D with
D = diag(T) has an upper-triangular solution X; Sec. 5 gives its entries
above the diagonal, column by column, as

    X_ij = (T_ij X_jj + sum_{k=i+1}^{j-1} T_ik X_kj) / (T_jj - T_ii),  i < j,

with X_jj free.  Here X_jj = 1.  This is that definition written out, one
entry at a time (the blocked schedule of Alg. 8 computes the same sums in
another order).  The same recurrence for an upper-triangular pencil (T, S),
whose j-th eigenvalue is lambda_j = T_jj / S_jj, follows from
(T - lambda_j S) x = 0 with x_j = 1:

    x_i = -(sum_{k=i+1}^{j} (T_ik - lambda_j S_ik) x_k) / (T_ii - lambda_j S_ii),

which for S = I is the formula above.

A denominator smaller than eps (|T_ii| + |lambda_j S_ii|) + the smallest
normal number is replaced by that bound with its sign (as LAPACK's TREVC
guards its divisions); with distinct, well-separated eigenvalues this never
happens.  Only the upper triangles of T and S are read.
"""
from __future__ import annotations

import numpy as np

EPS = np.finfo(np.float64).eps
TINY = np.finfo(np.float64).tiny


def _guard(den: float, t_ii: float, ls_ii: float) -> float:
    smin = EPS * (abs(t_ii) + abs(ls_ii)) + TINY
    if abs(den) < smin:
        return smin if den >= 0.0 else -smin
    return den


def trevc(t: np.ndarray, s: np.ndarray | None = None) -> np.ndarray:
    """X (n x n, upper triangular, unit diagonal) with T X = S X diag(lambda),
    lambda_j = T_jj / S_jj (S = I when s is None)."""
    t = np.triu(np.asarray(t, dtype=np.float64))
    n = t.shape[0]
    s = np.eye(n) if s is None else np.triu(np.asarray(s, dtype=np.float64))
    lam = np.diag(t) / np.diag(s)
    x = np.zeros((n, n))
    for j in range(n):
        x[j, j] = 1.0
        for i in range(j - 1, -1, -1):
            # sum over k = i+1 .. j of (T_ik - lambda_j S_ik) x_kj (a dot product)
            acc = float(np.dot(t[i, i + 1:j + 1] - lam[j] * s[i, i + 1:j + 1], x[i + 1:j + 1, j]))
            x[i, j] = -acc / _guard(t[i, i] - lam[j] * s[i, i], t[i, i], lam[j] * s[i, i])
    return x


def eigenvalues(t: np.ndarray, s: np.ndarray | None = None) -> np.ndarray:
    """lambda_j = T_jj / S_jj, the diagonal of D."""
    d = np.diag(np.asarray(t, dtype=np.float64))
    return d if s is None else d / np.diag(np.asarray(s, dtype=np.float64))
