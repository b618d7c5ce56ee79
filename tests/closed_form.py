"""Closed form of implicit repeated squaring for a symmetric A = Q diag(d) Q^T
with B = I and the half-plane map (sigma, s).  Used only to pin the oracle.

Derivation (from the IRS step and the identity Q12^T B_j = Q22^T A_j of
Sec. 3.2): write a0 = d - sigma + s, b0 = d - sigma - s, so the mapped pencil is
(Q diag(a0) Q^T, Q diag(b0) Q^T).  If A_j = Z Q diag(a) Q^T and
B_j = Z Q diag(b) Q^T with Z orthogonal, the columns of
[Q diag(a/r) Q^T; Q diag(b/r) Q^T], r = sqrt(a^2 + b^2), are orthonormal and
orthogonal to [B_j; -A_j], so any IRS step yields
A_{j+1} = Z' Q diag(a^2/r) Q^T and B_{j+1} = Z' Q diag(b^2/r) Q^T.  Hence
R_j (non-negative diagonal) is the upper Cholesky factor of Q diag(r^2) Q^T,
and (A_p + B_p)^{-1} A_p = Q diag(a/(a+b)) Q^T.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def norm1(x):
    return float(np.max(np.sum(np.abs(x), axis=0)))


def irs_sym_closed_form(d, q, sigma=0.0, s=1.0, tau=None, maxit=60):
    """Returns (R list, p, converged, final a, final b) following the same
    stopping rule as the algorithm (test from j >= 1, p = j + 1)."""
    if tau is None:
        tau = np.finfo(np.float64).eps ** 0.5
    a = np.asarray(d, dtype=np.float64) - sigma + s
    b = np.asarray(d, dtype=np.float64) - sigma - s
    rs = []
    r_prev = None
    j = 0
    while True:
        r = np.sqrt(a * a + b * b)
        gram = (q * (r * r)[None, :]) @ q.T
        gram = 0.5 * (gram + gram.T)
        rj = sla.cholesky(gram, lower=False)
        rs.append(rj)
        conv = False
        if r_prev is not None:
            conv = norm1(rj - r_prev) <= tau * norm1(r_prev)
        a, b = a * a / r, b * b / r
        if conv:
            return rs, j + 1, True, a, b
        r_prev = rj
        j += 1
        if j > maxit:
            return rs, j, False, a, b


def predicted_p_sym(d, sigma=0.0, s=1.0, tau=None):
    """Iteration count from the scalar recursion alone (no matrices): the
    relative change of R at step j is ~ max_i min(|a_i|,|b_i|)/max(...)
    of that step's iterate.  Used as a coarse cross-check."""
    rs, p, conv, _, _ = irs_sym_closed_form(d, np.eye(len(d)), sigma, s, tau)
    return p
