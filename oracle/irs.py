"""Implicit repeated squaring (Alg. 3, Sec. 3.1; correctness in Sec. 3.2).

Starting from (A_0, B_0) = (A, B), each step takes the QR factorization of the
stacked 2n x n matrix [B_j; -A_j] = Q [R_j; 0], splits the 2n x 2n Q into n x n
blocks Q11..Q22 and sets A_{j+1} = Q12^T A_j, B_{j+1} = Q22^T B_j.  The loop
stops once ||R_j - R_{j-1}||_1 <= tau ||R_{j-1}||_1 and returns (A_p, B_p) with
p = j + 1, or gives up when j exceeds maxit.

Readings the paper leaves open:
* R_j is only defined up to the signs of its rows; the oracle normalizes its
  diagonal to be non-negative, so R_j is the unique upper Cholesky factor of
  A_j^T A_j + B_j^T B_j and the convergence test compares like with like.
* tau defaults to sqrt(eps) of the working precision and maxit to 60 (the
  range over which the paper plots its experiments).
* the iterate returned on convergence is the (A_{j+1}, B_{j+1}) already formed
  at the test; no extra step is taken.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .qr import qr_signed

EPS64 = float(np.finfo(np.float64).eps)


def norm1(x: np.ndarray) -> float:
    """Matrix 1-norm: largest column sum of absolute values."""
    return float(np.max(np.sum(np.abs(x), axis=0))) if x.size else 0.0


@dataclass
class IRSResult:
    A: np.ndarray
    B: np.ndarray
    p: int
    converged: bool
    R_history: list = field(default_factory=list)
    rel_change: list = field(default_factory=list)


def irs(a0: np.ndarray, b0: np.ndarray, tau: float | None = None, maxit: int = 60,
        record: bool = False) -> IRSResult:
    n = a0.shape[0]
    if tau is None:
        tau = EPS64 ** 0.5
    aj = np.array(a0, dtype=np.float64, copy=True)
    bj = np.array(b0, dtype=np.float64, copy=True)
    r_prev = None
    hist, changes = [], []
    j = 0
    while True:
        m = np.vstack([bj, -aj])
        q, r = qr_signed(m, full=True)
        rj = r[:n, :n]
        q12 = q[:n, n:]
        q22 = q[n:, n:]
        a_next = q12.T @ aj
        b_next = q22.T @ bj
        if record:
            hist.append(rj.copy())
        converged = False
        if r_prev is not None:
            diff = norm1(rj - r_prev)
            ref = norm1(r_prev)
            changes.append(diff / ref if ref > 0 else np.inf)
            converged = diff <= tau * ref
        aj, bj = a_next, b_next
        if converged:
            return IRSResult(aj, bj, j + 1, True, hist, changes)
        r_prev = rj
        j += 1
        if j > maxit:
            return IRSResult(aj, bj, j, False, hist, changes)
