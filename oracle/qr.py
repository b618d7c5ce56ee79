"""QR, RQ and QL factorizations for the oracle.

The paper only needs orthogonal-triangular factorizations (QR, RQ, QL, LQ;
Sec. 3 preamble and Sec. 4.2 "Subroutines", which notes the RQ/QL/LQ variants
cost the same as QR).  It fixes no sign convention; the oracle normalizes every
triangular factor to a non-negative diagonal, which makes each factorization of
a full-rank matrix unique (so two correct implementations must agree).

``householder_qr_loop`` is a pure-Python Householder QR used only to cross-check
the LAPACK path on small inputs.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def householder_qr_loop(m: np.ndarray):
    """Householder QR by explicit loops (no blocking): returns (Q, R) with
    Q (rows x rows) orthogonal, R (rows x cols) upper trapezoidal and
    Q @ R == m.  Each reflector is I - tau v v^T with v[j] = 1 and
    beta = -sign(alpha) * ||x||, the usual convention."""
    a = np.array(m, dtype=np.float64, copy=True)
    rows, cols = a.shape
    q = np.eye(rows)
    for j in range(min(rows, cols)):
        x = a[j:, j].copy()
        alpha = x[0]
        sub = 0.0
        for i in range(1, x.size):
            sub += x[i] * x[i]
        if sub == 0.0:
            continue  # H = I
        norm = (alpha * alpha + sub) ** 0.5
        beta = -norm if alpha >= 0 else norm
        tau = (beta - alpha) / beta
        v = x / (alpha - beta)
        v[0] = 1.0
        # apply H = I - tau v v^T to the trailing columns of a, and accumulate q
        for c in range(j, cols):
            w = 0.0
            for i in range(v.size):
                w += v[i] * a[j + i, c]
            for i in range(v.size):
                a[j + i, c] -= tau * v[i] * w
        for r in range(rows):
            w = 0.0
            for i in range(v.size):
                w += q[r, j + i] * v[i]
            for i in range(v.size):
                q[r, j + i] -= tau * w * v[i]
        a[j + 1:, j] = 0.0
    return q, a


def _sign_vec(d: np.ndarray) -> np.ndarray:
    s = np.sign(d)
    s[s == 0] = 1.0
    return s


def qr_signed(m: np.ndarray, full: bool = True):
    """QR with R's diagonal made non-negative: m = Q R.

    full=True returns Q square (rows x rows), R (rows x cols); the sign flip
    touches only the first min(rows, cols) columns of Q."""
    mode = "full" if full else "economic"
    q, r = sla.qr(np.asarray(m, dtype=np.float64), mode=mode)
    k = min(r.shape)
    s = _sign_vec(np.diag(r)[:k])
    q = q.copy()
    r = r.copy()
    q[:, :k] *= s[None, :]
    r[:k, :] *= s[:, None]
    return q, r


def rq_signed(x: np.ndarray):
    """RQ of a square matrix through the reversal J (Sec. 4.2 notes RQ costs
    what QR costs): with Y = J X^T J = Qt Rt, X = (J Rt^T J)(J Qt^T J).
    Returns (R, W) with R upper triangular, non-negative diagonal, W orthogonal,
    X = R W."""
    x = np.asarray(x, dtype=np.float64)
    y = x.T[::-1, ::-1]
    qt, rt = qr_signed(y)
    r = rt.T[::-1, ::-1]
    w = qt.T[::-1, ::-1]
    return np.ascontiguousarray(r), np.ascontiguousarray(w)


def ql_signed(x: np.ndarray):
    """QL of a square matrix through the reversal J: with X J = Qt Rt,
    X = (Qt J)(J Rt J).  Returns (Q, L) with L lower triangular, non-negative
    diagonal, X = Q L."""
    x = np.asarray(x, dtype=np.float64)
    qt, rt = qr_signed(x[:, ::-1])
    q = qt[:, ::-1]
    l_ = rt[::-1, ::-1]
    return np.ascontiguousarray(q), np.ascontiguousarray(l_)
