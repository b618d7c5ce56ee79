"""FP64 Newton refinement of a symmetric split -- TEST INFRASTRUCTURE ONLY.

Not in the paper (it has no mixed precision): the library's FP32
repeated-squaring path ends with this step, and the oracle states what it
computes, written from the definition.

Given a symmetric A and an orthogonal Q whose leading k columns nearly span an
invariant subspace, A_hat = Q^T A Q = [A11 E^T; E A22].  For
U = [I -X^T; X I] the (2,1) block of U^T A_hat U is
E + A22 X - X A11 - X E^T X, so the Newton step takes X with
X A11 - A22 X = E (a Sylvester equation, solved here by the Bartels-Stewart
routine of SciPy, a library primitive).  U^T U = diag(I + X^T X, I + X X^T),
so Q U diag((I + X^T X)^{-1/2}, (I + X X^T)^{-1/2}) is orthogonal and keeps
the two column blocks' spans.  The step is repeated until
||E||_1 / ||A||_1 <= tol.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .irs import norm1


def _inv_sqrt_spd(m: np.ndarray) -> np.ndarray:
    w, v = np.linalg.eigh(m)
    return (v / np.sqrt(w)) @ v.T


def refine_sym(a: np.ndarray, q: np.ndarray, k: int, tol: float = 1e-14, rounds: int = 3):
    """Returns (Q, A_hat, e history) after at most `rounds` Newton steps."""
    a = np.asarray(a, dtype=np.float64)
    q = np.array(q, dtype=np.float64)
    n = a.shape[0]
    na = norm1(a)
    hist = []
    for _ in range(rounds + 1):
        ah = q.T @ a @ q
        ah = 0.5 * (ah + ah.T)
        e = ah[k:, :k]
        hist.append(norm1(e) / na)
        if hist[-1] <= tol or len(hist) > rounds:
            break
        x = sla.solve_sylvester(-ah[k:, k:], ah[:k, :k], e)
        u = np.block([[np.eye(k), -x.T], [x, np.eye(n - k)]])
        c = sla.block_diag(_inv_sqrt_spd(np.eye(k) + x.T @ x), _inv_sqrt_spd(np.eye(n - k) + x @ x.T))
        q = q @ u @ c
    return q, ah, hist
