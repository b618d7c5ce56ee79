"""Randomized rank-revealing factorizations (Sec. 2).

* Alg. 1 (RURV): draw G with i.i.d. N(0,1) entries, take V from QR(G), form
  A V^T and factor it, A V^T = U R, so that A = U R V.
* RULV: the same with QL in place of QR (lower-triangular middle factor).
* Alg. 2 (GRURV) for k = 2: the U factor of a rank-revealing factorization of
  A_1^{m_1} A_2^{m_2} without forming inverses or the product.

V is made Haar distributed by moving the signs of R-hat's diagonal into it
(the paper states V is Haar; that holds once those signs are fixed).  The
Gaussian G is an input, so that two implementations can be fed the same draw.
"""
from __future__ import annotations

import numpy as np

from .qr import qr_signed, rq_signed, ql_signed


def haar_from_gaussian(g: np.ndarray) -> np.ndarray:
    """Alg. 1 lines 1-2: V from the QR of the Gaussian G (sign-fixed)."""
    v, _ = qr_signed(g)
    return v


def rurv(a: np.ndarray, g: np.ndarray):
    """Alg. 1: returns (U, R, V) with A = U R V, R upper triangular with a
    non-negative diagonal."""
    v = haar_from_gaussian(g)
    a_hat = a @ v.T
    u, r = qr_signed(a_hat)
    return u, r, v


def rulv(a: np.ndarray, g: np.ndarray):
    """RULV: returns (U, L, V) with A = U L V, L lower triangular with a
    non-negative diagonal."""
    v = haar_from_gaussian(g)
    a_hat = a @ v.T
    u, l_ = ql_signed(a_hat)
    return u, l_, v


def grurv2(a1: np.ndarray, a2: np.ndarray, m1: int, m2: int, g: np.ndarray):
    """Alg. 2 with k = 2: U factor of a rank-revealing factorization of
    A_1^{m_1} A_2^{m_2}.

    Returns (U_current, R1, R2, V) such that
    A_1^{m_1} A_2^{m_2} = U_current R1^{m_1} R2^{m_2} V (the Lemma after Alg. 2).
    """
    assert m1 in (-1, 1) and m2 in (-1, 1)
    if m2 == 1:
        u, r2, v = rurv(a2, g)
    else:
        u, l2, v = rulv(a2.T, g)
        r2 = l2.T
    u_cur = u
    if m1 == 1:
        u1, r1 = qr_signed(a1 @ u_cur)
        u_cur = u1
    else:
        r1, w = rq_signed(u_cur.T @ a1)
        u_cur = w.T
    return u_cur, r1, r2, v
