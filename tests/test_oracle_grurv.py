"""Pins of the oracle's randomized rank-revealing factorizations (Sec. 2).

* The Lemma after Alg. 2: GRURV returns the same factorization as QR of the
  explicitly formed product A_1^{m_1} A_2^{m_2} V^T (all four sign patterns;
  explicit inverses appear in the test only).  With every triangular factor
  normalized to a non-negative diagonal the QR is unique, so U_current and
  R1^{m1} R2^{m2} must match that QR exactly (up to rounding).
* Thm 2.1 (RURV is a strong rank-revealing factorization): statistical check
  over many draws.  The theorem's constants c1, c3 are not given in the paper,
  so the bounds below use generous constants: parity unpinned for the constants,
  pinned only for the n-scaling.
"""
import numpy as np
import pytest

from oracle.qr import qr_signed
from oracle.rurv import grurv2, rurv, rulv, haar_from_gaussian


def _pow(m, e):
    return m if e == 1 else np.linalg.inv(m)


@pytest.mark.parametrize("m1,m2", [(1, 1), (1, -1), (-1, 1), (-1, -1)])
@pytest.mark.parametrize("seed", [1, 2])
def test_grurv_equals_qr_of_explicit_product(m1, m2, seed):
    rng = np.random.default_rng(seed * 10 + (m1 + 1) + (m2 + 1) // 2)
    n = 10
    a1 = rng.standard_normal((n, n)) + 3 * np.eye(n)
    a2 = rng.standard_normal((n, n)) + 3 * np.eye(n)
    g = rng.standard_normal((n, n))
    u, r1, r2, v = grurv2(a1, a2, m1, m2, g)
    prod = _pow(a1, m1) @ _pow(a2, m2)
    assert np.allclose(u @ _pow(r1, m1) @ _pow(r2, m2) @ v, prod, atol=1e-11 * np.abs(prod).max())
    q_ref, r_ref = qr_signed(prod @ v.T)
    assert np.allclose(u, q_ref, atol=1e-10)
    assert np.allclose(_pow(r1, m1) @ _pow(r2, m2), r_ref, atol=1e-10 * np.abs(r_ref).max())


def test_haar_v_is_orthogonal_and_sign_fixed():
    rng = np.random.default_rng(3)
    g = rng.standard_normal((20, 20))
    v = haar_from_gaussian(g)
    assert np.allclose(v.T @ v, np.eye(20), atol=1e-14)
    # V^T G is upper triangular with a positive diagonal (the sign fix)
    r = v.T @ g
    assert np.allclose(np.tril(r, -1), 0, atol=1e-12)
    assert np.all(np.diag(r) > 0)


def test_rurv_and_rulv_reconstruct():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((15, 15))
    g = rng.standard_normal((15, 15))
    u, r, v = rurv(a, g)
    assert np.allclose(u @ r @ v, a, atol=1e-13 * 15)
    assert np.allclose(np.tril(r, -1), 0)
    u, l_, v = rulv(a, g)
    assert np.allclose(u @ l_ @ v, a, atol=1e-13 * 15)
    assert np.allclose(np.triu(l_, 1), 0)


@pytest.mark.slow
def test_rurv_strong_rank_revealing_statistics():
    """Thm 2.1 on a matrix with a large gap at r: over 60 draws, the scaled
    quantities sigma_min(R11) sqrt(r(n-r))/sigma_r and
    ||R11^{-1} R12|| / sqrt(r(n-r)) stay O(1) (generous constants)."""
    rng = np.random.default_rng(5)
    n, r = 60, 20
    u0, _ = np.linalg.qr(rng.standard_normal((n, n)))
    w0, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sig = np.concatenate([np.linspace(1.0, 0.5, r), np.full(n - r, 1e-12)])
    a = u0 @ np.diag(sig) @ w0.T
    lows, highs = [], []
    for t in range(60):
        _, rr, _ = rurv(a, rng.standard_normal((n, n)))
        r11, r12 = rr[:r, :r], rr[:r, r:]
        smin = np.linalg.svd(r11, compute_uv=False)[-1]
        lows.append(smin * np.sqrt(r * (n - r)) / sig[r - 1])
        highs.append(np.linalg.norm(np.linalg.solve(r11, r12), 2) / np.sqrt(r * (n - r)))
        assert smin <= np.sqrt(2) * sig[r - 1] * (1 + 1e-12)
        assert np.linalg.svd(rr[r:, r:], compute_uv=False)[0] >= sig[r] * (1 - 1e-6)
    assert np.median(lows) > 0.05
    assert np.median(highs) < 5.0
