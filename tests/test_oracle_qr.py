"""Pins of the oracle's orthogonal-triangular factorizations.

The pure-loop Householder QR and the LAPACK path are independent
implementations; with the triangular factor normalized to a non-negative
diagonal the factorization of a full-rank matrix is unique, so they must agree.
RQ and QL (built by reversal) are checked against SciPy's own RQ routine and
against their defining properties.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.qr import householder_qr_loop, qr_signed, rq_signed, ql_signed


@pytest.mark.parametrize("shape", [(8, 8), (20, 7), (40, 40), (64, 32), (33, 17)])
def test_loop_householder_matches_lapack(shape):
    rng = np.random.default_rng(1 + shape[0] * 100 + shape[1])
    m = rng.standard_normal(shape)
    q, r = householder_qr_loop(m)
    assert np.allclose(q @ r, m, atol=1e-13 * np.abs(m).max())
    assert np.allclose(q.T @ q, np.eye(shape[0]), atol=1e-14 * shape[0])
    assert np.allclose(np.tril(r, -1), 0.0)
    # sign-normalize the loop result and compare with the LAPACK path
    k = min(shape)
    s = np.sign(np.diag(r)[:k])
    s[s == 0] = 1
    r_loop = r.copy()
    r_loop[:k] *= s[:, None]
    q2, r2 = qr_signed(m)
    assert np.allclose(r_loop[:k], r2[:k], rtol=0, atol=1e-12 * np.abs(m).max())
    assert np.allclose(q[:, :k] * s[None, :], q2[:, :k], atol=1e-12)


def test_qr_signed_diagonal_nonnegative_and_reconstructs():
    rng = np.random.default_rng(7)
    m = rng.standard_normal((50, 30))
    q, r = qr_signed(m)
    assert np.all(np.diag(r) >= 0)
    assert np.allclose(q @ r, m, atol=1e-13)
    assert np.allclose(q.T @ q, np.eye(50), atol=1e-13)


@pytest.mark.parametrize("n", [5, 16, 31])
def test_rq_by_reversal_matches_scipy_rq(n):
    rng = np.random.default_rng(100 + n)
    x = rng.standard_normal((n, n))
    r, w = rq_signed(x)
    assert np.allclose(r @ w, x, atol=1e-13 * n)
    assert np.allclose(np.tril(r, -1), 0.0)
    assert np.all(np.diag(r) >= 0)
    r_s, w_s = sla.rq(x)
    s = np.sign(np.diag(r_s))
    # X = R W = (R D)(D W) with D = diag(s): normalize SciPy's factors alike
    r_s = r_s * s[None, :]
    w_s = s[:, None] * w_s
    assert np.allclose(r, r_s, atol=1e-12 * n)
    assert np.allclose(w, w_s, atol=1e-12 * n)


@pytest.mark.parametrize("n", [6, 17, 32])
def test_ql_by_reversal_is_an_rq_of_the_transpose(n):
    """X = Q L  <=>  X^T = L^T Q^T, an RQ factorization of X^T: compare with
    SciPy's RQ (normalized to a non-negative diagonal)."""
    rng = np.random.default_rng(200 + n)
    x = rng.standard_normal((n, n))
    q, l_ = ql_signed(x)
    assert np.allclose(q @ l_, x, atol=1e-13 * n)
    assert np.allclose(np.triu(l_, 1), 0.0)
    assert np.all(np.diag(l_) >= 0)
    assert np.allclose(q.T @ q, np.eye(n), atol=1e-13 * n)
    r_s, w_s = sla.rq(x.T)
    s = np.sign(np.diag(r_s))
    r_s = r_s * s[None, :]
    w_s = s[:, None] * w_s
    assert np.allclose(l_.T, r_s, atol=1e-12 * n)
    assert np.allclose(q.T, w_s, atol=1e-12 * n)
