"""Pins of the oracle's divide-and-conquer (Sec. 3.3-3.5): the block spectra
equal the construction's eigenvalues, every block is at most leaf_max, the pair
is block upper triangular and orthogonally equivalent to the input up to the
dropped coupling blocks."""
import numpy as np
import pytest
import scipy.linalg as sla

import sdc_synth as S
from oracle.eig_dc import eig_dc


def _block_spectrum(t, s, blocks):
    ev = []
    for a0, a1 in blocks:
        if s is None:
            ev.append(np.linalg.eigvalsh(0.5 * (t[a0:a1, a0:a1] + t[a0:a1, a0:a1].T)))
        else:
            ev.append(sla.eigvals(t[a0:a1, a0:a1], s[a0:a1, a0:a1]))
    return np.concatenate(ev)


@pytest.mark.parametrize("n,leaf", [(60, 16), (128, 32)])
def test_eig_dc_symmetric(n, leaf):
    a, d, q = S.sym_problem(n, 50 + n)
    r = eig_dc(a, symmetric=True, leaf_max=leaf, seed=1)
    assert r["unsplit"] == 0
    assert all(e - s <= leaf for s, e in r["blocks"])
    assert r["blocks"][0][0] == 0 and r["blocks"][-1][1] == n
    ev = np.sort(_block_spectrum(r["T"], None, r["blocks"]))
    assert np.abs(ev - np.sort(d)).max() <= 1e-12
    qq = r["QR"]
    assert np.allclose(qq.T @ qq, np.eye(n), atol=1e-12)
    # T is block diagonal and Q^T A Q equals it up to the dropped couplings
    assert np.linalg.norm(qq.T @ a @ qq - r["T"], 2) <= 1e-11


@pytest.mark.parametrize("n,leaf", [(64, 16), (160, 32)])
def test_eig_dc_pencil(n, leaf):
    p = S.pencil_problem(n, 70 + n)
    r = eig_dc(p["A"], p["B"], leaf_max=leaf, seed=2)
    assert r["unsplit"] == 0
    assert all(e - s <= leaf for s, e in r["blocks"])
    t, s_ = r["T"], r["S"]
    for a0, a1 in r["blocks"]:
        assert np.all(t[a1:, a0:a1] == 0) and np.all(s_[a1:, a0:a1] == 0)
    got = np.sort_complex(_block_spectrum(t, s_, r["blocks"]))
    want = np.sort_complex(p["lam"].astype(complex))
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-10
    ql, qr = r["QL"], r["QR"]
    assert np.allclose(ql.T @ ql, np.eye(n), atol=1e-12) and np.allclose(qr.T @ qr, np.eye(n), atol=1e-12)
    assert np.linalg.norm(ql.T @ p["A"] @ qr - t, 2) <= 1e-10 * np.linalg.norm(p["A"], 2)
    assert np.linalg.norm(ql.T @ p["B"] @ qr - s_, 2) <= 1e-10 * np.linalg.norm(p["B"], 2)


# ---------------------------------------------------------------------------
# block_eigvals: the dense method at the leaves, pinned to constructions
# ---------------------------------------------------------------------------

def _haar(n, rng):
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))


def test_block_eigvals_symmetric_blocks_recover_construction():
    from oracle.eig_dc import block_eigvals
    rng = np.random.default_rng(11)
    sizes = [1, 5, 64, 7, 2]
    n = sum(sizes)
    t = np.zeros((n, n))
    starts, want = [0], []
    for m in sizes:
        s0 = starts[-1]
        d = rng.uniform(-2, 2, size=m)
        q = _haar(m, rng)
        t[s0:s0 + m, s0:s0 + m] = q @ np.diag(d) @ q.T
        starts.append(s0 + m)
        want.append(np.sort(d))
    wr, wi = block_eigvals(t, None, starts, True)
    assert np.all(wi == 0.0)
    for (a0, a1), w in zip(zip(starts[:-1], starts[1:]), want):
        assert np.all(np.diff(wr[a0:a1]) >= 0)
        assert np.max(np.abs(wr[a0:a1] - w)) <= 1e-13


def test_block_eigvals_pencil_order_one_and_two_blocks():
    """Closed forms: a 1x1 pair gives T/S; a 2x2 pair T = S X with X similar
    to [[x, y], [-y, x]] gives x +- iy, and with X similar to diag(l1, l2)
    gives l1, l2 (ascending).  Coupling entries above the blocks are ignored."""
    from oracle.eig_dc import block_eigvals
    rng = np.random.default_rng(12)
    n = 5
    t = np.triu(rng.standard_normal((n, n)))
    s = np.triu(rng.standard_normal((n, n))) + 3 * np.eye(n)
    # block 0: 1x1
    t[0, 0], s[0, 0] = 3.0, -1.5
    # block 1: complex pair 0.3 +- 1.7i
    r = rng.standard_normal((2, 2)) + 2 * np.eye(2)
    x = r @ np.array([[0.3, 1.7], [-1.7, 0.3]]) @ np.linalg.inv(r)
    sb = rng.standard_normal((2, 2)) + 2 * np.eye(2)
    s[1:3, 1:3], t[1:3, 1:3] = sb, sb @ x
    s[2, 1] = sb[1, 0]
    t[2, 1] = (sb @ x)[1, 0]
    # block 2: real pair 2.5, -0.75
    r = rng.standard_normal((2, 2)) + 2 * np.eye(2)
    x = r @ np.diag([2.5, -0.75]) @ np.linalg.inv(r)
    sb = rng.standard_normal((2, 2)) + 2 * np.eye(2)
    s[3:5, 3:5], t[3:5, 3:5] = sb, sb @ x
    wr, wi = block_eigvals(t, s, [0, 1, 3, 5], False)
    assert abs(wr[0] - (-2.0)) <= 1e-14 and wi[0] == 0.0
    assert np.allclose(wr[1:3], [0.3, 0.3], atol=1e-12) and np.allclose(wi[1:3], [1.7, -1.7], atol=1e-12)
    assert np.allclose(wr[3:5], [-0.75, 2.5], atol=1e-12) and np.all(wi[3:5] == 0.0)


def test_block_eigvals_after_eig_dc_give_the_spectrum():
    """End to end on the CPU: the recursion to blocks <= 8, then the leaves'
    eigenvalues, is the construction's spectrum."""
    from oracle.eig_dc import block_eigvals
    a, d, _ = S.sym_problem(48, S.family_seed(0, 5))
    r = eig_dc(a, symmetric=True, leaf_max=8, seed=4)
    starts = [b[0] for b in r["blocks"]] + [48]
    wr, _ = block_eigvals(r["T"], None, starts, True)
    assert np.max(np.abs(np.sort(wr) - np.sort(d))) <= 1e-12


# ---------------------------------------------------------------------------
# The pencil search of Sec. 3.5: circles 2^{-+2^k} down (up) to the smallest
# (largest) bounding circle, then lines; the reciprocal pair after a swap
# ---------------------------------------------------------------------------

def _check_bounds(r, tol=1e-9):
    """Every block's eigenvalues (reciprocals when inverted) lie in its bound."""
    for (a0, a1), (lo, hi, rad, inv) in zip(r["blocks"], r["bounds"]):
        ev = sla.eigvals(r["T"][a0:a1, a0:a1], r["S"][a0:a1, a0:a1])
        mu = 1.0 / ev if inv else ev
        assert np.all(mu.real >= lo - tol) and np.all(mu.real <= hi + tol), ((a0, a1), (lo, hi), mu)
        assert np.all(np.abs(mu) <= rad * (1 + tol)), ((a0, a1), rad, mu)


@pytest.mark.parametrize("lo,hi,radii,statuses", [
    # all inside the unit circle: 1, 1/2 (still all inside), 1/4 splits
    (0.02, 0.4, [1.0, 0.5, 0.25], [2, 2, 0]),
    # all outside: 1, 2 (still all outside), 4 splits
    (2.5, 50.0, [1.0, 2.0, 4.0], [2, 2, 0]),
    # inside 1 but outside 1/2: the smallest bounding circle is 1; lines inside it
    (0.55, 0.95, [1.0, 0.5], [2, 2]),
    # outside 1 but inside 2: the largest circle with all outside is 1; swap, lines
    (1.1, 1.9, [1.0, 2.0], [2, 2]),
])
def test_circle_search_stops_at_the_bounding_circle(lo, hi, radii, statuses):
    """The radius sequence of Sec. 3.5 for spectra entirely inside or outside
    the unit circle: it runs 2^{-2^k} (2^{2^k}) only until a circle splits the
    spectrum or finds it all on the other side, and never turns around; the
    block spectra are the construction's and every block lies in its bound."""
    p = S.pencil_problem(40, 91, lam_lo=lo, lam_hi=hi)
    r = eig_dc(p["A"], p["B"], leaf_max=8, seed=5)
    circ = [x for x in r["log"] if x[2] == "circle"]
    assert [x[3] for x in circ] == radii
    assert [x[4] for x in circ] == statuses
    assert r["unsplit"] == 0 and r["near_singular"] == 0
    got = np.sort_complex(_block_spectrum(r["T"], r["S"], r["blocks"]))
    want = np.sort_complex(p["lam"].astype(complex))
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-12
    _check_bounds(r)


def test_singular_pencil_is_flagged_near_singular():
    """A pencil with a common null vector of A and B (det(A - lambda B) = 0 for
    every lambda) meets the pseudospectrum on every curve (Sec. 3.5): the
    repeated squaring never converges, the block is given up after a few
    circles, returned whole with no bound, and flagged."""
    p = S.pencil_problem(24, 77)
    t, s = p["T"].copy(), p["S"].copy()
    t[3, 3] = s[3, 3] = 0.0
    a, b = p["U"] @ t @ p["V"].T, p["U"] @ s @ p["V"].T
    r = eig_dc(a, b, leaf_max=4, seed=3)
    assert r["near_singular"] == 1 and r["unsplit"] == 1
    assert r["blocks"] == [(0, 24)] and r["bounds"][0][2] == np.inf
    assert all(x[2] == "circle" and x[4] == 1 for x in r["log"])  # NOT_CONVERGED on every circle


def test_jordan_block_is_returned_unsplit_with_a_bound():
    """E4's matrix (a 16 x 16 Jordan block at 0.1 among random eigenvalues,
    Sec. 5): lines through the Jordan block's pseudospectrum cannot split it,
    so it comes back as one unsplit block (Sec. 3.6) whose bound holds its
    eigenvalues; it is not a singular pencil (B = I)."""
    n = 32
    a = S.jordan_problem(n, S.family_seed(7, 4))
    r = eig_dc(a, np.eye(n), leaf_max=2, seed=3)
    assert r["near_singular"] == 0 and r["unsplit"] >= 1
    blk = [(b, bd) for b, bd, u in zip(r["blocks"], r["bounds"], r["unsplit_blocks"]) if u]
    assert len(blk) == 1
    (a0, a1), (lo, hi, rad, inv) = blk[0]
    assert a1 - a0 >= 16 and inv == 0 and lo < 0.1 < hi
    _check_bounds(r, tol=1e-6)


# ---------------------------------------------------------------------------
# Multi-way splits (the remark after Alg. 4): a step that leaves several small
# coupling blocks divides its block at all of them
# ---------------------------------------------------------------------------

def repeated_eig_problem(n, seed, mult=5, value=0.7):
    """Symmetric A = Q diag(d) Q^T with a `mult`-fold eigenvalue `value`
    (no curve can separate equal eigenvalues) among n - mult others spread
    over [-1, 1] away from it."""
    rng = np.random.default_rng(seed)
    others = rng.uniform(-1.0, 0.5, n - mult)
    d = np.concatenate([np.full(mult, value), others])
    q = S.haar_orthogonal(n, rng)
    a = (q * d[None, :]) @ q.T
    return 0.5 * (a + a.T), d


def test_multiway_split_separates_a_repeated_eigenvalue_symmetric():
    """Recursion to blocks of order 1: the five equal eigenvalues cannot be
    split by any line, but once a split isolates their invariant subspace
    its block is 0.7 I up to rounding, every coupling block inside it is
    negligible, and the step divides it into blocks of order 1."""
    a, d = repeated_eig_problem(30, 11)
    r = eig_dc(a, symmetric=True, leaf_max=1, seed=2)
    assert r["unsplit"] == 0 and r["extra_splits"] >= 4
    assert all(e - s0 == 1 for s0, e in r["blocks"])
    ev = np.sort(np.diag(r["T"]))
    assert np.abs(ev - np.sort(d)).max() <= 1e-12
    assert np.abs(r["QR"].T @ a @ r["QR"] - r["T"]).max() <= 1e-10


def test_no_extra_splits_for_distinct_eigenvalues():
    """Random bases inside each side leave no other small coupling block:
    with distinct eigenvalues every step divides in two."""
    a, d, _ = S.sym_problem(40, S.family_seed(0, 41))
    r = eig_dc(a, symmetric=True, leaf_max=4, seed=1)
    assert r["extra_splits"] == 0
