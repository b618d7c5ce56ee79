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
