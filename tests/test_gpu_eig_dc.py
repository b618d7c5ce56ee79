"""Divide-and-conquer (sdc_eig_dc) on the GPU against the oracle and the
construction.

The split points are random, so the two sides' block structures differ; what
is unique is compared: the union of the block spectra (= the spectrum by
construction), and properties every correct result has: blocks of order
<= leaf_max, an exactly block-upper-triangular pair, orthogonal factors and
Q_L^T A Q_R = T up to the dropped coupling blocks (backward error).  The
full-size case is the benchmark workload: the order-2048 pencil, unit circle
first, then recursion to blocks of order <= 64.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import sdc_synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sdc():
    import paper_1011_3077_amd as P
    return P


@pytest.fixture(scope="module")
def handle(sdc):
    h = sdc.Handle(0)
    yield h
    h.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def block_spectrum(t, s, starts):
    ev = []
    for a0, a1 in zip(starts[:-1], starts[1:]):
        if s is None:
            blk = t[a0:a1, a0:a1]
            ev.append(np.linalg.eigvalsh(0.5 * (blk + blk.T)))
        else:
            ev.append(sla.eigvals(t[a0:a1, a0:a1], s[a0:a1, a0:a1]))
    return np.concatenate(ev)


def check_residual(d, a, starts, info, split_tol=1e-10):
    """d = Q_L^T A Q_R - T.  On and above the diagonal blocks T is the exact
    transformation, so d is rounding there (64 n eps |A|_2).  Below them d is
    what the accepted splits set to zero: each level's part is block diagonal
    with blocks E of 1-norm e21 |A_i|_1 <= e21_max sqrt(n) |A|_2 (A_i a
    diagonal block of an orthogonal transformation of A), so the 1-norm of the
    lower part is at most levels sqrt(n) e21_max |A|_2."""
    n = a.shape[0]
    blk = np.zeros(n, dtype=int)
    for i, (a0, a1) in enumerate(zip(starts[:-1], starts[1:])):
        blk[a0:a1] = i
    low = blk[:, None] > blk[None, :]
    na2 = np.linalg.norm(a, 2)
    rnd = 64 * n * np.finfo(float).eps * na2
    assert 0 <= info["e21_max"] <= split_tol
    assert np.linalg.norm(np.where(low, 0.0, d), 2) <= rnd
    bound = info["levels"] * np.sqrt(n) * info["e21_max"] * na2 + rnd
    assert np.abs(np.where(low, d, 0.0)).sum(axis=0).max() <= bound


def check_pencil(res, a, b, lam, leaf, rel_tol):
    st, t, s, ql, qr, starts, info = res
    t, s, ql, qr = (x.cpu().numpy() for x in (t, s, ql, qr))
    n = a.shape[0]
    assert st == 0 and info["unsplit"] == 0
    assert starts[0] == 0 and starts[-1] == n
    assert all(e - s0 <= leaf for s0, e in zip(starts[:-1], starts[1:]))
    for a0, a1 in zip(starts[:-1], starts[1:]):
        assert np.all(t[a1:, a0:a1] == 0) and np.all(s[a1:, a0:a1] == 0)
    eye = np.eye(n)
    assert np.abs(ql.T @ ql - eye).max() <= 1e-12 * np.sqrt(n) * 10
    assert np.abs(qr.T @ qr - eye).max() <= 1e-12 * np.sqrt(n) * 10
    check_residual(ql.T @ a @ qr - t, a, starts, info)
    check_residual(ql.T @ b @ qr - s, b, starts, info)
    got = np.sort_complex(block_spectrum(t, s, starts))
    want = np.sort_complex(lam.astype(complex))
    err = np.max(np.abs(got - want) / np.abs(want))
    assert err <= rel_tol, err
    return got


def test_eig_dc_pencil_matches_oracle(handle, sdc):
    from oracle.eig_dc import eig_dc
    n, leaf = 256, 32
    print("CASE eig_dc pencil", n, flush=True)
    p = S.pencil_problem(n, S.family_seed(1, 7))
    res = handle.eig_dc(dev(p["A"]), dev(p["B"]), leaf_max=leaf, o=sdc.opts(seed=3))
    got = check_pencil(res, p["A"], p["B"], p["lam"], leaf, 1e-10)
    ref = eig_dc(p["A"], p["B"], leaf_max=leaf, seed=3)
    ref_ev = []
    for a0, a1 in ref["blocks"]:
        ref_ev.append(sla.eigvals(ref["T"][a0:a1, a0:a1], ref["S"][a0:a1, a0:a1]))
    ref_ev = np.sort_complex(np.concatenate(ref_ev))
    assert np.max(np.abs(got - ref_ev) / np.abs(ref_ev)) <= 1e-10


def test_eig_dc_symmetric(handle, sdc):
    n, leaf = 300, 40
    print("CASE eig_dc symmetric", n, flush=True)
    a, d, q = S.sym_problem(n, S.family_seed(0, 9))
    st, t, s, ql, qr, starts, info = handle.eig_dc(dev(a), None, leaf_max=leaf, symmetric=True,
                                                    o=sdc.opts(seed=4))
    assert st == 0 and s is None and ql is None and info["unsplit"] == 0
    t, qr = t.cpu().numpy(), qr.cpu().numpy()
    assert all(e - s0 <= leaf for s0, e in zip(starts[:-1], starts[1:]))
    ev = np.sort(block_spectrum(t, None, starts))
    assert np.abs(ev - np.sort(d)).max() <= 1e-12
    assert np.abs(qr.T @ qr - np.eye(n)).max() <= 1e-12
    assert np.linalg.norm(qr.T @ a @ qr - t, 2) <= 1e-11


def _match_max(got, want):
    """Largest distance after greedily pairing each computed eigenvalue with
    the nearest unused one of the construction."""
    want = list(want)
    worst = 0.0
    for z in got:
        j = int(np.argmin([abs(z - w) for w in want]))
        worst = max(worst, abs(z - want.pop(j)))
    return worst


@pytest.mark.parametrize("n,leaf", [(300, 64), (97, 16), (128, 128)])
def test_block_eigvals_symmetric_leaves(handle, sdc, n, leaf):
    """Cyclic Jacobi on the leaves of a symmetric recursion (even and odd
    orders, down to the largest block the kernel takes, 128): each block's
    eigenvalues, ascending, equal the oracle's (LAPACK) on the same T within
    1e-13 |A|_2, and together they are the construction's spectrum."""
    from oracle.eig_dc import block_eigvals
    print("CASE block_eigvals symmetric", n, leaf, flush=True)
    a, d, _ = S.sym_problem(n, S.family_seed(0, 70 + n))
    st, t, s, ql, qr, starts, info = handle.eig_dc(dev(a), None, leaf_max=leaf, symmetric=True,
                                                    o=sdc.opts(seed=8))
    assert st == 0
    wr, wi = handle.block_eigvals(t, None, starts, symmetric=True)
    wr, wi = wr.cpu().numpy(), wi.cpu().numpy()
    ref_r, ref_i = block_eigvals(t.cpu().numpy(), None, starts, True)
    assert np.all(wi == 0.0)
    assert np.abs(wr - ref_r).max() <= 1e-13 * np.abs(d).max()
    assert np.abs(np.sort(wr) - np.sort(d)).max() <= 1e-12


def test_symmetric_eigendecomposition_from_leaves(handle, sdc):
    """eig_dc to blocks <= 64, then the leaves' Jacobi eigenvectors: Z = QR V
    has orthonormal columns, A Z = Z diag(wr) up to the dropped coupling
    blocks, and wr is the construction's spectrum.  A block above the
    eigenvector limit (64) gets NaN vectors but its eigenvalues."""
    n = 300
    print("CASE symmetric eigendecomposition", n, flush=True)
    a, d, _ = S.sym_problem(n, S.family_seed(0, 301))
    st, t, s, ql, qr, starts, info = handle.eig_dc(dev(a), None, leaf_max=64, symmetric=True,
                                                    o=sdc.opts(seed=3))
    assert st == 0
    wr, wi, v = handle.block_eigvals(t, None, starts, symmetric=True, vectors=True)
    z = qr.cpu().numpy() @ v.cpu().numpy()
    wr = wr.cpu().numpy()
    assert np.abs(z.T @ z - np.eye(n)).max() <= 1e-12
    assert np.abs(a @ z - z * wr[None, :]).max() <= 1e-10 * np.abs(d).max()
    assert np.abs(np.sort(wr) - np.sort(d)).max() <= 1e-12
    a2, d2, _ = S.sym_problem(100, S.family_seed(0, 302))
    wr2, _, v2 = handle.block_eigvals(dev(a2), None, [0, 100], symmetric=True, vectors=True)
    assert torch.isnan(v2).all()
    assert np.abs(np.sort(wr2.cpu().numpy()) - np.sort(d2)).max() <= 1e-12


def test_block_eigvals_pencil_to_order_two(handle, sdc):
    """A real normal matrix with complex-conjugate pairs (and one real
    eigenvalue, order 41) as the pencil (A, I), recursed to blocks of order
    <= 2: the closed forms give every eigenvalue (pairs as (re, +-im)) within
    1e-10 relative of the construction (against the smallest modulus: the
    FP64 bar), and match the oracle's on the same blocks."""
    from oracle.eig_dc import block_eigvals
    n = 41
    print("CASE block_eigvals pencil", n, flush=True)
    a, ev = S.normal_random_problem(n, S.family_seed(1, 41))
    b = np.eye(n)
    st, t, s, ql, qr, starts, info = handle.eig_dc(dev(a), dev(b), leaf_max=2, o=sdc.opts(seed=6))
    assert st == 0
    assert all(e - s0 <= 2 for s0, e in zip(starts[:-1], starts[1:])), info
    wr, wi = handle.block_eigvals(t, s, starts, symmetric=False)
    wr, wi = wr.cpu().numpy(), wi.cpu().numpy()
    got = wr + 1j * wi
    assert _match_max(got, ev) <= 1e-10 * np.abs(ev).min()
    ref_r, ref_i = block_eigvals(t.cpu().numpy(), s.cpu().numpy(), starts, False)
    assert np.abs(got - (ref_r + 1j * ref_i)).max() <= 1e-11


def test_block_eigvals_edges(handle, sdc):
    """A symmetric block above the Jacobi limit and a pencil block above
    the dense pencil solver's limit (64) give NaN, while the block after it
    gets its eigenvalues; inconsistent block starts are rejected."""
    print("CASE block_eigvals edges", flush=True)
    a, d, _ = S.sym_problem(129, S.family_seed(0, 129))
    A = dev(a)
    wr, wi = handle.block_eigvals(A, None, [0, 129], symmetric=True)
    assert torch.isnan(wr).all() and torch.isnan(wi).all()
    wr, wi = handle.block_eigvals(A[:5, :5].contiguous(), None, [0, 1, 5], symmetric=True)
    ref_r, _ = __import__("oracle.eig_dc", fromlist=["block_eigvals"]).block_eigvals(a[:5, :5], None, [0, 1, 5], True)
    assert np.abs(wr.cpu().numpy() - ref_r).max() <= 1e-14
    p = S.pencil_problem(70, S.family_seed(1, 70))
    wr, wi = handle.block_eigvals(dev(p["A"]), dev(p["B"]), [0, 65, 70], symmetric=False)
    assert torch.isnan(wr[:65]).all() and torch.isnan(wi[:65]).all()
    assert torch.isfinite(wr[65:]).all() and torch.isfinite(wi[65:]).all()
    with pytest.raises(sdc.SdcError):
        handle.block_eigvals(A, None, [0, 100], symmetric=True)
    with pytest.raises(sdc.SdcError):
        handle.block_eigvals(A, None, [0, 64, 64, 129], symmetric=True)


def test_eig_dc_benchmark_workload_full_size(handle, sdc):
    """Order-2048 pencil of the benchmark: unit circle, then blocks <= 64."""
    n, leaf = 2048, 64
    print("CASE eig_dc full size", n, flush=True)
    p = S.pencil_problem(n, S.family_seed(1))
    res = handle.eig_dc(dev(p["A"]), dev(p["B"]), leaf_max=leaf, o=sdc.opts(seed=1))
    check_pencil(res, p["A"], p["B"], p["lam"], leaf, 1e-10)
    info = res[-1]
    print("full-size info", info, flush=True)


def test_block_eigvals_all_order_one_blocks(handle, sdc):
    """Every block of order 1: the symmetric eigenvalues are the diagonal
    (V the identity), the pencil's are T_ii / S_ii."""
    print("CASE block_eigvals 1x1", flush=True)
    n = 9
    rng = np.random.default_rng(5)
    t = np.triu(rng.standard_normal((n, n)))
    s = np.triu(rng.standard_normal((n, n))) + 4 * np.eye(n)
    starts = list(range(n + 1))
    wr, wi, v = handle.block_eigvals(dev(np.diag(np.diag(t))), None, starts, symmetric=True, vectors=True)
    assert np.array_equal(wr.cpu().numpy(), np.diag(t)) and np.array_equal(v.cpu().numpy(), np.eye(n))
    wr, wi = handle.block_eigvals(dev(t), dev(s), starts, symmetric=False)
    assert np.allclose(wr.cpu().numpy(), np.diag(t) / np.diag(s), rtol=1e-15, atol=0)
    assert not wi.cpu().numpy().any()


def test_multiway_split_separates_a_repeated_eigenvalue(handle, sdc):
    """A five-fold eigenvalue of a symmetric matrix: no line separates equal
    eigenvalues, but the step that isolates their invariant subspace leaves
    every coupling block inside it negligible, and the library (like the
    oracle) divides there too, down to blocks of order 1."""
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_eig_dc import repeated_eig_problem
    from oracle.eig_dc import eig_dc
    print("CASE multiway", flush=True)
    a, d = repeated_eig_problem(30, 11)
    st, t, s, ql, qr, starts, info = handle.eig_dc(dev(a), None, leaf_max=1, symmetric=True, o=sdc.opts(seed=2))
    assert st == 0 and info["unsplit"] == 0 and info["extra_splits"] >= 4, info
    assert starts == list(range(31))
    t, qr = t.cpu().numpy(), qr.cpu().numpy()
    assert np.abs(np.sort(np.diag(t)) - np.sort(d)).max() <= 1e-12
    assert np.abs(qr.T @ a @ qr - t).max() <= 1e-10
    ref = eig_dc(a, symmetric=True, leaf_max=1, seed=2)
    assert ref["extra_splits"] >= 4 and np.abs(np.sort(np.diag(ref["T"])) - np.sort(np.diag(t))).max() <= 1e-12


def test_pencil_benchmark_workload_to_order_two_leaves(handle, sdc):
    """The order-2048 benchmark pencil recursed to blocks of order <= 2 and
    every eigenvalue taken from the leaves (closed forms): the construction's
    spectrum within 1e-10 relative, no block left unsplit."""
    n = 2048
    print("CASE eig_dc to order-2 leaves", n, flush=True)
    p = S.pencil_problem(n, S.family_seed(1))
    st, t, s, ql, qr, starts, info = handle.eig_dc(dev(p["A"]), dev(p["B"]), leaf_max=2, o=sdc.opts(seed=1),
                                                    factors=False)
    print("info", {k: v for k, v in info.items() if k != "bounds"}, flush=True)
    assert st == 0 and info["unsplit"] == 0 and info["near_singular"] == 0
    assert all(e - s0 <= 2 for s0, e in zip(starts[:-1], starts[1:]))
    wr, wi = handle.block_eigvals(t, s, starts, symmetric=False)
    got = np.sort_complex((wr + 1j * wi).cpu().numpy())
    want = np.sort_complex(p["lam"].astype(complex))
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-10
