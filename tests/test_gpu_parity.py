"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

What is compared, and why (the method's outputs are partly non-unique):
* IRS: the iteration count p, the last R_j (unique once its diagonal is made
  non-negative: the Cholesky factor of A_j^T A_j + B_j^T B_j), and the Gram
  invariants A_p^T A_p, B_p^T B_p, A_p^T B_p (the iterates themselves are only
  defined up to a common left orthogonal factor).
* split: k, n_inside and p exactly; the leading k columns of Q (Q_R, Q_L),
  which are unique given the same Gaussian draw, elementwise; A11 elementwise;
  the trailing subspace and the eigenvalues of both diagonal blocks; E21 / F21.
Tolerances follow FP64 backward stability: errors of order eps * growth on
matrices of norm O(1); every bound is stated in the test.
"""
import math

import numpy as np
import pytest

import sdc_synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HALF0 = {"kind": "halfplane", "shift": 0.0, "scale": 1.0}


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


def host(t):
    return t.detach().cpu().numpy()


def norm1(x):
    return float(np.max(np.sum(np.abs(x), axis=0)))


def sin_theta(x, y):
    qx, _ = np.linalg.qr(x)
    qy, _ = np.linalg.qr(y)
    return float(np.linalg.norm(qy - qx @ (qx.T @ qy), 2))


def gauss_stack(n, seed, attempts=3):
    """(attempt, side) Gaussians in the layout opts.G expects."""
    gs = []
    for a in range(attempts):
        for side in range(2):
            gs.append(S.gaussian(n, seed + 10 * a + side))
    # column-major n x n blocks, contiguous: block b occupies [b*n*n, (b+1)*n*n)
    flat = np.concatenate([g.ravel(order="F") for g in gs])
    return gs, dev(flat)


def oracle_gauss(gs):
    return lambda n, attempt, side: gs[2 * attempt + side]


def print_case(**kw):
    print("CASE", kw, flush=True)


# ---------------------------------------------------------------------------
def test_device_gaussian_matches_oracle_philox(handle):
    from oracle.philox import gaussian_matrix
    for n, seed, tag in ((7, 0, 0), (64, 123, 1), (200, 2**40 + 5, 0)):
        print_case(test="gaussian", n=n, seed=seed, tag=tag)
        g = host(handle.gaussian(n, seed, tag))
        ref = gaussian_matrix(n, seed, tag)
        assert np.allclose(g, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 8, 33, 96, 128, 300, 700])
def test_irs_matches_oracle_symmetric(handle, sdc, n):
    import oracle as O
    from oracle.split import premap
    print_case(test="irs_sym", n=n)
    a, d, q = S.sym_problem(n, S.family_seed(0, n))
    st, ap, bp, r, p, rc = handle.irs(dev(a), None, sdc.region("halfplane", shift=0.0, scale=1.0))
    ap, bp, r = host(ap), host(bp), host(r)
    a0, b0 = premap(a, np.eye(n), HALF0)
    ref = O.irs(a0, b0, record=True)
    assert st == sdc.SDC_OK and ref.converged
    assert p == ref.p
    rr = ref.R_history[-1]
    assert np.abs(r - rr).max() <= 1e-11 * np.abs(rr).max()
    for x, y in ((ap.T @ ap, ref.A.T @ ref.A), (bp.T @ bp, ref.B.T @ ref.B), (ap.T @ bp, ref.A.T @ ref.B)):
        assert np.abs(x - y).max() <= 1e-10 * max(1.0, np.abs(y).max())


@pytest.mark.parametrize("n,transpose", [(16, 0), (48, 1), (257, 0), (300, 1)])
def test_irs_matches_oracle_pencil(handle, sdc, n, transpose):
    import oracle as O
    print_case(test="irs_pencil", n=n, transpose=transpose)
    pb = S.pencil_problem(n, S.family_seed(1, n))
    a, b = pb["A"], pb["B"]
    st, ap, bp, r, p, rc = handle.irs(dev(a), dev(b), sdc.region(), transpose=bool(transpose))
    ap, bp, r = host(ap), host(bp), host(r)
    ref = O.irs(a.T if transpose else a, b.T if transpose else b, record=True)
    assert st == sdc.SDC_OK and ref.converged and p == ref.p
    rr = ref.R_history[-1]
    assert np.abs(r - rr).max() <= 1e-10 * np.abs(rr).max()
    for x, y in ((ap.T @ ap, ref.A.T @ ref.A), (bp.T @ bp, ref.B.T @ ref.B), (ap.T @ bp, ref.A.T @ ref.B)):
        assert np.abs(x - y).max() <= 1e-9 * max(1.0, np.abs(y).max())


@pytest.mark.parametrize("n", [2, 5, 32, 65, 128, 300])
def test_split_sym_matches_oracle(handle, sdc, n):
    import oracle as O
    print_case(test="split_sym", n=n)
    seed = S.family_seed(0, 100 + n)
    a, d, q = S.sym_problem(n, seed)
    gs, gdev = gauss_stack(n, seed)
    res = handle.split_sym(dev(a), sdc.region("halfplane", shift=0.0, scale=1.0), sdc.opts(G=gdev, diagnostics=1))
    ref = O.split_sym(a, HALF0, gauss=oracle_gauss(gs))
    info = res.info
    assert res.status == ref.status == sdc.SDC_OK
    k = info["k_lead"]
    assert k == ref.k and info["n_inside"] == int((d < 0).sum())
    assert info["iters_right"] == ref.p_right
    assert info["attempts"] == ref.attempts
    Q, Ah = host(res.Q), host(res.Ahat)
    assert np.abs(Q[:, :k] - ref.Q[:, :k]).max() <= 1e-10
    assert np.abs(Ah[:k, :k] - ref.A_hat[:k, :k]).max() <= 1e-10 * norm1(a)
    assert sin_theta(Q[:, k:], ref.Q[:, k:]) <= 1e-10
    assert info["e21_rel"] <= 1e-12 and abs(info["e21_rel"] - ref.e) <= 1e-12
    assert norm1(Ah[k:, :k]) <= 1e-12 * norm1(a)
    assert info["orth_err"] <= 1e-13 * n
    ev = np.sort(np.concatenate([np.linalg.eigvalsh(Ah[:k, :k]), np.linalg.eigvalsh(Ah[k:, k:])]))
    assert np.abs(ev - np.sort(d)).max() <= 1e-12


@pytest.mark.parametrize("n", [24, 48, 150, 300])
def test_split_pencil_matches_oracle(handle, sdc, n):
    import oracle as O
    import scipy.linalg as sla
    print_case(test="split_pencil", n=n)
    seed = S.family_seed(1, 200 + n)
    pb = S.pencil_problem(n, seed)
    a, b, lam = pb["A"], pb["B"], pb["lam"]
    gs, gdev = gauss_stack(n, seed)
    res = handle.split_pencil(dev(a), dev(b), sdc.region(), sdc.opts(G=gdev, diagnostics=1))
    ref = O.split_pencil(a, b, {"kind": "unit_disk"}, gauss=oracle_gauss(gs))
    info = res.info
    assert res.status == ref.status == sdc.SDC_OK
    k = info["k_lead"]
    assert k == ref.k and info["n_inside"] == int((np.abs(lam) < 1).sum())
    assert info["iters_right"] == ref.p_right and info["iters_left"] == ref.p_left
    QR, QL, Ah, Bh = host(res.Q), host(res.QL), host(res.Ahat), host(res.Bhat)
    assert np.abs(QR[:, :k] - ref.Q[:, :k]).max() <= 1e-9
    assert np.abs(QL[:, :k] - ref.QL[:, :k]).max() <= 1e-9
    assert sin_theta(QR[:, k:], ref.Q[:, k:]) <= 1e-9
    assert sin_theta(QL[:, k:], ref.QL[:, k:]) <= 1e-9
    assert np.abs(Ah[:k, :k] - ref.A_hat[:k, :k]).max() <= 1e-9 * norm1(a)
    assert info["e21_rel"] <= 1e-11 and abs(info["e21_rel"] - ref.e) <= 1e-11
    ev_out = sla.eigvals(Ah[:k, :k], Bh[:k, :k])
    ev_in = sla.eigvals(Ah[k:, k:], Bh[k:, k:])
    assert np.all(np.abs(ev_out) > 1) and np.all(np.abs(ev_in) < 1)
    got = np.sort_complex(np.concatenate([ev_out, ev_in]))
    want = np.sort_complex(lam.astype(complex))
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-10


def test_batched_equals_single_calls(handle, sdc):
    """Each problem's result is bitwise the same alone and in a batch of
    uneven sizes (per-problem seeds, per-problem kernels)."""
    sizes = [32, 77, 128, 45, 200, 64]
    mats = [S.sym_problem(n, S.family_seed(2, i))[0] for i, n in enumerate(sizes)]
    regs = [sdc.region("halfplane", shift=0.0, scale=1.0) for _ in sizes]
    print_case(test="batched", sizes=sizes)
    o = sdc.opts(seed=77)
    batch = handle.split_sym_batched([dev(m) for m in mats], regs, o)
    for i, (m, r) in enumerate(zip(mats, batch)):
        single = handle.split_sym(dev(m), regs[i], sdc.opts(seed=77 + i * 1000003))
        assert r.status == single.status == sdc.SDC_OK
        assert r.info["k_lead"] == single.info["k_lead"]
        assert torch.equal(r.Q, single.Q) and torch.equal(r.Ahat, single.Ahat)


@pytest.mark.parametrize("lookahead", [0, 1200])
def test_batched_mixed_with_lookahead_size_equals_single(sdc, lookahead):
    """A batch that mixes a problem large enough for the look-ahead schedule
    (two streams, when the handle enables it from 1200 factored columns)
    with small ones that take the wide update, and, with the default
    one-stream schedule, a problem of three tree levels with ones of one
    and two: each result is still bitwise the one of a single call, since
    the kernel that updates a column is chosen from its own problem's shape
    and the handle."""
    sizes = [1300, 100, 300]
    mats = [S.sym_problem(n, S.family_seed(2, 40 + i))[0] for i, n in enumerate(sizes)]
    regs = [sdc.region("halfplane", shift=0.0, scale=1.0) for _ in sizes]
    print_case(test="batched_mixed_lookahead", sizes=sizes, lookahead=lookahead)
    h = sdc.Handle(0)
    try:
        h.lookahead_set(lookahead)
        batch = h.split_sym_batched([dev(m) for m in mats], regs, sdc.opts(seed=91))
        for i, (m, r) in enumerate(zip(mats, batch)):
            single = h.split_sym(dev(m), regs[i], sdc.opts(seed=91 + i * 1000003))
            assert r.status == single.status == sdc.SDC_OK
            assert r.info["k_lead"] == single.info["k_lead"]
            assert torch.equal(r.Q, single.Q) and torch.equal(r.Ahat, single.Ahat)
    finally:
        h.close()


def test_batched_many_equal_sizes(handle, sdc):
    """64 problems of order 128 (the sym128 recipe, per-problem seeds) in one
    batched FP64 call: every split succeeds with the construction's rank and
    E21 <= 1e-12 |A|_1, and a sample matches single calls bitwise."""
    n = 128
    probs = [S.sym_problem(n, S.family_seed(0, 300 + i)) for i in range(64)]
    print_case(test="batched64x128")
    regs = [sdc.region("halfplane", shift=0.0, scale=1.0)] * 64
    out = handle.split_sym_batched([dev(a) for a, _, _ in probs], regs, sdc.opts(seed=5))
    for i, ((a, d, q), r) in enumerate(zip(probs, out)):
        assert r.status == sdc.SDC_OK, (i, r.status, r.info)
        k = r.info["k_lead"]
        assert k == int((d > 0).sum())
        ah = host(r.Ahat)
        assert norm1(ah[k:, :k]) <= 1e-12 * norm1(a)
    for i in (0, 31, 63):
        single = handle.split_sym(dev(probs[i][0]), regs[i], sdc.opts(seed=5 + i * 1000003))
        assert torch.equal(single.Q, out[i].Q) and torch.equal(single.Ahat, out[i].Ahat)


def test_edge_cases(handle, sdc):
    print_case(test="edges")
    # n = 1: no split possible
    res = handle.split_sym(dev(np.array([[0.5]])), sdc.region("halfplane", shift=0.0, scale=1.0))
    assert res.status == sdc.SDC_NO_SPLIT and res.info["n_inside"] == 0
    res = handle.split_sym(dev(np.array([[-0.5]])), sdc.region("halfplane", shift=0.0, scale=1.0))
    assert res.status == sdc.SDC_NO_SPLIT and res.info["n_inside"] == 1
    # all eigenvalues on one side
    a, d, q = S.sym_problem(40, 9)
    res = handle.split_sym(dev(a), sdc.region("halfplane", shift=3.0, scale=1.0))
    assert res.status == sdc.SDC_NO_SPLIT and res.info["n_inside"] == 40
    # iteration cap
    res = handle.split_sym(dev(a), sdc.region("halfplane", shift=0.0, scale=1.0), sdc.opts(maxit=1))
    assert res.status == sdc.SDC_NOT_CONVERGED
    # non-finite input
    bad = a.copy()
    bad[3, 5] = np.nan
    with pytest.raises(sdc.SdcError, match="NONFINITE"):
        handle.split_sym(dev(bad), sdc.region("halfplane", shift=0.0, scale=1.0))
    # invalid region
    with pytest.raises(sdc.SdcError, match="INVALID"):
        handle.split_sym(dev(a), sdc.region("disk", center=0.0, radius=-1.0))


# ---------------------------------------------------------------------------
# RNEP (sdc_split_nonsym): non-symmetric A, B = I
# ---------------------------------------------------------------------------

def _sin_theta(x, y):
    qx, _ = np.linalg.qr(x)
    qy, _ = np.linalg.qr(y)
    return float(np.linalg.norm(qy - qx @ (qx.T @ qy), 2))


@pytest.mark.parametrize("n", [40, 150])
def test_split_nonsym_matches_oracle(handle, sdc, n):
    from oracle.split import split_nonsym
    a, lam = S.nonsym_problem(n, S.family_seed(6, 100 + n))
    print_case(test="split_nonsym", n=n)
    res = handle.split_nonsym(dev(a), sdc.region(), sdc.opts(seed=9))
    ref = split_nonsym(a, {"kind": "unit_disk"}, seed=9)
    k = int((np.abs(lam) > 1).sum())
    assert res.status == sdc.SDC_OK and res.info["k_lead"] == k == ref.k
    q, ah = host(res.Q), host(res.Ahat)
    assert np.abs(q.T @ q - np.eye(n)).max() <= 1e-13
    assert norm1(ah[k:, :k]) <= 1e-10 * norm1(a)
    assert _sin_theta(q[:, :k], ref.Q[:, :k]) <= 1e-10
    assert np.abs(q.T @ a @ q - ah).max() <= 1e-12 * norm1(a)  # not symmetrized
    for blk, rblk in ((ah[:k, :k], ref.A_hat[:k, :k]), (ah[k:, k:], ref.A_hat[k:, k:])):
        ev, rev = np.sort_complex(np.linalg.eigvals(blk)), np.sort_complex(np.linalg.eigvals(rblk))
        assert np.abs(ev - rev).max() <= 1e-9 * np.abs(lam).max()


def test_split_nonsym_equals_pencil_with_identity(handle, sdc):
    """The pencil step with B = I runs the same right side: its Q_R is RNEP's Q."""
    n = 64
    a, lam = S.nonsym_problem(n, S.family_seed(6, 7))
    print_case(test="split_nonsym_vs_pencil", n=n)
    r1 = handle.split_nonsym(dev(a), sdc.region(), sdc.opts(seed=4))
    r2 = handle.split_pencil(dev(a), dev(np.eye(n)), sdc.region(), sdc.opts(seed=4))
    assert r1.status == r2.status == sdc.SDC_OK and r1.info["k_lead"] == r2.info["k_lead"]
    assert r1.info["iters_right"] == r2.info["iters_right"]
    assert torch.allclose(r1.Q, r2.Q, rtol=0, atol=1e-12)


def test_split_nonsym_complex_pairs(handle, sdc):
    from oracle.split import split_nonsym
    n = 64
    a, ev = S.normal_random_problem(n, S.family_seed(6, 64))
    print_case(test="split_nonsym_pairs", n=n)
    reg = sdc.region("halfplane", shift=0.0, scale=1.0)
    res = handle.split_nonsym(dev(a), reg, sdc.opts(seed=2))
    k = int((ev.real > 0).sum())
    assert res.status == sdc.SDC_OK and res.info["k_lead"] == k
    ah = host(res.Ahat)
    got = np.sort_complex(np.linalg.eigvals(ah[:k, :k]))
    assert np.abs(got - np.sort_complex(ev[ev.real > 0])).max() <= 1e-9
    ref = split_nonsym(a, {"kind": "halfplane", "shift": 0.0, "scale": 1.0}, seed=2)
    assert _sin_theta(host(res.Q)[:, :k], ref.Q[:, :k]) <= 1e-10
    with pytest.raises(sdc.SdcError):
        handle.split_nonsym(dev(a), reg, sdc.opts(prec=sdc.SDC_FP32_REFINE))


def test_split_nonsym_order_one_and_one_sided(handle, sdc):
    """RNEP's degenerate cases: order 1 (no split possible) and every
    eigenvalue on one side of the curve."""
    print_case(test="split_nonsym_edges")
    res = handle.split_nonsym(dev(np.array([[3.0]])), sdc.region())
    assert res.status == sdc.SDC_NO_SPLIT and res.info["n_inside"] == 0
    res = handle.split_nonsym(dev(np.array([[0.25]])), sdc.region())
    assert res.status == sdc.SDC_NO_SPLIT and res.info["n_inside"] == 1
    a, lam = S.nonsym_problem(30, S.family_seed(6, 30), lam_lo=1.5, lam_hi=8.0)
    res = handle.split_nonsym(dev(a), sdc.region())
    assert res.status == sdc.SDC_NO_SPLIT and res.info["n_inside"] == 0
