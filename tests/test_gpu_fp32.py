"""FP32 repeated squaring with the FP64 refinement (symmetric problems),
through the C ABI, against the FP64 oracle and the construction.

The FP32 iterates carry errors of order eps32 * |A| / gap into the basis, so
what is compared is what the refinement must restore to FP64 quality: the
split rank exactly (= #(d > shift) by construction and the oracle's k), the
leading invariant subspace (against the oracle's Q and the construction's
eigenvectors, sin(angle) <= 1e-9), ||E21||_1 <= split_tol ||A||_1, the
eigenvalues of the diagonal blocks (<= 1e-9 |A|_2, the accuracy target of
the FP32+refine path) and the orthogonality of Q.  The refinement step is
not in the paper; the oracle's version of it is pinned separately on the CPU.
"""
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


def check_split(res, a, d, n, shift=0.0, eig_tol=1e-9, sub_tol=1e-9):
    assert res.status == 0, res.status
    k = res.info["k_lead"]
    assert k == int((d > shift).sum())
    assert res.info["n_inside"] == n - k
    Q, Ah = host(res.Q), host(res.Ahat)
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 1e-13 * max(1.0, np.sqrt(n))
    assert norm1(Ah[k:, :k]) <= 1e-10 * norm1(a)
    ev = np.sort(np.concatenate([np.linalg.eigvalsh(Ah[:k, :k]), np.linalg.eigvalsh(Ah[k:, k:])]))
    assert np.abs(ev - np.sort(d)).max() <= eig_tol * np.abs(d).max()
    return k, Q, Ah


@pytest.mark.parametrize("n", [16, 64, 128, 257])
def test_fp32_refine_split_matches_fp64_oracle(handle, sdc, n):
    import oracle as O
    print("CASE fp32 split_sym", n, flush=True)
    a, d, q = S.sym_problem(n, S.family_seed(2, n))
    res = handle.split_sym(dev(a), sdc.region("halfplane", shift=0.0, scale=1.0),
                           sdc.opts(prec=sdc.SDC_FP32_REFINE, seed=5))
    k, Q, Ah = check_split(res, a, d, n)
    ref = O.split_sym(a, HALF0, seed=5)
    assert ref.k == k
    assert sin_theta(Q[:, :k], ref.Q[:, :k]) <= 1e-9
    assert sin_theta(Q[:, :k], q[:, d > 0]) <= 1e-9
    if n >= 64:
        assert res.info["refine_rounds"] >= 1


def test_fp32_irs_converges_like_closed_form(handle, sdc):
    """FP32 repeated squaring stops where the closed form with tau = sqrt(eps32)
    says (within one iteration: FP32 rounding moves the relative change), and
    its projector (A_p + B_p)^{-1} A_p is the outside projector to FP32 accuracy."""
    from closed_form import predicted_p_sym
    n = 96
    print("CASE fp32 irs", n, flush=True)
    a, d, q = S.sym_problem(n, S.family_seed(2, 1))
    st, ap, bp, r, p, rc = handle.irs(dev(a), None, sdc.region("halfplane", shift=0.0, scale=1.0),
                                      sdc.opts(prec=sdc.SDC_FP32_REFINE))
    assert st == 0
    p_pred = predicted_p_sym(d, tau=float(np.finfo(np.float32).eps) ** 0.5)
    assert abs(p - p_pred) <= 1
    ap, bp = host(ap), host(bp)
    proj = np.linalg.solve(ap + bp, ap)
    want = (q[:, d > 0]) @ (q[:, d > 0]).T
    assert np.abs(proj - want).max() <= 2e-4


def test_fp32_refine_batched_equals_single(handle, sdc):
    sizes = [32, 45, 64, 100, 150, 256]
    print("CASE fp32 batched", sizes, flush=True)
    probs = [S.sym_problem(n, S.family_seed(2, 100 + i)) for i, n in enumerate(sizes)]
    o = sdc.opts(prec=sdc.SDC_FP32_REFINE, seed=11)
    reg = sdc.region("halfplane", shift=0.0, scale=1.0)
    out = handle.split_sym_batched([dev(a) for a, _, _ in probs], [reg] * len(sizes), o)
    for i, ((a, d, q), r) in enumerate(zip(probs, out)):
        check_split(r, a, d, sizes[i])
        single = handle.split_sym(dev(a), reg, sdc.opts(prec=sdc.SDC_FP32_REFINE, seed=11 + i * 1000003))
        assert single.status == r.status
        assert torch.equal(single.Q, r.Q) and torch.equal(single.Ahat, r.Ahat)


def test_fp32_refine_clustered_vs_fp64(handle, sdc):
    """The clustered spectrum (5% of eigenvalues within 1e-3 of +-0.01) at
    order 1024: FP32+refine and FP64 give the same rank and subspace."""
    n = 1024
    print("CASE fp32 clustered", n, flush=True)
    a, d, q = S.clustered_sym_problem(n, S.family_seed(3, 1))
    reg = sdc.region("halfplane", shift=0.0, scale=1.0)
    r32 = handle.split_sym(dev(a), reg, sdc.opts(prec=sdc.SDC_FP32_REFINE, seed=2))
    r64 = handle.split_sym(dev(a), reg, sdc.opts(prec=sdc.SDC_FP64, seed=2))
    k32, Q32, A32 = check_split(r32, a, d, n)
    k64, Q64, A64 = check_split(r64, a, d, n, eig_tol=1e-12)
    assert k32 == k64 == n // 2
    # Davis-Kahan: each leading block is within |E21|_F / gap of the exact
    # invariant subspace (gap = 0.02 between the clusters at -+0.01)
    gap = d[d > 0].min() - d[d < 0].max()
    b32 = np.linalg.norm(A32[k32:, :k32]) / gap
    b64 = np.linalg.norm(A64[k64:, :k64]) / gap
    exact = q[:, d > 0]
    assert sin_theta(Q32[:, :k32], exact) <= b32 + 1e-12
    assert sin_theta(Q64[:, :k64], exact) <= b64 + 1e-12
    assert sin_theta(Q32[:, :k32], Q64[:, :k64]) <= b32 + b64 + 1e-12
    assert r32.info["iters_right"] <= r64.info["iters_right"]


def test_fp32_refine_eig_dc_symmetric(handle, sdc):
    n, leaf = 300, 40
    print("CASE fp32 eig_dc", n, flush=True)
    a, d, q = S.sym_problem(n, S.family_seed(2, 9))
    st, t, s, ql, qr, starts, info = handle.eig_dc(dev(a), None, leaf_max=leaf, symmetric=True,
                                                    o=sdc.opts(prec=sdc.SDC_FP32_REFINE, seed=4))
    assert st == 0 and info["unsplit"] == 0
    t, qr = host(t), host(qr)
    assert all(e - s0 <= leaf for s0, e in zip(starts[:-1], starts[1:]))
    ev = np.sort(np.concatenate([np.linalg.eigvalsh(0.5 * (t[x:y, x:y] + t[x:y, x:y].T))
                                 for x, y in zip(starts[:-1], starts[1:])]))
    assert np.abs(ev - np.sort(d)).max() <= 1e-9
    assert np.abs(qr.T @ qr - np.eye(n)).max() <= 1e-12


def test_fp32_refine_rejected_for_pencils(handle, sdc):
    p = S.pencil_problem(16, S.family_seed(1, 3))
    with pytest.raises(sdc.SdcError):
        handle.split_pencil(dev(p["A"]), dev(p["B"]), sdc.region(), sdc.opts(prec=sdc.SDC_FP32_REFINE))


def near_shift_problem(n, seed, d0):
    """Symmetric problem with one eigenvalue at d0 (next to the split point 0)
    and the others with |d| >= 0.05."""
    a, d, q = S.sym_problem(n, seed)
    d = d.copy()
    d[0] = d0
    a = (q * d[None, :]) @ q.T
    return np.asfortranarray(0.5 * (a + a.T)), d


def test_fp32_near_shift_eigenvalue_either_side(handle, sdc):
    """An eigenvalue 1e-12 from the split point is below FP32 resolution: the
    FP32 iterates may put it on either side, and what comes back is still an
    exact (FP64-quality) invariant-subspace split with every other eigenvalue
    on its own side."""
    n = 64
    print("CASE fp32 near shift", n, flush=True)
    a, d = near_shift_problem(n, S.family_seed(2, 77), 1e-12)
    res = handle.split_sym(dev(a), sdc.region("halfplane", shift=0.0, scale=1.0),
                           sdc.opts(prec=sdc.SDC_FP32_REFINE, seed=9))
    assert res.status == 0, res.status
    k = res.info["k_lead"]
    kpos = int((d > 0).sum())
    assert k in (kpos - 1, kpos)
    Q, Ah = host(res.Q), host(res.Ahat)
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 1e-13 * np.sqrt(n)
    assert norm1(Ah[k:, :k]) <= 1e-10 * norm1(a)
    e1 = np.linalg.eigvalsh(Ah[:k, :k])
    e2 = np.linalg.eigvalsh(Ah[k:, k:])
    assert np.abs(np.sort(np.concatenate([e1, e2])) - np.sort(d)).max() <= 1e-9
    assert e1.min() >= -1e-9 and e2.max() <= 1e-9


def overflow_problem(n, seed, sign):
    """Symmetric problem scaled past the FP32 range (|a_ij| up to ~1e39 >
    FLT_MAX): FP32 iterates cannot hold it, FP64 can.  The half-plane map
    takes the problem's scale (A0 = A + sI, B0 = A - sI with s = 1e40), so
    the FP64 iteration converges as for the unscaled problem."""
    a, d, q = S.sym_problem(n, seed)
    s = sign * 1e40
    return np.asfortranarray(a * s), d * s


def test_fp32_falls_back_to_fp64(handle, sdc):
    """The FP32 iterates overflow (SDC_ERR_NONFINITE on the FP32 attempt):
    the split is redone in FP64 and is exact."""
    n = 64
    print("CASE fp32 fallback", n, flush=True)
    a, d = overflow_problem(n, S.family_seed(2, 77), 1.0)
    assert np.abs(a).max() > np.finfo(np.float32).max
    res = handle.split_sym(dev(a), sdc.region("halfplane", shift=0.0, scale=1e40),
                           sdc.opts(prec=sdc.SDC_FP32_REFINE, seed=9))
    assert res.info["fp64_fallback"] == 1
    check_split(res, a, d, n, eig_tol=1e-12)


def test_fp32_fallback_in_server(handle, sdc):
    n = 64
    print("CASE fp32 fallback server", n, flush=True)
    a, d = overflow_problem(n, S.family_seed(2, 78), -1.0)
    srv = sdc.Server(0)
    try:
        t = srv.submit(dev(a), None, sdc.region("halfplane", shift=0.0, scale=1e40),
                       sdc.opts(prec=sdc.SDC_FP32_REFINE, seed=9))
        r = srv.wait(t)
    finally:
        srv.close()
    assert r.info["fp64_fallback"] == 1
    check_split(r, a, d, n, eig_tol=1e-12)
