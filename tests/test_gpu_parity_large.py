"""Element-by-element parity with the FP64 oracle at sizes that reach the
kernel paths of the full-size workloads.

Orders 1250-1300 give 2n > 2048 stacked rows, so every panel's TSQR tree has
leaves of up to 256 rows and internal levels (the tree of the order-2048 and
order-8192 problems).  Each case runs on two handles against one oracle
result: the default one-stream schedule (the tree above the leaves factored
beside the leaf-level update), and the two-stream look-ahead schedule
(sdc_lookahead_set(1200): the next panel factored while the bulk of the
trailing matrix is updated, the row-split kernel on its columns).  Same
caller Gaussians on both sides, so the
leading bases are unique and compared entry by entry; what is unique of the
rest (subspaces, block spectra, E21) is compared as in the small-size tests.
The FP32+refine path is held to the FP64 oracle at the same order.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import sdc_synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HALF0 = {"kind": "halfplane", "shift": 0.0, "scale": 1.0}


@pytest.fixture(scope="module")
def sdc():
    import paper_1011_3077_amd as P
    return P


@pytest.fixture(scope="module")
def handles(sdc):
    one, la = sdc.Handle(0), sdc.Handle(0)
    la.lookahead_set(1200)
    yield [("one-stream", one), ("look-ahead", la)]
    one.close()
    la.close()


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
    gs = [S.gaussian(n, seed + 10 * a + side) for a in range(attempts) for side in range(2)]
    return gs, dev(np.concatenate([g.ravel(order="F") for g in gs]))


def print_case(**kw):
    print("CASE", kw, flush=True)


def test_split_sym_matches_oracle_order_1300(handles, sdc):
    import oracle as O
    n = 1300
    seed = S.family_seed(0, 1300)
    a, d, q = S.sym_problem(n, seed)
    gs, gdev = gauss_stack(n, seed)
    ref = O.split_sym(a, HALF0, gauss=lambda nn, att, side: gs[2 * att + side])
    for name, handle in handles:
        print_case(test="split_sym_large", n=n, schedule=name)
        check_split_sym_1300(sdc, handle, a, d, gdev, ref, n)


def check_split_sym_1300(sdc, handle, a, d, gdev, ref, n):
    res = handle.split_sym(dev(a), sdc.region("halfplane", shift=0.0, scale=1.0), sdc.opts(G=gdev, diagnostics=1))
    info = res.info
    assert res.status == ref.status == sdc.SDC_OK
    k = info["k_lead"]
    assert k == ref.k == int((d > 0).sum())
    assert info["iters_right"] == ref.p_right and info["attempts"] == ref.attempts
    Q, Ah = host(res.Q), host(res.Ahat)
    assert np.abs(Q[:, :k] - ref.Q[:, :k]).max() <= 1e-10
    assert np.abs(Ah[:k, :k] - ref.A_hat[:k, :k]).max() <= 1e-10 * norm1(a)
    assert sin_theta(Q[:, k:], ref.Q[:, k:]) <= 1e-10
    # E21 is rounding: about n eps |A|_1 for both (the order-128 bar of 1e-12
    # scales with n), and the two agree to that level
    e_tol = 10 * n * np.finfo(float).eps
    assert info["e21_rel"] <= e_tol and abs(info["e21_rel"] - ref.e) <= e_tol
    assert info["orth_err"] <= 1e-13 * n
    ev = np.sort(np.concatenate([np.linalg.eigvalsh(Ah[:k, :k]), np.linalg.eigvalsh(Ah[k:, k:])]))
    assert np.abs(ev - np.sort(d)).max() <= 1e-10 * np.abs(d).max()


def test_irs_pencil_matches_oracle_order_1250(handles, sdc):
    """R_j of the last iteration (unique with a non-negative diagonal) entry
    by entry, the count p, and the Gram invariants of the iterates."""
    import oracle as O
    n = 1250
    pb = S.pencil_problem(n, S.family_seed(1, 1250))
    ref = O.irs(pb["A"], pb["B"], record=True)
    rr = ref.R_history[-1]
    for name, handle in handles:
        print_case(test="irs_pencil_large", n=n, schedule=name)
        st, ap, bp, r, p, rc = handle.irs(dev(pb["A"]), dev(pb["B"]), sdc.region())
        assert st == sdc.SDC_OK and ref.converged and p == ref.p
        assert np.abs(host(r) - rr).max() <= 1e-10 * np.abs(rr).max()
        ap, bp = host(ap), host(bp)
        for x, y in ((ap.T @ ap, ref.A.T @ ref.A), (bp.T @ bp, ref.B.T @ ref.B), (ap.T @ bp, ref.A.T @ ref.B)):
            assert np.abs(x - y).max() <= 1e-9 * max(1.0, np.abs(y).max())


def test_split_pencil_matches_oracle_order_1250(handles, sdc):
    import oracle as O
    n = 1250
    seed = S.family_seed(1, 1250)
    pb = S.pencil_problem(n, seed)
    a, b, lam = pb["A"], pb["B"], pb["lam"]
    gs, gdev = gauss_stack(n, seed)
    ref = O.split_pencil(a, b, {"kind": "unit_disk"}, gauss=lambda nn, att, side: gs[2 * att + side])
    for name, handle in handles:
        print_case(test="split_pencil_large", n=n, schedule=name)
        check_split_pencil_1250(sdc, handle, a, b, lam, gdev, ref)


def check_split_pencil_1250(sdc, handle, a, b, lam, gdev, ref):
    res = handle.split_pencil(dev(a), dev(b), sdc.region(), sdc.opts(G=gdev, diagnostics=1))
    info = res.info
    assert res.status == ref.status == sdc.SDC_OK
    k = info["k_lead"]
    assert k == ref.k == int((np.abs(lam) > 1).sum())
    assert info["iters_right"] == ref.p_right and info["iters_left"] == ref.p_left
    assert info["attempts"] == ref.attempts
    QR, QL, Ah, Bh = host(res.Q), host(res.QL), host(res.Ahat), host(res.Bhat)
    assert np.abs(QR[:, :k] - ref.Q[:, :k]).max() <= 1e-9
    assert np.abs(QL[:, :k] - ref.QL[:, :k]).max() <= 1e-9
    assert sin_theta(QR[:, k:], ref.Q[:, k:]) <= 1e-9
    assert sin_theta(QL[:, k:], ref.QL[:, k:]) <= 1e-9
    assert np.abs(Ah[:k, :k] - ref.A_hat[:k, :k]).max() <= 1e-9 * norm1(a)
    assert np.abs(Bh[:k, :k] - ref.B_hat[:k, :k]).max() <= 1e-9 * norm1(b)
    assert info["e21_rel"] <= 1e-11 and abs(info["e21_rel"] - ref.e) <= 1e-11
    blocks = lambda ah, bh: np.sort_complex(np.concatenate([sla.eigvals(ah[:k, :k], bh[:k, :k]),
                                                            sla.eigvals(ah[k:, k:], bh[k:, k:])]))
    want = np.sort_complex(lam.astype(complex))
    err = np.max(np.abs(blocks(Ah, Bh) - want) / np.abs(want))
    # the construction's eigenvalues are conditioned so that at this order
    # even the oracle's blocks (and LAPACK's QZ of the whole pencil) are
    # about 2e-10 off: the bar is 1e-10, or the oracle's own error
    err_ref = np.max(np.abs(blocks(ref.A_hat, ref.B_hat) - want) / np.abs(want))
    assert err <= max(1e-10, 2 * err_ref), (err, err_ref)


def test_fp32_refine_matches_fp64_oracle_order_1300(handles, sdc):
    """FP32 repeated squaring (the FP32 panel and update kernels on the
    three-level tree, both schedules) + FP64 refinement, against
    the FP64 oracle's split of the same matrix: exact rank, the outside
    subspace within 1e-9 (or the Davis-Kahan bound of the remaining E21),
    block eigenvalues within 1e-9 |A|_2, E21 within split_tol."""
    import oracle as O
    n = 1300
    seed = S.family_seed(0, 1301)
    a, d, q = S.sym_problem(n, seed)
    ref = O.split_sym(a, HALF0, seed=3)
    for name, handle in handles:
        print_case(test="fp32_refine_large", n=n, schedule=name)
        check_fp32_refine_1300(sdc, handle, a, d, ref, n)


def check_fp32_refine_1300(sdc, handle, a, d, ref, n):
    res = handle.split_sym(dev(a), sdc.region("halfplane", shift=0.0, scale=1.0),
                           sdc.opts(prec=sdc.SDC_FP32_REFINE, seed=3, diagnostics=1))
    info = res.info
    assert res.status == ref.status == sdc.SDC_OK and info["fp64_fallback"] == 0
    k = info["k_lead"]
    assert k == ref.k == int((d > 0).sum())
    Q, Ah = host(res.Q), host(res.Ahat)
    gap = float(np.min(d[d > 0]) - np.max(d[d < 0]))
    e21 = np.linalg.norm(Ah[k:, :k])
    assert sin_theta(Q[:, :k], ref.Q[:, :k]) <= max(1e-9, 2 * e21 / gap)
    assert info["e21_rel"] <= 1e-10
    assert info["orth_err"] <= 1e-13 * np.sqrt(n) * 10
    ev = np.sort(np.concatenate([np.linalg.eigvalsh(Ah[:k, :k]), np.linalg.eigvalsh(Ah[k:, k:])]))
    assert np.abs(ev - np.sort(d)).max() <= 1e-9 * np.abs(d).max()
    ev_ref = np.sort(np.concatenate([np.linalg.eigvalsh(ref.A_hat[:k, :k]), np.linalg.eigvalsh(ref.A_hat[k:, k:])]))
    assert np.abs(ev - ev_ref).max() <= 1e-9 * np.abs(d).max()
