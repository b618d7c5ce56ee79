"""Replay of the repeated-squaring iterations from a HIP graph
(sdc_graphs_enable): every result bitwise equal to the direct launches, for
single splits (one panel to two-level trees), pencils, FP32 iterates, a
batch whose problems finish at different iterations (switched off between
replays), and the divide-and-conquer (one graph per level); graph calls
interleaved with eager work and with each other, and the fallbacks to
direct launches (profiling on; a handle whose QRs from 1200 factored
columns run the two-stream look-ahead schedule, which is not captured)."""
import numpy as np
import pytest

import sdc_synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sdc():
    import paper_1011_3077_amd as P
    return P


@pytest.fixture(scope="module")
def handles(sdc):
    hd, hg = sdc.Handle(0), sdc.Handle(0)
    hg.graphs_enable(True)
    yield hd, hg
    hd.close()
    hg.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def print_case(**kw):
    print("CASE", kw, flush=True)


def same(a, b):
    """Bitwise equal outputs and info, except the call's wall time and the
    orth_err diagnostic (its sum over blocks is accumulated atomically, so
    its last bit depends on their order in any two runs)."""
    assert a.status == b.status
    skip = ("ms", "orth_err")
    assert {k: v for k, v in a.info.items() if k not in skip} == {k: v for k, v in b.info.items() if k not in skip}
    assert abs(a.info["orth_err"] - b.info["orth_err"]) <= 1e-15 * max(1.0, abs(a.info["orth_err"])) + 1e-30
    for x, y in ((a.Q, b.Q), (a.Ahat, b.Ahat), (a.QL, b.QL), (a.Bhat, b.Bhat)):
        if x is None:
            assert y is None
        else:
            assert torch.equal(x, y)


@pytest.mark.parametrize("n,prec", [(2, 0), (128, 0), (700, 0), (1300, 0), (300, 1), (1300, 1)])
def test_split_sym_graph_equals_direct(sdc, handles, n, prec):
    hd, hg = handles
    print_case(test="graph_split_sym", n=n, prec=prec)
    a, d, q = S.sym_problem(n, S.family_seed(0, 2000 + n))
    A = dev(a)
    reg = sdc.region("halfplane", shift=0.0, scale=1.0)
    o = sdc.opts(prec=prec, seed=5, diagnostics=1)
    r_d = hd.split_sym(A, reg, o)
    r_g = hg.split_sym(A, reg, o)
    assert r_g.status == sdc.SDC_OK and r_g.info["k_lead"] == int((d > 0).sum())
    same(r_d, r_g)
    # eager work between graph calls, then the same call again
    junk = torch.randn(512, 512, device="cuda:0", dtype=torch.float64) @ torch.randn(512, 512, device="cuda:0",
                                                                                   dtype=torch.float64)
    r_g2 = hg.split_sym(A, reg, o)
    same(r_g, r_g2)
    del junk


@pytest.mark.parametrize("n", [48, 300])
def test_split_pencil_graph_equals_direct(sdc, handles, n):
    hd, hg = handles
    print_case(test="graph_split_pencil", n=n)
    pb = S.pencil_problem(n, S.family_seed(1, 2000 + n))
    A, B = dev(pb["A"]), dev(pb["B"])
    o = sdc.opts(seed=8)
    same(hd.split_pencil(A, B, sdc.region(), o), hg.split_pencil(A, B, sdc.region(), o))


def test_batched_graph_equals_direct(sdc, handles):
    """64 problems of orders 32 to 256 (FP32 iterates and FP64 refinement):
    sides converge at different iterations and are switched off between
    replays; every problem bitwise as with direct launches."""
    hd, hg = handles
    sizes = S.batch_sizes(64, S.family_seed(2, 2100))
    print_case(test="graph_batched", count=len(sizes), nmin=min(sizes), nmax=max(sizes))
    As = [dev(S.sym_problem(n, S.family_seed(2, 2100 + i))[0]) for i, n in enumerate(sizes)]
    regs = [sdc.region("halfplane", shift=0.0, scale=1.0)] * len(sizes)
    o = sdc.opts(prec=sdc.SDC_FP32_REFINE, seed=3)
    out_d = hd.split_sym_batched(As, regs, o)
    out_g = hg.split_sym_batched(As, regs, o)
    iters = set()
    for x, y in zip(out_d, out_g):
        same(x, y)
        iters.add(x.info["iters_right"])
    assert len(iters) > 1  # the switch-off path ran


def test_eig_dc_graph_equals_direct(sdc, handles):
    hd, hg = handles
    n = 200
    print_case(test="graph_eig_dc", n=n)
    pb = S.pencil_problem(n, S.family_seed(1, 2200))
    A, B = dev(pb["A"]), dev(pb["B"])
    rd = hd.eig_dc(A, B, leaf_max=16, o=sdc.opts(seed=2))
    rg = hg.eig_dc(A, B, leaf_max=16, o=sdc.opts(seed=2))
    assert rd[0] == rg[0] == sdc.SDC_OK
    for x, y in zip(rd[1:5], rg[1:5]):
        assert torch.equal(x, y)
    assert list(rd[5]) == list(rg[5])


def test_profiling_falls_back_to_direct_launches(sdc, handles):
    hd, hg = handles
    print_case(test="graph_profile_fallback")
    a, d, q = S.sym_problem(256, S.family_seed(0, 2300))
    A = dev(a)
    reg = sdc.region("halfplane", shift=0.0, scale=1.0)
    hg.profile_enable(True)
    try:
        r = hg.split_sym(A, reg, sdc.opts(seed=1))
        st = hg.profile_read(sdc.KERNEL_PANEL)
        assert r.status == sdc.SDC_OK and st["launches"] > 0 and st["ms"] > 0
    finally:
        hg.profile_enable(False)
    same(hd.split_sym(A, reg, sdc.opts(seed=1)), hg.split_sym(A, reg, sdc.opts(seed=1)))


def test_lookahead_falls_back_to_direct_launches(sdc):
    """With the look-ahead schedule enabled from 1200 factored columns, an
    order-1300 split is not captured: the graph handle launches it directly,
    with the same bits as a direct-launch handle of the same schedule."""
    hd, hg = sdc.Handle(0), sdc.Handle(0)
    try:
        for h in (hd, hg):
            h.lookahead_set(1200)
        hg.graphs_enable(True)
        n = 1300
        print_case(test="graph_lookahead_fallback", n=n)
        a, d, q = S.sym_problem(n, S.family_seed(0, 2400))
        A = dev(a)
        reg = sdc.region("halfplane", shift=0.0, scale=1.0)
        o = sdc.opts(seed=4, diagnostics=1)
        r_d = hd.split_sym(A, reg, o)
        assert r_d.status == sdc.SDC_OK and r_d.info["k_lead"] == int((d > 0).sum())
        same(r_d, hg.split_sym(A, reg, o))
    finally:
        hd.close()
        hg.close()
