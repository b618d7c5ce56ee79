"""The QR schedule that factors a panel's reduction tree above its leaves in
the same launch as the leaves' trailing update (sdc_tree_overlap_enable, the
default) against the schedule that factors the whole tree first: every
output bitwise equal, for trees of two, three and four levels (stacked
heights up to 16400 rows), FP64 and FP32 iterates, pencils, a batch of
mixed orders, the divide-and-conquer, and with the iterations replayed from
a HIP graph."""
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
    h_on, h_off = sdc.Handle(0), sdc.Handle(0)
    h_off.tree_overlap_enable(False)
    yield h_on, h_off
    h_on.close()
    h_off.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def print_case(**kw):
    print("CASE", kw, flush=True)


def same(a, b):
    """Bitwise equal outputs and info, except the call's wall time and the
    orth_err diagnostic (summed over blocks with atomics, so its last bit
    depends on their order)."""
    assert a.status == b.status
    skip = ("ms", "orth_err")
    assert {k: v for k, v in a.info.items() if k not in skip} == {k: v for k, v in b.info.items() if k not in skip}
    assert abs(a.info["orth_err"] - b.info["orth_err"]) <= 1e-15 * max(1.0, abs(a.info["orth_err"])) + 1e-30
    for x, y in ((a.Q, b.Q), (a.Ahat, b.Ahat), (a.QL, b.QL), (a.Bhat, b.Bhat)):
        if x is None:
            assert y is None
        else:
            assert torch.equal(x, y)


# orders whose stacked heights 2n give one leaf (n = 100), two levels
# (200, 700) and three levels (1100: 2200 rows, nine leaves)
@pytest.mark.parametrize("n,prec", [(100, 0), (200, 0), (700, 0), (1100, 0), (700, 1), (1100, 1)])
def test_split_sym_overlap_equals_serial(sdc, handles, n, prec):
    h_on, h_off = handles
    print_case(test="tree_overlap_split_sym", n=n, prec=prec)
    a, d, q = S.sym_problem(n, S.family_seed(0, 3000 + n))
    A = dev(a)
    reg = sdc.region("halfplane", shift=0.0, scale=1.0)
    o = sdc.opts(prec=prec, seed=4, diagnostics=1)
    r_on = h_on.split_sym(A, reg, o)
    r_off = h_off.split_sym(A, reg, o)
    assert r_on.status == sdc.SDC_OK and r_on.info["k_lead"] == int((d > 0).sum())
    same(r_on, r_off)


@pytest.mark.parametrize("n", [300, 1100])
def test_split_pencil_overlap_equals_serial(sdc, handles, n):
    h_on, h_off = handles
    print_case(test="tree_overlap_split_pencil", n=n)
    pb = S.pencil_problem(n, S.family_seed(1, 3000 + n))
    A, B = dev(pb["A"]), dev(pb["B"])
    o = sdc.opts(seed=6)
    r_on = h_on.split_pencil(A, B, sdc.region(), o)
    assert r_on.status == sdc.SDC_OK
    same(r_on, h_off.split_pencil(A, B, sdc.region(), o))


def test_batched_overlap_equals_serial(sdc, handles):
    """64 problems of orders 32 to 256 (one- and two-level trees in one
    launch), FP32 iterates with FP64 refinement."""
    h_on, h_off = handles
    sizes = S.batch_sizes(64, S.family_seed(2, 3100))
    print_case(test="tree_overlap_batched", count=len(sizes), nmin=min(sizes), nmax=max(sizes))
    As = [dev(S.sym_problem(n, S.family_seed(2, 3100 + i))[0]) for i, n in enumerate(sizes)]
    regs = [sdc.region("halfplane", shift=0.0, scale=1.0)] * len(sizes)
    o = sdc.opts(prec=sdc.SDC_FP32_REFINE, seed=3)
    for x, y in zip(h_on.split_sym_batched(As, regs, o), h_off.split_sym_batched(As, regs, o)):
        same(x, y)


def test_eig_dc_overlap_equals_serial(sdc, handles):
    h_on, h_off = handles
    n = 600
    print_case(test="tree_overlap_eig_dc", n=n)
    pb = S.pencil_problem(n, S.family_seed(1, 3200))
    A, B = dev(pb["A"]), dev(pb["B"])
    r_on = h_on.eig_dc(A, B, leaf_max=32, o=sdc.opts(seed=2))
    r_off = h_off.eig_dc(A, B, leaf_max=32, o=sdc.opts(seed=2))
    assert r_on[0] == r_off[0] == sdc.SDC_OK
    for x, y in zip(r_on[1:5], r_off[1:5]):
        assert torch.equal(x, y)
    assert list(r_on[5]) == list(r_off[5])


def test_graph_replay_overlap_equals_serial(sdc, handles):
    """The overlapped schedule captured in a HIP graph and replayed, against
    direct launches of the serial schedule."""
    h_on, h_off = handles
    hg = sdc.Handle(0)
    try:
        hg.graphs_enable(True)
        n = 700
        print_case(test="tree_overlap_graph", n=n)
        a, d, q = S.sym_problem(n, S.family_seed(0, 3300))
        A = dev(a)
        reg = sdc.region("halfplane", shift=0.0, scale=1.0)
        o = sdc.opts(seed=9, diagnostics=1)
        r_off = h_off.split_sym(A, reg, o)
        same(hg.split_sym(A, reg, o), r_off)
        same(hg.split_sym(A, reg, o), r_off)
    finally:
        hg.close()


def test_four_level_tree_overlap_equals_serial(sdc, handles):
    """Order 8200: a stacked height of 16400 rows gives 65 leaves and four
    tree levels (the climb beside the leaf-level update goes through two
    level-2 nodes to the root).  The matrix is built on the device (seeded):
    the comparison is between the two schedules, whose outputs must be
    bitwise equal."""
    h_on, h_off = handles
    n = 8200
    print_case(test="tree_overlap_four_levels", n=n)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(S.family_seed(0, 3400))
    q, _ = torch.linalg.qr(torch.randn(n, n, device="cuda:0", dtype=torch.float64, generator=gen))
    d = torch.linspace(-1.0, 1.0, n, device="cuda:0", dtype=torch.float64)
    d = torch.where(d.abs() < 0.05, torch.sign(d + 1e-300) * 0.05, d)
    A = (q * d) @ q.T
    A = 0.5 * (A + A.T)
    del q
    reg = sdc.region("halfplane", shift=0.0, scale=1.0)
    o = sdc.opts(seed=5)
    r_on = h_on.split_sym(A, reg, o)
    assert r_on.status == sdc.SDC_OK and r_on.info["k_lead"] == int((d > 0).sum())
    r_off = h_off.split_sym(A, reg, o)
    same(r_on, r_off)
