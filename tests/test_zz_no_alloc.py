"""sdc_split_sym_noalloc (the entry point for callers that cannot allocate
device memory) against sdc_split_sym: the same kernels in the same order on
preallocated static memory, so the results are bitwise equal.  Two calls in
a row share the device's scratch; the second is smaller and must not see
the first one's leftovers.  Sizes beyond the stated maximum are refused."""
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
def handle(sdc):
    h = sdc.Handle(0)
    yield h
    h.close()


def cm(x):
    """Column-major device copy: the tensor holding x's transpose."""
    return torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda:0")


def run_pair(handle, sdc, a, reg, o):
    n = a.shape[0]
    print("CASE noalloc n", n, "prec", o.prec, flush=True)
    ref = handle.split_sym(torch.from_numpy(a).to("cuda:0"), reg, o)
    A = cm(a)
    Q = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda:0")
    Ah = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda:0")
    st, info = handle.split_sym_noalloc(A, Q, Ah, reg, o)
    assert st == ref.status
    for key in ("k_lead", "n_inside", "iters_right", "attempts", "refine_rounds", "k_rho", "fp64_fallback"):
        assert info[key] == ref.info[key], key
    assert info["e21_rel"] == ref.info["e21_rel"]
    # Q, Ahat are the transposes' memory: compare as the same column-major arrays
    assert torch.equal(Q.t(), ref.Q) and torch.equal(Ah.t(), ref.Ahat)
    return info


def test_noalloc_equals_split_sym_twice_second_smaller(handle, sdc):
    reg = sdc.region("halfplane", shift=0.0, scale=1.0)
    a1, d1, _ = S.sym_problem(700, S.family_seed(0, 4700))
    a2, d2, _ = S.sym_problem(130, S.family_seed(0, 4130))
    i1 = run_pair(handle, sdc, a1, reg, sdc.opts(seed=11))
    i2 = run_pair(handle, sdc, a2, reg, sdc.opts(seed=12))
    assert i1["k_lead"] == int((d1 > 0).sum()) and i2["k_lead"] == int((d2 > 0).sum())


def test_noalloc_fp32_refine_and_largest_order(handle, sdc):
    reg = sdc.region("halfplane", shift=0.0, scale=1.0)
    n = sdc.NOALLOC_MAX_N
    a, d, _ = S.sym_problem(n, S.family_seed(0, 5000 + n))
    info = run_pair(handle, sdc, a, reg, sdc.opts(prec=sdc.SDC_FP32_REFINE, seed=2))
    assert info["k_lead"] == int((d > 0).sum())
    a2, d2, _ = S.sym_problem(64, S.family_seed(0, 5064))
    run_pair(handle, sdc, a2, reg, sdc.opts(seed=3))


def test_noalloc_refuses_orders_beyond_the_maximum(handle, sdc):
    n = sdc.NOALLOC_MAX_N + 1
    print("CASE noalloc refuse", n, flush=True)
    t = torch.zeros((n, n), dtype=torch.float64, device="cuda:0")
    with pytest.raises(sdc.SdcError, match="INVALID"):
        handle.split_sym_noalloc(t, t.clone(), t.clone(), sdc.region("halfplane", shift=0.0, scale=1.0))
