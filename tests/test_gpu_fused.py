"""Persistent fused repeated squaring for batches of small problems (one
launch running every iteration of every side, one workgroup per side, with
an autotuner choosing it or the per-iteration launches per size bucket).

SKIPPED: the first GPU run of this file (its first case, a mixed batch of
orders 1 to 256 in FP64) hung, with no fault reported, and the cause was not
found by reading the code, so the fused kernel and its autotuner were taken
out of the library; the per-iteration launches are the only path.  The cases
below are kept as they were run, for a later design of the fused launch.
"""
import os

import numpy as np
import pytest

import sdc_synth as S

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="the fused repeated-squaring kernel hung on its first GPU run (cause not "
                                      "found) and was taken out of the library")]


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


class forced_path:
    def __init__(self, path):
        self.path = path

    def __enter__(self):
        self.old = os.environ.get("SDC_IRS_PATH")
        os.environ["SDC_IRS_PATH"] = self.path

    def __exit__(self, *a):
        if self.old is None:
            os.environ.pop("SDC_IRS_PATH", None)
        else:
            os.environ["SDC_IRS_PATH"] = self.old


def same(r1, r2):
    assert r1.status == r2.status
    for key in ("k_lead", "n_inside", "iters_right", "iters_left", "attempts", "refine_rounds", "k_rho"):
        assert r1.info[key] == r2.info[key], key
    assert torch.equal(r1.Q, r2.Q) and torch.equal(r1.Ahat, r2.Ahat)


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_fused_batch_equals_lockstep_bitwise(handle, sdc, prec):
    sizes = [200, 1, 37, 256, 64, 2, 129, 96, 33]
    mats = [S.sym_problem(n, S.family_seed(2, 700 + i))[0] for i, n in enumerate(sizes)]
    regs = [sdc.region("halfplane", shift=0.0, scale=1.0)] * len(sizes)
    o = sdc.opts(prec=sdc.SDC_FP32_REFINE if prec == "fp32_refine" else sdc.SDC_FP64, seed=21)
    with forced_path("lockstep"):
        a = handle.split_sym_batched([dev(m) for m in mats], regs, o)
    with forced_path("fused"):
        b = handle.split_sym_batched([dev(m) for m in mats], regs, o)
    for r1, r2 in zip(a, b):
        same(r1, r2)


def test_fused_pencils_and_divide_and_conquer_equal_lockstep(handle, sdc):
    n = 300
    p = S.pencil_problem(n, S.family_seed(1, 77))
    outs = []
    for path in ("lockstep", "fused"):
        with forced_path(path):
            outs.append(handle.eig_dc(dev(p["A"]), dev(p["B"]), leaf_max=32, o=sdc.opts(seed=4)))
    (s1, t1, u1, l1, q1, b1, i1), (s2, t2, u2, l2, q2, b2, i2) = outs
    assert s1 == s2 == 0 and b1 == b2
    for x, y in ((t1, t2), (u1, u2), (l1, l2), (q1, q2)):
        assert torch.equal(x, y)
