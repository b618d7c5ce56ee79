"""Served form (sdc_server_*): continuous batching, HBM-budget admission and
latency statistics, through the C ABI.

The property the served form must keep: a request's result is the same
whether it runs alone or in a mix with requests that arrive while it runs.
Every kernel works per problem from its own descriptor and every reduction
has a fixed order, so "the same" is checked bitwise against the
single-problem entry points with identical arguments.
"""
import threading
import time

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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def mix(sdc):
    """(A, B or None, region, opts, expected k) for a mixed request set."""
    half = sdc.region("halfplane", shift=0.0, scale=1.0)
    out = []
    for i, n in enumerate((64, 100, 200, 333)):
        a, d, q = S.sym_problem(n, S.family_seed(4, i))
        out.append((a, None, half, sdc.opts(seed=20 + i), int((d > 0).sum())))
    for i, n in enumerate((128, 256)):
        a, d, q = S.sym_problem(n, S.family_seed(4, 10 + i))
        out.append((a, None, half, sdc.opts(prec=sdc.SDC_FP32_REFINE, seed=30 + i), int((d > 0).sum())))
    for i, n in enumerate((48, 150, 96)):
        p = S.pencil_problem(n, S.family_seed(4, 20 + i))
        out.append((p["A"], p["B"], sdc.region(), sdc.opts(seed=40 + i), int((np.abs(p["lam"]) > 1).sum())))
    return out


def alone(handle, a, b, reg, o):
    if b is None:
        return handle.split_sym(dev(a), reg, o)
    return handle.split_pencil(dev(a), dev(b), reg, o)


def same(x, y):
    for u, v in ((x.Q, y.Q), (x.Ahat, y.Ahat), (x.QL, y.QL), (x.Bhat, y.Bhat)):
        if u is None or v is None:
            assert u is None and v is None
        else:
            assert torch.equal(u, v)


def test_server_mix_equals_alone(handle, sdc):
    reqs = mix(sdc)
    print("CASE server mix", len(reqs), flush=True)
    solo = [alone(handle, a, b, reg, o) for a, b, reg, o, k in reqs]
    srv = sdc.Server(0)
    try:
        tickets = []
        # arrivals in three waves while earlier requests are on the GPU
        for wave in (reqs[:3], reqs[3:6], reqs[6:]):
            for a, b, reg, o, k in wave:
                tickets.append(srv.submit(dev(a), None if b is None else dev(b), reg, o))
            time.sleep(0.02)
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    print("stats", st, flush=True)
    for (a, b, reg, o, k), r, s1 in zip(reqs, res, solo):
        assert r.status == 0 and s1.status == 0
        assert r.info["k_lead"] == k == s1.info["k_lead"]
        same(r, s1)
    assert st["completed"] == st["submitted"] == len(reqs) and st["failed"] == 0
    assert st["peak_active"] >= 2
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert st["nominal_flops"] > 0


def test_server_budget_admission(handle, sdc):
    print("CASE server budget", flush=True)
    half = sdc.region("halfplane", shift=0.0, scale=1.0)
    probs = [S.sym_problem(192, S.family_seed(4, 50 + i)) for i in range(6)]
    probe = sdc.Server(0)
    try:
        probe.wait(probe.submit(dev(probs[0][0]), None, half, sdc.opts(seed=1)))
        one = probe.stats()["peak_bytes"]
    finally:
        probe.close()
    assert one > 0
    srv = sdc.Server(0, budget_bytes=int(2.5 * one))
    try:
        ts = [srv.submit(dev(a), None, half, sdc.opts(seed=1)) for a, d, q in probs]
        res = [srv.wait(t) for t in ts]
        st = srv.stats()
    finally:
        srv.close()
    for (a, d, q), r in zip(probs, res):
        assert r.status == 0 and r.info["k_lead"] == int((d > 0).sum())
    assert st["peak_bytes"] <= int(2.5 * one)
    assert st["peak_active"] <= 2


def test_server_oversize_request_fails_cleanly(handle, sdc):
    print("CASE server oversize", flush=True)
    a, d, q = S.sym_problem(128, S.family_seed(4, 60))
    srv = sdc.Server(0, budget_bytes=1 << 16)
    try:
        t = srv.submit(dev(a), None, sdc.region("halfplane"), sdc.opts())
        r = srv.wait(t)
        assert r.status == sdc.SDC_ERR_NOMEM
        with pytest.raises(sdc.SdcError):
            srv.poll(t)  # released
    finally:
        srv.close()


def test_server_poll_and_threads(handle, sdc):
    """Submissions from several host threads; poll until done."""
    print("CASE server threads", flush=True)
    half = sdc.region("halfplane", shift=0.0, scale=1.0)
    probs = [S.sym_problem(n, S.family_seed(4, 70 + i)) for i, n in enumerate((40, 80, 120, 160))]
    srv = sdc.Server(0)
    tickets = [None] * len(probs)
    inputs = [dev(a) for a, d, q in probs]

    def go(i):
        tickets[i] = srv.submit(inputs[i], None, half, sdc.opts(seed=i))

    try:
        th = [threading.Thread(target=go, args=(i,)) for i in range(len(probs))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        res = [None] * len(probs)
        deadline = time.time() + 60
        while any(r is None for r in res) and time.time() < deadline:
            for i, t in enumerate(tickets):
                if res[i] is None:
                    res[i] = srv.poll(t)
            time.sleep(0.005)
    finally:
        srv.close()
    for (a, d, q), r in zip(probs, res):
        assert r is not None and r.status == 0 and r.info["k_lead"] == int((d > 0).sum())


def test_server_two_waiters_on_one_ticket(handle, sdc):
    """Two threads wait on the same ticket: one receives the result, the
    other returns SDC_ERR_INVALID instead of blocking."""
    import ctypes as C
    print("CASE server two waiters", flush=True)
    a, d, q = S.sym_problem(90, S.family_seed(4, 91))
    srv = sdc.Server(0)
    try:
        t = srv.submit(dev(a), None, sdc.region("halfplane", shift=0.0, scale=1.0), sdc.opts(seed=3))
        out = [None, None]

        def waiter(i):
            st, info = C.c_int(), sdc.Info()
            out[i] = sdc.lib.sdc_server_wait(srv._s, t, C.byref(st), C.byref(info))

        th = [threading.Thread(target=waiter, args=(i,)) for i in range(2)]
        for x in th:
            x.start()
        for x in th:
            x.join(timeout=60)
        assert not any(x.is_alive() for x in th)
        assert sorted(out) == [sdc.SDC_ERR_INVALID, sdc.SDC_OK]
        srv._live.pop(t, None)
    finally:
        srv.close()
