#!/usr/bin/env python3
"""Benchmark of the inverse-free spectral split on one MI355X.

Workload (default): one symmetric split of the clustered order-8192 problem
A = Q diag(d) Q^T (Q Haar; half of d in [-1, -0.01], half in [0.01, 1], 5%
per side within 1e-3 of +-0.01; seed 10113077 + 3000) at the half plane
Re z < 0, inputs resident in HBM.  One step is one FP64 split
(sdc_split_sym); the FP32+refine split of the same problem is timed beside
it (FP32 repeated squaring, FP64 convergence test, rank, block form and
refinement).  The other configurations (order-128 symmetric split, the
order-2048 pencil divide-and-conquer, 512 batched FP32+refine problems) are
measured briefly and reported in `other_configs`.

metric: split GFLOP/s = nominal split flops / wall time, with the paper's
cost model and LAPACK leading terms: (40/3 p + 16) n^3 for a symmetric split
with p repeated-squaring iterations, (40/3 (p_R + p_L) + 32) m^3 per pencil
step (refinement and retries not credited).

roofline: the tree-level trailing update of the QR (the kernel with the
largest time), timed per launch with HIP events on its stream
(sdc_profile_*), against the roof its algorithmic intensity puts it under.

cpu_baseline: the FP64 oracle (NumPy/LAPACK) on the host cores, splitting a
clustered symmetric problem of the same family at order 1536 (a bounded
sample), in the same GFLOP/s unit.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64_tflops": 78.6, "fp32_tflops": 157.3, "hbm_gbs": 8000.0}

# HBM traffic of the dominant kernel (the tree-level trailing update), from
# two rocprofv3 --pmc runs of `bench.py --steps 1 --warmup 0 --calibrate-copy
# --no-profile --no-extras --fp32-steps 1` (FETCH_SIZE, then WRITE_SIZE, KiB
# per dispatch): summed over the update's dispatches in the FP64 split, each
# counter scaled by what it reads for a plain 256 MiB device copy
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0), divided by the number of dispatches.  Valid only for the kernel sources it was measured
# on (their SHA-256 below); otherwise reported as null.
TRAFFIC = {"bytes_per_launch": 1598099948, "sha256": "38306c9eab3fe1d73d0f6b50df873936e5b9e4246de662133c7df75ef389af6f", "n": 8192, "note": "rocprofv3 FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 over the 10536 update dispatches of one FP64 split"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha():
    import hashlib
    hsh = hashlib.sha256()
    for f in ("qr_kernels.hip", "sdc_internal.hpp", "mfma.hpp", "rawbuf.hpp"):
        with open(os.path.join(ROOT, "paper_1011_3077_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def serve_main(args):
    """Serving benchmark: Poisson arrivals of split requests (sizes
    log-uniform in [nmin, nmax]; 70% symmetric, half of them FP32+refine; 30%
    nonsymmetric pencils, FP64) into the continuous-batching server, inputs
    resident in HBM; one JSON line per offered rate (--rate takes a
    comma-separated list) with p50/p99 latency, throughput, the queue at the
    end of the arrivals, and a check that sampled requests' results are
    bitwise those of single calls with the same arguments.  Requests reuse a
    pool of distinct problems (each request draws its own Gaussian seed)."""
    import numpy as np
    import torch
    import sdc_synth as S
    import paper_1011_3077_amd as P

    rng = np.random.default_rng(S.family_seed(4))
    pool_size = 24
    log(f"[serve] generating a pool of {pool_size} problems, n in [{args.nmin}, {args.nmax}]")
    pool = []
    for i in range(pool_size):
        n = int(round(math.exp(rng.uniform(math.log(args.nmin), math.log(args.nmax)))))
        u = rng.uniform()
        if u < 0.7:
            a, d, q = S.sym_problem(n, S.family_seed(4, i))
            prec = P.SDC_FP32_REFINE if u < 0.35 else P.SDC_FP64
            pool.append(dict(kind="sym", n=n, A=torch.from_numpy(a).to("cuda:0"), B=None,
                             reg=P.region("halfplane", shift=0.0, scale=1.0), prec=prec, k=int((d > 0).sum())))
        else:
            pb = S.pencil_problem(n, S.family_seed(4, i))
            pool.append(dict(kind="pencil", n=n, A=torch.from_numpy(pb["A"]).to("cuda:0"),
                             B=torch.from_numpy(pb["B"]).to("cuda:0"), reg=P.region(), prec=P.SDC_FP64,
                             k=int((np.abs(pb["lam"]) > 1).sum())))
    torch.cuda.synchronize()
    for rate in [float(x) for x in str(args.rate).split(",")]:
        arrivals = []
        t = 0.0
        while True:
            t += rng.exponential(1.0 / rate)
            if t > args.duration:
                break
            arrivals.append(t)
        log(f"[serve] {len(arrivals)} arrivals over {args.duration} s at {rate}/s")
        srv = P.Server(0, max_active=args.max_active)
        tickets = []
        t0 = time.perf_counter()
        for i, ta in enumerate(arrivals):
            dt = ta - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            q = pool[i % pool_size]
            tickets.append((srv.submit(q["A"], q["B"], q["reg"], P.opts(prec=q["prec"], seed=1000 + i)), q, i))
        queued_at_end = srv.stats()["pending"]
        bad = 0
        statuses = {}
        sample = {}
        for cnt, (tk, q, i) in enumerate(tickets):
            r = srv.wait(tk)
            if cnt % 50 == 49:
                log(f"[serve] {cnt + 1} of {len(tickets)} done")
            statuses[r.status] = statuses.get(r.status, 0) + 1
            if r.status != 0 or r.info["k_lead"] != q["k"]:
                bad += 1
            if i < 4 or i == len(tickets) - 1:
                sample[i] = r
        st = srv.stats()
        srv.close()
        # the sampled requests alone, through the single-problem entry points
        h = P.Handle(0)
        same = True
        for i, r in sample.items():
            q = pool[i % pool_size]
            o = P.opts(prec=q["prec"], seed=1000 + i)
            a = h.split_sym(q["A"], q["reg"], o) if q["kind"] == "sym" else h.split_pencil(q["A"], q["B"], q["reg"], o)
            same &= a.status == r.status and torch.equal(a.Q, r.Q) and torch.equal(a.Ahat, r.Ahat)
        h.close()
        wall = st["wall_ms"] / 1e3
        out = {
            "metric": "served split requests: p99 latency (submission to completion)",
            "value": st["p99_ms"],
            "unit": "ms",
            "higher_is_better": False,
            "n_gpus": 1,
            "p50_ms": st["p50_ms"],
            "mean_ms": st["mean_ms"],
            "max_ms": st["max_ms"],
            "throughput_req_s": st["completed"] / wall if wall > 0 else None,
            "nominal_gflops": st["nominal_flops"] / wall / 1e9 if wall > 0 else None,
            "offered_rate_req_s": rate,
            "requests": st["completed"],
            "queued_when_arrivals_ended": queued_at_end,
            "wrong_or_failed": bad,
            "statuses": {str(k): v for k, v in statuses.items()},
            "sampled_results_equal_single_calls": bool(same),
            "peak_active": st["peak_active"],
            "max_active": args.max_active or 64,
            "peak_bytes": st["peak_bytes"],
            "budget_bytes": st["budget_bytes"],
            "dtype": "f64 / f32+f64-refine",
            "data": "synthetic",
            "config": {"workload": f"Poisson {rate}/s for {args.duration} s, n log-uniform in "
                                   f"[{args.nmin}, {args.nmax}], 70% symmetric (half FP32+refine), 30% pencils",
                       "pool": pool_size},
        }
        print(json.dumps(out), flush=True)


def suite_main(args):
    """The other configurations of the measurement plan, one JSON line each
    (not the headline line): the order-128 symmetric split (latency, FP64,
    median of 10 after 3 warm-ups), 512 symmetric problems with n
    log-uniform in [32, 256] in one batched FP32+refine call (median of 3
    after 1 warm-up), and the clustered order-8192 symmetric split in FP64 and
    in FP32+refine (one warm-up, one timed run each).  Nominal flops follow
    the cost model of the headline metric for a symmetric split,
    (40/3 p + 16) n^3 with p repeated-squaring iterations (refinement not
    credited).  Single calls are timed by the library (info.ms, inside the C
    call, inputs resident in HBM); the batched call by the host clock around it."""
    import statistics
    import numpy as np
    import torch
    import sdc_synth as S
    import paper_1011_3077_amd as P

    h = P.Handle(0)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    half = P.region("halfplane", shift=0.0, scale=1.0)
    sym_flops = lambda n, p: (40.0 / 3.0 * p + 16.0) * float(n) ** 3

    def line(name, dtype, ms, flops, extra):
        out = {"metric": f"{name}: split GFLOP/s (nominal split flops / time)", "value": flops / ms / 1e6,
               "unit": "GFLOP/s", "ms": ms, "higher_is_better": True, "n_gpus": 1, "dtype": dtype,
               "data": "synthetic", "pct_peak": flops / ms / 1e6 / (
                   (PEAK["fp32_tflops"] if dtype.startswith("f32") else PEAK["fp64_tflops"]) * 1e3)}
        out.update(extra)
        print(json.dumps(out), flush=True)

    # order 128, FP64: latency
    a, d, q = S.sym_problem(128, S.family_seed(0))
    A = dev(a)
    runs = []
    for i in range(13):
        r = h.split_sym(A, half, P.opts(seed=1))
        if i >= 3:
            runs.append(r)
    ms = statistics.median(r.info["ms"] for r in runs)
    ok = all(r.status == 0 and r.info["k_lead"] == int((d > 0).sum()) for r in runs)
    line("symmetric split, order 128", "f64", ms, sym_flops(128, runs[0].info["iters_right"]),
         {"config": {"workload": "symmetric split of one order-128 problem at the half plane Re z < 0"},
          "iters": runs[0].info["iters_right"], "exact_rank": ok})

    # 512 batched, FP32 + refine
    sizes = S.batch_sizes(512, S.family_seed(2))
    probs = [S.sym_problem(n, S.family_seed(2, i)) for i, n in enumerate(sizes)]
    As = [dev(x) for x, _, _ in probs]
    regs = [half] * len(sizes)
    o = P.opts(prec=P.SDC_FP32_REFINE, seed=3)
    times = []
    for i in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = h.split_sym_batched(As, regs, o)
        torch.cuda.synchronize()
        if i >= 1:
            times.append((time.perf_counter() - t0) * 1e3)
    ms = statistics.median(times)
    flops = sum(sym_flops(n, r.info["iters_right"]) for n, r in zip(sizes, out))
    ok = all(r.status == 0 and r.info["k_lead"] == int((dd > 0).sum()) for r, (_, dd, _) in zip(out, probs))
    line("batched symmetric splits, 512 problems", "f32+f64-refine", ms, flops,
         {"config": {"workload": "512 symmetric problems, n log-uniform in [32, 256], one batched call, "
                                 "half plane Re z < 0", "n_min": min(sizes), "n_max": max(sizes)},
          "exact_rank": ok, "fp64_fallbacks": sum(r.info.get("fp64_fallback", 0) for r in out)})

    # order 8192 clustered, FP64 and FP32 + refine
    a, d, q = S.clustered_sym_problem(8192, S.family_seed(3))
    A = dev(a)
    del q
    for prec, dtype in ((P.SDC_FP64, "f64"), (P.SDC_FP32_REFINE, "f32+f64-refine")):
        h.split_sym(A, half, P.opts(prec=prec, seed=1))
        r = h.split_sym(A, half, P.opts(prec=prec, seed=1))
        line("symmetric split, clustered order 8192", dtype, r.info["ms"], sym_flops(8192, r.info["iters_right"]),
             {"config": {"workload": "clustered symmetric order-8192 problem (half the eigenvalues on each side "
                                     "of 0, 5% per side within 1e-3 of +-0.01), half plane Re z < 0"},
              "iters": r.info["iters_right"], "refine_rounds": r.info["refine_rounds"],
              "exact_rank": r.status == 0 and r.info["k_lead"] == int((d > 0).sum())})
    h.close()


def _roofline(P, stats, k, names, peak_tflops, traffic=None):
    """Roofline object of kernel k from its event-timed launches.  The bound
    is the lower of the two roofs at the kernel's algorithmic intensity
    (flops per byte of its minimum traffic): HBM below the machine balance,
    MFMA above it; the fraction of the MFMA peak is given either way.  The
    panel factorization is a sequential column loop in few workgroups and is
    set against the vector peak of its precision."""
    sd = stats[k]
    if sd["ms"] <= 0:
        return None
    secs = sd["ms"] / 1e3
    fl = sd["flops"] / secs / 1e12
    if k == P.KERNEL_PANEL:
        r = {"bound": "alu", "achieved": fl, "peak": peak_tflops, "unit": "TFLOP/s", "frac": fl / peak_tflops,
             "traffic": None}
    else:
        inten = sd["flops"] / max(sd["bytes"], 1.0)
        if inten < peak_tflops * 1e12 / (PEAK["hbm_gbs"] * 1e9):
            ach = sd["bytes"] / secs / 1e9
            r = {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                 "frac": ach / PEAK["hbm_gbs"], "traffic": None}
        else:
            r = {"bound": "mfma", "achieved": fl, "peak": peak_tflops, "unit": "TFLOP/s", "frac": fl / peak_tflops,
                 "traffic": None}
        r["intensity_flop_per_byte"] = inten
        r["mfma_achieved_tflops"] = fl
        r["mfma_frac"] = fl / peak_tflops
    if traffic is not None:
        r["traffic"] = traffic["bytes_per_launch"]
        r["traffic_note"] = traffic["note"]
    r["kernel"] = names[k]
    r["launches"] = sd["launches"]
    r["avg_launch_us"] = sd["ms"] * 1e3 / max(sd["launches"], 1)
    r["algorithmic_flops_per_launch"] = sd["flops"] / max(sd["launches"], 1)
    r["algorithmic_bytes_per_launch"] = sd["bytes"] / max(sd["launches"], 1)
    return r


def kernel_names(P, prec):
    t = "f32" if prec == "f32" else "f64"
    return {P.KERNEL_UPDATE: f"k_update (tree-level trailing update, MFMA {t})",
            P.KERNEL_PANEL: "k_panel (TSQR panel Householder)",
            P.KERNEL_GEMM: "k_gemm (MFMA)",
            P.KERNEL_LA: f"k_la (look-ahead update of the next panel, MFMA {t})"}


def sym_flops(n, p):
    """Nominal flops of one symmetric split with p repeated-squaring iterations."""
    return (40.0 / 3.0 * p + 16.0) * float(n) ** 3


def cpu_baseline_sym(n: int = 1536):
    """The FP64 oracle on the host's cores: split_sym of one clustered
    symmetric problem of the headline family at order n (a bounded sample).
    The same leg also runs the oracle's split of the order-128 problem that
    check_sym128 compares the library with (the only place the bench runs
    the oracle); it is returned beside the timing, untimed."""
    import sdc_synth as S
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([x.get("num_threads", 1) for x in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    a, d, _ = S.clustered_sym_problem(n, S.family_seed(3, 1))
    t0 = time.perf_counter()
    r = O.split_sym(a, {"kind": "halfplane", "shift": 0.0, "scale": 1.0}, seed=1)
    dt = time.perf_counter() - t0
    flops = sym_flops(n, r.p_right)
    a128, _, _ = S.sym_problem(128, S.family_seed(0))
    ref128 = O.split_sym(a128, {"kind": "halfplane", "shift": 0.0, "scale": 1.0}, seed=1)
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle split_sym (half plane Re z < 0) of one clustered symmetric order-{n} problem of "
                      f"the same family, p={r.p_right}, {dt:.1f} s, nominal {flops:.3e} flops",
            "seconds": dt}, {"sym128": (ref128.k, ref128.Q, ref128.A_hat)}


def other_configs(P, h):
    """The other configurations, measured briefly beside the headline line:
    the order-128 symmetric split (latency, FP64; median of 10 after 3
    warm-ups; its outputs are returned beside the figures so that
    check_sym128() can compare them with the oracle's split of the same
    problem once the CPU leg has run), the order-2048 pencil
    divide-and-conquer to blocks <= 64 (FP64; mean of 3 after 1 warm-up), and
    512 symmetric problems with n log-uniform in [32, 256] in one batched
    FP32+refine call (median of 3 after 1 warm-up).  Inputs resident in HBM;
    host clock around each call after a device synchronization."""
    import statistics
    import numpy as np
    import scipy.linalg as sla
    import torch
    import sdc_synth as S
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    half = P.region("halfplane", shift=0.0, scale=1.0)
    out = {}

    def timed(fn, reps, warm):
        res, ts = None, []
        for i in range(warm + reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = fn()
            torch.cuda.synchronize()
            if i >= warm:
                ts.append((time.perf_counter() - t0) * 1e3)
        return res, ts

    # order 128 symmetric, FP64 (latency)
    a, d, _ = S.sym_problem(128, S.family_seed(0))
    A = dev(a)
    r, ts = timed(lambda: h.split_sym(A, half, P.opts(seed=1)), 10, 3)
    k = r.info["k_lead"]
    ah = r.Ahat.cpu().numpy()
    ev = np.sort(np.concatenate([np.linalg.eigvalsh(ah[:k, :k]), np.linalg.eigvalsh(ah[k:, k:])]))
    ms = statistics.median(ts)
    fl = sym_flops(128, r.info["iters_right"])
    out["sym128_fp64"] = {
        "workload": "symmetric split of one order-128 problem at Re z < 0 (FP64)", "ms": ms,
        "gflops": fl / ms / 1e6, "pct_fp64_peak": fl / ms / 1e6 / (PEAK["fp64_tflops"] * 1e3),
        "iters": r.info["iters_right"], "k": k,
        "exact_rank": r.status == 0 and k == int((d > 0).sum()),
        "e21_rel": r.info["e21_rel"], "eig_abs_err_vs_construction": float(np.abs(ev - np.sort(d)).max()),
        "eig_abs_err_vs_oracle": None, "subspace_sin_vs_oracle": None, "oracle_k": None, "runs": len(ts)}
    sym128_out = (k, r.Q.cpu().numpy(), ev)
    log(f"[bench] order 128: {ms:.2f} ms")

    # order-2048 pencil divide-and-conquer to blocks <= 64, then the leaf
    # blocks' eigenvalues (the whole eigenvalue solve on the GPU), FP64
    pb = S.pencil_problem(2048, S.family_seed(1))
    A, B = dev(pb["A"]), dev(pb["B"])

    def c1_solve():
        rr = h.eig_dc(A, B, leaf_max=64, o=P.opts(seed=1))
        return rr, h.block_eigvals(rr[1], rr[2], rr[5], symmetric=False)

    (r, (wr, wi)), ts = timed(c1_solve, 3, 1)
    st, t, s_, ql, qr, starts, info = r
    got = np.sort_complex(wr.cpu().numpy() + 1j * wi.cpu().numpy())
    t, s_ = t.cpu().numpy(), s_.cpu().numpy()
    lap = np.sort_complex(np.concatenate([sla.eigvals(t[a0:a1, a0:a1], s_[a0:a1, a0:a1])
                                          for a0, a1 in zip(starts[:-1], starts[1:])]))
    want = np.sort_complex(pb["lam"].astype(complex))
    ms = statistics.mean(ts)
    out["pencil2048_dc_fp64"] = {
        "workload": "divide-and-conquer of the order-2048 real pencil (unit circle, then blocks <= 64) and the "
                    "blocks' eigenvalues, FP64",
        "ms": ms, "gflops": info["nominal_flops"] / ms / 1e6,
        "pct_fp64_peak": info["nominal_flops"] / ms / 1e6 / (PEAK["fp64_tflops"] * 1e3),
        "nominal_flops": info["nominal_flops"], "splits": info["splits"], "accepted": info["accepted"],
        "blocks": info["nblocks"], "unsplit": info["unsplit"],
        "nominal_flops_note": "every split attempt counted, including those that divided nothing; the leaf "
                              "eigenvalue solve is timed but not credited",
        "eig_rel_err_vs_construction": float(np.max(np.abs(got - want) / np.abs(want))),
        "eig_rel_err_lapack_on_same_blocks": float(np.max(np.abs(lap - want) / np.abs(want))), "runs": len(ts)}
    log(f"[bench] order-2048 pencil recursion: {ms:.1f} ms")
    del A, B

    # 512 batched symmetric problems, FP32 + refine
    sizes = S.batch_sizes(512, S.family_seed(2))
    probs = [S.sym_problem(n, S.family_seed(2, i)) for i, n in enumerate(sizes)]
    As = [dev(x) for x, _, _ in probs]
    o = P.opts(prec=P.SDC_FP32_REFINE, seed=3)
    res, ts = timed(lambda: h.split_sym_batched(As, [half] * len(sizes), o), 3, 1)
    ms = statistics.median(ts)
    fl = sum(sym_flops(n, r.info["iters_right"]) for n, r in zip(sizes, res))
    worst = 0.0
    for r, (_, dd, _) in zip(res, probs):
        k = r.info["k_lead"]
        ah = r.Ahat.cpu().numpy()
        ev = np.sort(np.concatenate([np.linalg.eigvalsh(ah[:k, :k]), np.linalg.eigvalsh(ah[k:, k:])]))
        worst = max(worst, float(np.abs(ev - np.sort(dd)).max()))
    out["batched512_fp32_refine"] = {
        "workload": "512 symmetric problems, n log-uniform in [32, 256], one batched FP32+refine call",
        "ms": ms, "gflops": fl / ms / 1e6, "pct_fp32_peak": fl / ms / 1e6 / (PEAK["fp32_tflops"] * 1e3),
        "exact_rank": all(r.status == 0 and r.info["k_lead"] == int((dd > 0).sum()) for r, (_, dd, _) in zip(res, probs)),
        "fp64_fallbacks": sum(r.info.get("fp64_fallback", 0) for r in res),
        "eig_abs_err_vs_construction": worst, "runs": len(ts)}
    log(f"[bench] 512 batched: {ms:.1f} ms")
    return out, sym128_out


def check_sym128(extras, sym128_out, refs):
    """The order-128 split against the oracle's split of the same problem
    (run by the CPU leg): eigenvalues of the two diagonal blocks, the angle
    between the two invariant subspaces, and the split point."""
    import numpy as np
    if not refs or "sym128" not in refs:
        return
    k, q, ev = sym128_out
    k_o, q_o, ah_o = refs["sym128"]
    ev_ref = np.sort(np.concatenate([np.linalg.eigvalsh(ah_o[:k, :k]), np.linalg.eigvalsh(ah_o[k:, k:])]))
    qs, qo = q[:, :k], q_o[:, :k]
    e = extras["sym128_fp64"]
    e.update({"eig_abs_err_vs_oracle": float(np.abs(ev - ev_ref).max()),
              "subspace_sin_vs_oracle": float(np.linalg.norm(qo - qs @ (qs.T @ qo), 2)), "oracle_k": int(k_o)})
    e["exact_rank"] = e["exact_rank"] and int(k_o) == k


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--fp32-steps", type=int, default=3, help="timed FP32+refine splits (at most --steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without per-launch events")
    ap.add_argument("--no-extras", action="store_true", help="skip the other configurations")
    ap.add_argument("--extras-only", action="store_true",
                    help="only the other configurations (order 128, the order-2048 pencil recursion and its leaf "
                         "eigenvalues, the 512-problem batch), one JSON line; for profiling them alone")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy first (reference kernel for HBM counters)")
    ap.add_argument("--serve", action="store_true", help="serving benchmark instead (see serve_main)")
    ap.add_argument("--suite", action="store_true",
                    help="the other measured configurations instead, one JSON line each (see suite_main)")
    ap.add_argument("--rate", type=str, default="4", help="--serve: Poisson arrival rate(s), requests/s, comma-separated")
    ap.add_argument("--duration", type=float, default=15.0, help="--serve: seconds of arrivals")
    ap.add_argument("--max-active", type=int, default=0, help="--serve: requests run at once (0: the server's default, 64)")
    ap.add_argument("--nmin", type=int, default=64)
    ap.add_argument("--nmax", type=int, default=2048)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the independent subproblems would shard across GPUs; a single large split would split its rows)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import sdc_synth as S
    import paper_1011_3077_amd as P

    if args.serve:
        return serve_main(args)
    if args.suite:
        return suite_main(args)
    if args.extras_only:
        h = P.Handle(0)
        print(json.dumps({"other_configs": other_configs(P, h)[0], "n_gpus": 1, "data": "synthetic"}), flush=True)
        h.close()
        return 0
    if args.calibrate_copy:
        x = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    n = args.n
    log(f"[bench] generating clustered symmetric order-{n} problem")
    a, d, q = S.clustered_sym_problem(n, S.family_seed(3))
    del q
    kexp = int((d > 0).sum())
    A = torch.from_numpy(a).to("cuda:0")
    del a
    half = P.region("halfplane", shift=0.0, scale=1.0)
    h = P.Handle(0)

    def step(prec):
        return h.split_sym(A, half, P.opts(prec=prec, seed=1))

    for i in range(args.warmup):
        r = step(P.SDC_FP64)
        log(f"[bench] warmup {i}: {r.info['ms']:.1f} ms, p {r.info['iters_right']}")
    torch.cuda.synchronize()
    # the headline: K FP64 splits, without per-launch events
    flops = 0.0
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = step(P.SDC_FP64)
        flops += sym_flops(n, r.info["iters_right"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r64 = r
    log(f"[bench] timed {args.steps} FP64 splits: {dt:.3f} s")
    # FP32 repeated squaring + FP64 refinement of the same problem
    k32 = max(1, min(args.fp32_steps, args.steps))
    step(P.SDC_FP32_REFINE)
    torch.cuda.synchronize()
    flops32 = 0.0
    t1 = time.perf_counter()
    for i in range(k32):
        r = step(P.SDC_FP32_REFINE)
        flops32 += sym_flops(n, r.info["iters_right"])
    torch.cuda.synchronize()
    dt32 = time.perf_counter() - t1
    r32 = r
    log(f"[bench] timed {k32} FP32+refine splits: {dt32:.3f} s")

    def accuracy(res):
        k = res.info["k_lead"]
        e21 = res.Ahat[k:, :k].abs().sum(dim=0).max().item() / A.abs().sum(dim=0).max().item()
        ah = res.Ahat.cpu().numpy()
        ev = np.sort(np.concatenate([np.linalg.eigvalsh(ah[:k, :k]), np.linalg.eigvalsh(ah[k:, k:])]))
        return {"exact_rank": res.status == 0 and k == kexp, "k": k, "iters": res.info["iters_right"],
                "e21_rel": e21, "eig_rel_err_vs_construction": float(np.abs(ev - np.sort(d)).max() / np.abs(d).max()),
                "refine_rounds": res.info["refine_rounds"], "fp64_fallback": res.info["fp64_fallback"]}

    acc64, acc32 = accuracy(r64), accuracy(r32)
    # per-kernel times: one more split of each precision with HIP events
    # around every launch of the hot kernels (on the launch's stream)
    stats64 = stats32 = None
    if not args.no_profile:
        h.profile_enable(True)
        step(P.SDC_FP64)
        torch.cuda.synchronize()
        stats64 = {k: h.profile_read(k) for k in (P.KERNEL_UPDATE, P.KERNEL_PANEL, P.KERNEL_GEMM, P.KERNEL_LA)}
        h.profile_enable(True)
        step(P.SDC_FP32_REFINE)
        torch.cuda.synchronize()
        stats32 = {k: h.profile_read(k) for k in (P.KERNEL_UPDATE, P.KERNEL_PANEL, P.KERNEL_GEMM, P.KERNEL_LA)}
        h.profile_enable(False)
    # the other configurations, timed before the CPU leg (whose host threads
    # would otherwise compete with the launching thread of the
    # latency-bound ones)
    extras = sym128_out = None
    if not args.no_extras:
        del A
        torch.cuda.empty_cache()
        extras, sym128_out = other_configs(P, h)
    h.close()
    # the CPU leg (the oracle on the host cores; it also gives the oracle's
    # reference for the order-128 check)
    cpu, refs = None, None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cpu, refs = cpu_baseline_sym()
    if extras is not None:
        check_sym128(extras, sym128_out, refs)

    value = flops / dt / 1e9
    value32 = flops32 / dt32 / 1e9
    roof = roof32 = None
    if stats64 is not None:
        names = kernel_names(P, "f64")
        tr = TRAFFIC if (TRAFFIC and TRAFFIC.get("sha256") == kernel_sources_sha() and TRAFFIC.get("n") == n) else None
        roof = _roofline(P, stats64, P.KERNEL_UPDATE, names, PEAK["fp64_tflops"], tr)
        roof32 = _roofline(P, stats32, P.KERNEL_UPDATE, kernel_names(P, "f32"), PEAK["fp32_tflops"])
    out = {
        "metric": "split GFLOP/s (nominal split flops / wall time), FP64; FP32+refine beside it",
        "value": value,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"symmetric split of one clustered order-{n} problem at Re z < 0 (half the eigenvalues "
                               f"on each side, 5% per side within 1e-3 of +-0.01), FP64", "n": n,
                   "generator": "sdc_synth.clustered_sym_problem seed 10113077+3000"},
        "pct_fp64_peak": value / (PEAK["fp64_tflops"] * 1e3),
        "nominal_flops_per_step": flops / args.steps,
        "accuracy": acc64,
        "fp32_refine": {"value": value32, "unit": "GFLOP/s", "steps": k32, "ms_per_step": dt32 / k32 * 1e3,
                        "pct_fp32_peak": value32 / (PEAK["fp32_tflops"] * 1e3),
                        "pct_fp64_peak": value32 / (PEAK["fp64_tflops"] * 1e3),
                        "speedup_vs_fp64": (dt / args.steps) / (dt32 / k32),
                        "dtype": "f32 squaring + f64 test, rank, block form and refinement",
                        "nominal_flops_note": "refinement flops not credited", "accuracy": acc32,
                        "roofline_update": roof32},
        "accuracy_note": "eigenvalues of the two diagonal blocks against the construction's (the FP64 oracle "
                         "at this order is the construction up to its own rounding); order 128 against the oracle",
        "kernels_fp64": None if stats64 is None else {kernel_names(P, "f64")[k]: v for k, v in stats64.items()},
        "kernel_timing": "HIP events around every launch of the hot kernels, in one extra split per precision",
        "roofline": roof,
        "other_configs": extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
