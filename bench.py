#!/usr/bin/env python3
"""Benchmark of the inverse-free spectral divide-and-conquer on one MI355X.

Workload (default, `pencil2048`): the order-2048 real pencil A = U T V^T,
B = U S V^T (T, S upper triangular, |lambda| log-uniform in [0.1, 10],
U, V Haar, seed 10113077 + 1000), split at the unit circle and then
recursively to diagonal blocks of order <= 64, in FP64.  One step is one
whole divide-and-conquer run (sdc_eig_dc) on inputs already resident in HBM.

metric: split GFLOP/s = nominal split flops / wall time, with the nominal
flops of every split step counted by the paper's cost model with LAPACK
leading terms: (40/3 (p_R + p_L) + 32) m^3 for a pencil step of order m with
p_R, p_L repeated-squaring iterations (refinement and retries not credited).

roofline: the kernel with the largest total time in the timed region, timed
per launch with HIP events on its stream (sdc_profile_*), against its bound:
the tree-level trailing update is a dense contraction with 8 flop/byte in
FP64 (4 R nb ntr flops on 2 R ntr words of 8 bytes, nb = 32), below the
chip's 9.8 flop/byte balance, so its bound is HBM bandwidth; the panel
factorization is vector-ALU work.

cpu_baseline: the FP64 oracle (NumPy/LAPACK) on the host cores, running the
top split of the same pencil family at order 1024 (a bounded sample; about
1/8 of the order-2048 split's flops), in the same GFLOP/s unit.
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
# two rocprofv3 --pmc runs of `bench.py --steps 1 --warmup 0 --calibrate-copy`
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch): summed over the update's
# dispatches in the step, each counter scaled by what it reads for a plain
# 256 MiB device copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0), divided by the
# number of dispatches.  Valid only for the kernel sources it was measured
# on (their SHA-256 below); otherwise reported as null.
TRAFFIC = {"bytes_per_launch": 104149743, "sha256": "8da58b698a64b6f50779c27be1f16b1f1c636739e8a02126cbd01fe818b79e80", "n": 2048, "leaf": 64, "note": "rocprofv3 FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 over 6831 update dispatches of one step"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha():
    import hashlib
    hsh = hashlib.sha256()
    for f in ("qr_kernels.hip", "sdc_internal.hpp", "mfma.hpp"):
        with open(os.path.join(ROOT, "paper_1011_3077_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def cpu_baseline(n: int = 1024):
    import numpy as np
    import sdc_synth as S
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([x.get("num_threads", 1) for x in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    p = S.pencil_problem(n, S.family_seed(1, 500))
    t0 = time.perf_counter()
    r = O.split_pencil(p["A"], p["B"], {"kind": "unit_disk"}, seed=1)
    dt = time.perf_counter() - t0
    flops = (40.0 / 3.0 * (r.p_right + r.p_left) + 32.0) * n ** 3
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle split_pencil (unit circle) of one order-{n} pencil of the same family, "
                      f"p_R={r.p_right}, p_L={r.p_left}, {dt:.1f} s, nominal {flops:.3e} flops",
            "seconds": dt}


def serve_main(args):
    """Serving benchmark: Poisson arrivals of split requests (sizes
    log-uniform in [nmin, nmax]; 70% symmetric, half of them FP32+refine; 30%
    nonsymmetric pencils, FP64) into the continuous-batching server, inputs
    resident in HBM; reports p50/p99 latency and throughput.  Requests reuse a
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
    arrivals = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / args.rate)
        if t > args.duration:
            break
        arrivals.append(t)
    log(f"[serve] {len(arrivals)} arrivals over {args.duration} s at {args.rate}/s")
    srv = P.Server(0)
    tickets = []
    t0 = time.perf_counter()
    for i, ta in enumerate(arrivals):
        dt = ta - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        q = pool[i % pool_size]
        tickets.append((srv.submit(q["A"], q["B"], q["reg"], P.opts(prec=q["prec"], seed=1000 + i)), q))
    bad = 0
    statuses = {}
    for tk, q in tickets:
        r = srv.wait(tk)
        statuses[r.status] = statuses.get(r.status, 0) + 1
        if r.status != 0 or r.info["k_lead"] != q["k"]:
            bad += 1
    st = srv.stats()
    srv.close()
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
        "offered_rate_req_s": args.rate,
        "requests": st["completed"],
        "wrong_or_failed": bad,
        "statuses": {str(k): v for k, v in statuses.items()},
        "peak_active": st["peak_active"],
        "peak_bytes": st["peak_bytes"],
        "budget_bytes": st["budget_bytes"],
        "dtype": "f64 / f32+f64-refine",
        "data": "synthetic",
        "config": {"workload": f"Poisson {args.rate}/s for {args.duration} s, n log-uniform in "
                               f"[{args.nmin}, {args.nmax}], 70% symmetric (half FP32+refine), 30% pencils",
                   "pool": pool_size},
    }
    print(json.dumps(out))


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without per-launch events")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy first (reference kernel for HBM counters)")
    ap.add_argument("--serve", action="store_true", help="serving benchmark instead (see serve_main)")
    ap.add_argument("--suite", action="store_true",
                    help="the other measured configurations instead, one JSON line each (see suite_main)")
    ap.add_argument("--rate", type=float, default=4.0, help="--serve: Poisson arrival rate, requests/s")
    ap.add_argument("--duration", type=float, default=15.0, help="--serve: seconds of arrivals")
    ap.add_argument("--nmin", type=int, default=64)
    ap.add_argument("--nmax", type=int, default=2048)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the independent subproblems would shard across GPUs; a single large split would split its rows)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import scipy.linalg as sla
    import torch
    import sdc_synth as S
    import paper_1011_3077_amd as P

    if args.serve:
        return serve_main(args)
    if args.suite:
        return suite_main(args)
    if args.calibrate_copy:
        x = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    n, leaf = args.n, args.leaf
    log(f"[bench] generating order-{n} pencil")
    pb = S.pencil_problem(n, S.family_seed(1))
    A = torch.from_numpy(pb["A"]).to("cuda:0")
    B = torch.from_numpy(pb["B"]).to("cuda:0")
    h = P.Handle(0)
    o = P.opts(seed=1)

    def step():
        return h.eig_dc(A, B, leaf_max=leaf, o=o)

    for i in range(args.warmup):
        r = step()
        log(f"[bench] warmup {i}: {r[-1]['ms']:.1f} ms, splits {r[-1]['splits']}")
    torch.cuda.synchronize()
    # throughput: the timed steps without per-launch events
    flops = 0.0
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = step()
        flops += r[-1]["nominal_flops"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"[bench] timed {args.steps} steps: {dt:.3f} s")
    # per-kernel times: the same steps again with HIP events around every
    # launch of the hot kernels (on the launch's stream); the events add
    # host calls and GPU packets to every launch (about a fifth of the step
    # time), so they stay out of the throughput pass above
    stats = {}
    dt_prof = None
    if not args.no_profile:
        h.profile_enable(True)
        t1 = time.perf_counter()
        for i in range(args.steps):
            step()
        torch.cuda.synchronize()
        dt_prof = time.perf_counter() - t1
        log(f"[bench] profiled {args.steps} steps: {dt_prof:.3f} s")
        stats = {k: h.profile_read(k) for k in (P.KERNEL_UPDATE, P.KERNEL_PANEL, P.KERNEL_GEMM, P.KERNEL_LA)}
        h.profile_enable(False)

    # accuracy of the last step against the construction (outside the timed region)
    st, t, s, ql, qr, starts, info = r
    t, s = t.cpu().numpy(), s.cpu().numpy()
    ev = []
    for a0, a1 in zip(starts[:-1], starts[1:]):
        ev.append(sla.eigvals(t[a0:a1, a0:a1], s[a0:a1, a0:a1]))
    got = np.sort_complex(np.concatenate(ev))
    want = np.sort_complex(pb["lam"].astype(complex))
    eig_err = float(np.max(np.abs(got - want) / np.abs(want)))
    h.close()

    value = flops / dt / 1e9
    names = {P.KERNEL_UPDATE: "k_update (tree-level trailing update, MFMA f64)",
             P.KERNEL_PANEL: "k_panel (TSQR panel Householder)",
             P.KERNEL_GEMM: "k_gemm (MFMA f64)",
             P.KERNEL_LA: "k_la (look-ahead update of the next panel, MFMA f64)"}
    def roofline(k):
        """Roofline object of kernel k from its event-timed launches: the
        panel factorization against the FP64 vector peak (it is a sequential
        column loop in few workgroups), the MFMA kernels against HBM or FP64
        MFMA by their algorithmic intensity."""
        sd = stats[k]
        if sd["ms"] <= 0:
            return None
        secs = sd["ms"] / 1e3
        if k == P.KERNEL_PANEL:
            ach = sd["flops"] / secs / 1e12
            r = {"bound": "alu", "achieved": ach, "peak": PEAK["fp64_tflops"], "unit": "TFLOP/s",
                 "frac": ach / PEAK["fp64_tflops"], "traffic": None}
        else:
            inten = sd["flops"] / max(sd["bytes"], 1.0)
            if inten < PEAK["fp64_tflops"] * 1e12 / (PEAK["hbm_gbs"] * 1e9):
                ach = sd["bytes"] / secs / 1e9
                r = {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                     "frac": ach / PEAK["hbm_gbs"], "traffic": None}
            else:
                ach = sd["flops"] / secs / 1e12
                r = {"bound": "mfma", "achieved": ach, "peak": PEAK["fp64_tflops"], "unit": "TFLOP/s",
                     "frac": ach / PEAK["fp64_tflops"], "traffic": None}
        if k == P.KERNEL_UPDATE and TRAFFIC and TRAFFIC.get("sha256") == kernel_sources_sha() \
                and TRAFFIC.get("n") == n and TRAFFIC.get("leaf") == leaf:
            r["traffic"] = TRAFFIC["bytes_per_launch"]
            r["traffic_note"] = TRAFFIC["note"]
        r["kernel"] = names[k]
        r["launches"] = sd["launches"]
        r["avg_launch_us"] = sd["ms"] * 1e3 / max(sd["launches"], 1)
        r["algorithmic_flops_per_launch"] = sd["flops"] / max(sd["launches"], 1)
        r["algorithmic_bytes_per_launch"] = sd["bytes"] / max(sd["launches"], 1)
        return r

    roof = roof_upd = None
    if not args.no_profile:
        # dominant = largest summed launch time (the panel and the update
        # kernels run on two streams, so their times overlap); the bulk
        # HBM-bound update is reported beside it when it is not the dominant
        dom = max(stats, key=lambda k: stats[k]["ms"])
        roof = roofline(dom)
        if dom != P.KERNEL_UPDATE:
            roof_upd = roofline(P.KERNEL_UPDATE)
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline()
    out = {
        "metric": "split GFLOP/s (nominal split flops / wall time), FP64",
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
        "config": {"workload": f"divide-and-conquer of an order-{n} real pencil (unit circle, then recursion "
                               f"to blocks <= {leaf}), FP64", "n": n, "leaf_max": leaf,
                   "generator": "sdc_synth.pencil_problem seed 10113077+1000"},
        "pct_fp64_peak": value / (PEAK["fp64_tflops"] * 1e3),
        "nominal_flops_per_step": flops / args.steps,
        "splits_per_step": info["splits"],
        "blocks": info["nblocks"],
        "eig_rel_err_vs_construction": eig_err,
        "kernels": {names[k]: v for k, v in stats.items()},
        "kernel_timing": "HIP events around every launch, in a second pass of the same steps "
                         "(ms_per_step of that pass: %s)" % (None if dt_prof is None else round(dt_prof / args.steps * 1e3, 1)),
        "roofline": roof,
        "roofline_update": roof_upd,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
