"""bench.py on the CPU: more than one GPU is refused with a message and exit
status 2, before anything touches a device; the order-128 comparison with
the oracle, which runs after the CPU leg."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus 2 is not supported" in r.stderr
    assert r.stdout == ""


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_order128_check_after_the_cpu_leg():
    """The order-128 figures are timed before the CPU leg and compared with
    the oracle's split afterwards: the comparison fields stay null without
    the leg, are filled from it (eigenvalues of the two diagonal blocks, the
    subspace angle, the split point), and a split point that differs from
    the oracle's clears exact_rank."""
    import numpy as np
    bench = _bench_module()
    rng = np.random.default_rng(7)
    n, k = 12, 5
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = np.concatenate([np.linspace(1.0, 2.0, k), np.linspace(-2.0, -1.0, n - k)])
    ah = np.diag(d)
    ev = np.sort(d)
    fresh = lambda: {"sym128_fp64": {"exact_rank": True, "eig_abs_err_vs_oracle": None,
                                     "subspace_sin_vs_oracle": None, "oracle_k": None}}
    extras = fresh()
    bench.check_sym128(extras, (k, q, ev), None)
    assert extras["sym128_fp64"]["eig_abs_err_vs_oracle"] is None and extras["sym128_fp64"]["exact_rank"]
    extras = fresh()
    bench.check_sym128(extras, (k, q, ev), {"sym128": (k, q, ah)})
    e = extras["sym128_fp64"]
    assert e["oracle_k"] == k and e["exact_rank"]
    assert e["eig_abs_err_vs_oracle"] <= 1e-15 and e["subspace_sin_vs_oracle"] <= 1e-12
    # a rotated trailing block leaves the leading subspace, and the angle, unchanged
    q2 = q.copy()
    q2[:, k:] = q2[:, k:] @ np.linalg.qr(rng.standard_normal((n - k, n - k)))[0]
    extras = fresh()
    bench.check_sym128(extras, (k, q2, ev), {"sym128": (k, q, ah)})
    assert extras["sym128_fp64"]["subspace_sin_vs_oracle"] <= 1e-12
    extras = fresh()
    bench.check_sym128(extras, (k, q, ev), {"sym128": (k + 1, q, ah)})
    assert not extras["sym128_fp64"]["exact_rank"] and extras["sym128_fp64"]["oracle_k"] == k + 1
