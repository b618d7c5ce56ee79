"""Pins of the oracle's implicit repeated squaring (Alg. 3).

* the exact closed form for symmetric inputs (every R_j and the iteration
  count p);
* the squaring identity A_1^{-1} B_1 = (A_0^{-1} B_0)^2 of Sec. 3.2 on small,
  well-conditioned pencils (explicit inverses in the test only);
* the limit (A_p + B_p)^{-1} A_p -> projector onto the right deflating subspace
  of the eigenvalues outside the unit circle (Sec. 3.2), checked against an
  eigendecomposition from SciPy;
* the behaviour the paper reports for its experiments (Sec. 3.3.1).
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import sdc_synth as S
from oracle.irs import irs, norm1
from oracle.split import premap
from closed_form import irs_sym_closed_form

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_experiments.json")


@pytest.mark.parametrize("n,seed", [(16, 1), (48, 2), (128, S.family_seed(0))])
def test_irs_matches_symmetric_closed_form(n, seed):
    a, d, q = S.sym_problem(n, seed)
    a0, b0 = premap(a, np.eye(n), {"kind": "halfplane", "shift": 0.0, "scale": 1.0})
    res = irs(a0, b0, record=True)
    rs, p, conv, af, bf = irs_sym_closed_form(d, q)
    assert res.converged and conv
    assert res.p == p
    assert len(res.R_history) == len(rs)
    for rj, rc in zip(res.R_history, rs):
        assert np.allclose(rj, rc, rtol=0, atol=1e-12 * norm1(rc))
    # projector of the returned iterate equals Q diag(a/(a+b)) Q^T
    proj = np.linalg.solve(res.A + res.B, res.A)
    proj_cf = (q * (af / (af + bf))[None, :]) @ q.T
    assert np.allclose(proj, proj_cf, atol=1e-11)
    # ... which is the orthogonal projector onto the d > 0 eigenvectors
    pos = q[:, d > 0]
    assert np.allclose(proj, pos @ pos.T, atol=1e-10)


def test_c0_iteration_count_is_nine():
    """The c0 workload (n=128, |d| >= 0.05, split at 0) needs p = 9 by the
    closed form (2^{p-1} * ln(1.05/0.95) >= ln(1/sqrt(eps)))."""
    a, d, q = S.sym_problem(128, S.family_seed(0))
    _, p, conv, _, _ = irs_sym_closed_form(d, q)
    a0, b0 = premap(a, np.eye(128), {"kind": "halfplane", "shift": 0.0, "scale": 1.0})
    assert conv and p == 9 and irs(a0, b0).p == 9


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_one_step_squares_inverse_product(seed):
    rng = np.random.default_rng(seed)
    n = 6
    a = rng.standard_normal((n, n)) + 3 * np.eye(n)
    b = rng.standard_normal((n, n))
    res = irs(a, b, maxit=0)           # exactly one step: returns (A_1, B_1)
    assert not res.converged and res.p == 1
    lhs = np.linalg.solve(res.A, res.B)
    x = np.linalg.solve(a, b)
    assert np.allclose(lhs, x @ x, atol=1e-11 * np.abs(x @ x).max())
    res2 = irs(a, b, maxit=1)          # two steps: fourth power
    assert np.allclose(np.linalg.solve(res2.A, res2.B), np.linalg.matrix_power(x, 4),
                       atol=1e-10 * np.abs(np.linalg.matrix_power(x, 4)).max())


@pytest.mark.parametrize("seed", [21, 22, 23, 24])
def test_limit_is_outside_projector(seed):
    rng = np.random.default_rng(seed)
    n = 12
    # eigenvalues (of det(A - lambda B)) away from the unit circle
    mags = np.where(rng.uniform(size=n) < 0.5, rng.uniform(0.2, 0.7, n), rng.uniform(1.4, 4.0, n))
    lam = mags * np.where(rng.uniform(size=n) < 0.5, -1, 1)
    x = rng.standard_normal((n, n)) + 2 * np.eye(n)
    b = rng.standard_normal((n, n)) + 2 * np.eye(n)
    a = b @ x @ np.diag(lam) @ np.linalg.inv(x)        # B^{-1} A = X diag(lam) X^{-1}
    res = irs(a, b)
    assert res.converged
    proj = np.linalg.solve(res.A + res.B, res.A)
    w, vr = sla.eig(a, b)
    outside = np.abs(w) > 1
    p_true = (vr * outside[None, :]) @ np.linalg.inv(vr)
    assert np.allclose(proj, p_true.real, atol=1e-9)
    assert np.isclose(np.trace(proj), outside.sum(), atol=1e-8)


def _line_map(a):
    n = a.shape[0]
    return premap(a, np.eye(n), {"kind": "halfplane", "shift": 0.0, "scale": 1.0})


def test_paper_experiment_near_axis_converges_within_40():
    g = json.load(open(GOLDEN))["E3_near_imaginary_axis_n25"]
    a, _ = S.near_axis_problem(g["n"], seed=5, re_abs=g["real_part_abs"], box=g["imag_box"])
    res = irs(*_line_map(a), maxit=60)
    assert res.converged
    assert res.p <= g["max_iterations_to_converge"]
    # the count is close to the limit: eigenvalues 1e-10 from the line need ~38
    assert res.p >= 30


def test_paper_experiment_jordan_block_does_not_converge():
    g = json.load(open(GOLDEN))["E4_jordan_block_n32"]
    a = S.jordan_problem(g["n"], seed=6, jordan_value=g["jordan_value"])
    res = irs(*_line_map(a), maxit=g["iterations_plotted"])
    assert not res.converged


@pytest.mark.slow
def test_paper_experiments_random_normal_converge_at_similar_iterations():
    g = json.load(open(GOLDEN))
    ps = []
    for key, seed in (("E1_random_normal_n100", 3), ("E2_random_normal_n1000", 4)):
        n = g[key]["n"]
        a, ev = S.normal_random_problem(n, seed=seed, box=g[key]["eig_box"])
        res = irs(*_line_map(a))
        assert res.converged
        ps.append(res.p)
    # "convergence occurs at about the same iteration"
    assert abs(ps[0] - ps[1]) <= 4
