"""Pins of the oracle's FP64 Newton refinement of a symmetric split.

The refinement is not in the paper; these checks tie it to what the
mathematics fixes: starting from a rotated copy of the exact invariant
subspace, it must return that subspace (eigh of the construction), converge
quadratically, and keep Q orthogonal."""
import numpy as np
import scipy.linalg as sla

import sdc_synth as S
from oracle.refine import refine_sym
from oracle.irs import norm1


def exact_split(n, seed):
    a, d, q = S.sym_problem(n, seed)
    order = np.argsort(-d)  # outside (d > 0) first
    q, d = q[:, order], d[order]
    k = int((d > 0).sum())
    return a, d, q, k


def rotated(q, k, scale, seed):
    rng = np.random.default_rng(seed)
    n = q.shape[0]
    y = scale * rng.standard_normal((n - k, k))
    s = np.block([[np.zeros((k, k)), -y.T], [y, np.zeros((n - k, n - k))]])
    return q @ sla.expm(s)


def sin_theta(u, v):
    # largest principal angle sine between orthonormal bases
    r = v - u @ (u.T @ v)
    return np.linalg.norm(r, 2)


def test_recovers_exact_subspace_quadratically():
    a, d, q, k = exact_split(96, S.family_seed(0, 41))
    q0 = rotated(q, k, 1e-4, 1)
    q1, ah, hist = refine_sym(a, q0, k, tol=1e-15, rounds=4)
    assert hist[0] > 1e-6
    assert hist[1] <= 10 * hist[0] ** 2 / 0.05 + 1e-15  # Newton: e_1 = O(e_0^2 / gap)
    assert hist[-1] <= 1e-14
    assert sin_theta(q[:, :k], q1[:, :k]) <= 1e-13
    assert np.abs(q1.T @ q1 - np.eye(96)).max() <= 1e-14
    ev = np.sort(np.concatenate([np.linalg.eigvalsh(ah[:k, :k]), np.linalg.eigvalsh(ah[k:, k:])]))
    assert np.abs(ev - np.sort(d)).max() <= 1e-14


def test_exact_input_is_a_fixed_point():
    a, d, q, k = exact_split(40, S.family_seed(0, 42))
    q1, ah, hist = refine_sym(a, q, k, tol=1e-13)
    assert len(hist) == 1 and hist[0] <= 1e-13
    assert np.array_equal(q1, q)


def test_larger_rotation_still_converges():
    a, d, q, k = exact_split(64, S.family_seed(0, 43))
    q0 = rotated(q, k, 3e-3, 2)
    q1, ah, hist = refine_sym(a, q0, k, tol=1e-14, rounds=4)
    assert hist[-1] <= 1e-14
    assert sin_theta(q[:, :k], q1[:, :k]) <= 1e-12
    assert norm1(ah[k:, :k]) <= 1e-14 * norm1(a)
