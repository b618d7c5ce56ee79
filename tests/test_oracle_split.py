"""Pins of the oracle's split step (Alg. 4 / Alg. 6 with the map of Sec. 3.3).

* split-point search against a brute-force loop recomputation (tiny n);
* the Moebius map against the eigenvalues SciPy computes for the mapped pencil;
* symmetric splits: rank equal to #(d < shift) by construction, E21 at
  rounding level, block eigenvalues equal to the construction, the invariant
  subspace equal to the known eigenvectors, the Hermitian off-block lemma;
* pencils: rank equal to #(|lambda| < 1) by construction, block eigenvalues
  equal to the construction, and for outside-first triangular factors the
  computed subspaces equal the known deflating subspaces exactly;
* failure paths: no split, non-convergence, a bad random draw retried.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import sdc_synth as S
from oracle.split import (premap, split_search, split_sym, split_pencil, rank_from_rho,
                          OK, NOT_CONVERGED, NO_SPLIT)
from oracle.irs import irs, norm1

HALF0 = {"kind": "halfplane", "shift": 0.0, "scale": 1.0}


def _sin_theta(x, y):
    """Largest sine of the principal angles between range(x) and range(y)."""
    qx, _ = np.linalg.qr(x)
    qy, _ = np.linalg.qr(y)
    resid = qy - qx @ (qx.T @ qy)
    return float(np.linalg.norm(resid, 2))


@pytest.mark.parametrize("n", [2, 3, 9, 24])
def test_split_search_brute_force(n):
    rng = np.random.default_rng(n)
    ah = rng.standard_normal((n, n))
    bh = rng.standard_normal((n, n))
    na, nb = 3.7, 1.9
    k, e, ev = split_search(ah, na, bh, nb)
    brute = []
    for kk in range(1, n):
        best_a = 0.0
        best_b = 0.0
        for c in range(kk):
            sa = 0.0
            sb = 0.0
            for i in range(kk, n):
                sa += abs(ah[i, c])
                sb += abs(bh[i, c])
            best_a = max(best_a, sa)
            best_b = max(best_b, sb)
        brute.append(best_a / na + best_b / nb)
    assert np.allclose(ev, brute, rtol=1e-14)
    assert k == int(np.argmin(brute)) + 1


def test_halfplane_and_disk_maps_move_eigenvalues_as_stated():
    rng = np.random.default_rng(3)
    n = 7
    a = rng.standard_normal((n, n))
    b = rng.standard_normal((n, n)) + 2 * np.eye(n)
    lam = sla.eigvals(a, b)
    sigma, s = 0.3, 0.8
    a0, b0 = premap(a, b, {"kind": "halfplane", "shift": sigma, "scale": s})
    mu = sla.eigvals(a0, b0)
    want = (lam - sigma + s) / (lam - sigma - s)
    for w in want:
        assert np.min(np.abs(mu - w)) < 1e-10 * max(1, abs(w))
    # inside the unit circle exactly when Re(lambda) < sigma
    assert np.array_equal(np.sort(np.abs(want) < 1), np.sort(lam.real < sigma))
    c, r = -0.2, 1.7
    a0, b0 = premap(a, b, {"kind": "disk", "center": c, "radius": r})
    mu = sla.eigvals(a0, b0)
    for w in (lam - c) / r:
        assert np.min(np.abs(mu - w)) < 1e-10 * max(1, abs(w))


@pytest.mark.parametrize("n,seed", [(32, 1), (128, S.family_seed(0))])
def test_split_sym_against_construction(n, seed):
    a, d, q = S.sym_problem(n, seed)
    res = split_sym(a, HALF0, seed=seed)
    assert res.status == OK
    assert res.n_inside == int((d < 0).sum())
    assert res.k == int((d > 0).sum())
    assert res.e <= 1e-12
    k = res.k
    e21 = res.A_hat[k:, :k]
    assert norm1(e21) <= 1e-12 * norm1(a)
    ev = np.concatenate([np.linalg.eigvalsh(res.A_hat[:k, :k]), np.linalg.eigvalsh(res.A_hat[k:, k:])])
    assert np.max(np.abs(np.sort(ev) - np.sort(d))) <= 1e-12 * np.abs(d).max()
    assert np.all(np.linalg.eigvalsh(res.A_hat[:k, :k]) > 0)
    assert np.all(np.linalg.eigvalsh(res.A_hat[k:, k:]) < 0)
    # Davis-Kahan: sin(theta) <= ||E21||_2 / gap, with a spectral gap of 0.1 here
    gap = d[d > 0].min() - d[d < 0].max()
    assert _sin_theta(res.Q[:, :k], q[:, d > 0]) <= 2 * np.linalg.norm(e21, 2) / gap + 1e-13
    assert np.allclose(res.Q.T @ res.Q, np.eye(n), atol=1e-13 * n)


def test_hermitian_off_block_lemma():
    """||A21||_2 <= (lambda_max - lambda_min)/2 for any partition (Sec. 3.4)."""
    rng = np.random.default_rng(9)
    for _ in range(20):
        n = int(rng.integers(2, 30))
        x = rng.standard_normal((n, n))
        a = x + x.T
        k = int(rng.integers(1, n)) if n > 1 else 1
        w = np.linalg.eigvalsh(a)
        assert np.linalg.norm(a[k:, :k], 2) <= (w[-1] - w[0]) / 2 + 1e-12


@pytest.mark.parametrize("n,seed", [(48, 2), (96, 3)])
def test_split_pencil_against_construction(n, seed):
    p = S.pencil_problem(n, seed)
    a, b, lam = p["A"], p["B"], p["lam"]
    res = split_pencil(a, b, {"kind": "unit_disk"}, seed=seed)
    assert res.status == OK
    inside = np.abs(lam) < 1
    assert res.n_inside == int(inside.sum())
    k = res.k
    assert norm1(res.A_hat[k:, :k]) <= 1e-12 * norm1(a)
    assert norm1(res.B_hat[k:, :k]) <= 1e-12 * norm1(b)
    ev_out = sla.eigvals(res.A_hat[:k, :k], res.B_hat[:k, :k])
    ev_in = sla.eigvals(res.A_hat[k:, k:], res.B_hat[k:, k:])
    assert np.all(np.abs(ev_out) > 1) and np.all(np.abs(ev_in) < 1)
    got = np.sort_complex(np.concatenate([ev_out, ev_in]))
    want = np.sort_complex(lam.astype(complex))
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-10
    for qq in (res.Q, res.QL):
        assert np.allclose(qq.T @ qq, np.eye(n), atol=1e-13 * n)


def test_split_pencil_subspaces_equal_known_deflating_subspaces():
    """With T, S upper triangular and the outside eigenvalues first on their
    diagonals, span V[:, :k] is the right and span U[:, :k] the left deflating
    subspace of the outside eigenvalues."""
    n = 40
    p = S.pencil_problem(n, 17, outside_first=True)
    res = split_pencil(p["A"], p["B"], {"kind": "unit_disk"}, seed=5)
    k = int((np.abs(p["lam"]) > 1).sum())
    assert res.status == OK and res.k == k
    assert _sin_theta(res.Q[:, :k], p["V"][:, :k]) <= 1e-11
    assert _sin_theta(res.QL[:, :k], p["U"][:, :k]) <= 1e-11


def test_no_split_when_all_eigenvalues_on_one_side():
    a, d, q = S.sym_problem(24, 4, gap=0.05, lo=-1.0, hi=1.0)
    res = split_sym(a, {"kind": "halfplane", "shift": 3.0, "scale": 1.0}, seed=1)
    assert res.status == NO_SPLIT and res.n_inside == 24
    res = split_sym(a, {"kind": "halfplane", "shift": -3.0, "scale": 1.0}, seed=1)
    assert res.status == NO_SPLIT and res.n_inside == 0


def test_not_converged_with_tiny_maxit():
    a, d, q = S.sym_problem(32, 5)
    res = split_sym(a, HALF0, seed=1, maxit=1)
    assert res.status == NOT_CONVERGED


def test_bad_random_draw_is_detected_and_retried():
    """A 'Gaussian' whose Q factor is orthogonal with its leading rows in the
    null space of the projector hides the rank from RURV; the split must
    notice (rank or norm check) and succeed on the next draw."""
    n = 30
    a, d, q = S.sym_problem(n, 6)
    k = int((d > 0).sum())
    nullvecs = q[:, d < 0]
    rowvecs = q[:, d > 0]
    assert nullvecs.shape[1] >= k
    bad_v = np.vstack([nullvecs.T, rowvecs.T])      # orthogonal, rows 0..k-1 in null(P)
    good = np.random.default_rng(1)

    def gauss(nn, attempt, side):
        return bad_v.copy() if attempt == 0 else good.standard_normal((nn, nn))

    res = split_sym(a, HALF0, gauss=gauss)
    assert res.status == OK
    assert res.attempts == 2
    assert res.n_inside == n - k


def test_rank_from_rho_cases():
    assert rank_from_rho(np.full(5, 1e-9))[2] == "inside"
    assert rank_from_rho(np.full(5, 0.9))[2] == "outside"
    k, gap, side = rank_from_rho(np.array([0.5, 0.1, 0.02, 1e-14, 1e-15]))
    assert side == "split" and k == 3 and gap > 1e10


# ---------------------------------------------------------------------------
# RSVD by the symmetric embedding, pinned to LAPACK's SVD of the construction
# ---------------------------------------------------------------------------

def _sin_theta(x, y):
    qx, _ = np.linalg.qr(x)
    qy, _ = np.linalg.qr(y)
    return float(np.linalg.norm(qy - qx @ (qx.T @ qy), 2))


@pytest.mark.parametrize("m,n", [(30, 20), (20, 30), (24, 24)])
def test_split_svd_recovers_singular_subspaces(m, n):
    from oracle.split import split_svd
    import sdc_synth as S
    a, sig, p_, q_ = S.svd_problem(m, n, S.family_seed(5, m * 100 + n), level=1.0)
    res, u, v, s11 = split_svd(a, {"kind": "halfplane", "shift": 1.0, "scale": 1.0}, seed=2)
    k = int((sig > 1.0).sum())
    assert res.status == 0 and res.k == k and 0 < k < min(m, n)
    assert np.abs(u.T @ u - np.eye(k)).max() <= 1e-12
    assert np.abs(v.T @ v - np.eye(k)).max() <= 1e-12
    # the subspaces of LAPACK's SVD (independent of the construction's basis)
    pu, sv, qvt = np.linalg.svd(a)
    assert np.allclose(sv[:len(sig)], sig, rtol=1e-12)
    assert _sin_theta(u, pu[:, :k]) <= 1e-10 and _sin_theta(v, qvt[:k].T) <= 1e-10
    assert np.abs(np.linalg.eigvalsh(s11) - np.sort(sig[:k])).max() <= 1e-11 * sig[0]
    assert np.abs(u.T @ a @ v - s11).max() <= 1e-11 * sig[0]


# ---------------------------------------------------------------------------
# RNEP (B = I): the right side of the pencil step alone
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [20, 45])
def test_split_nonsym_equals_pencil_right_side_and_construction(n):
    """With B = I the pencil step's right side is the same computation, so
    RNEP's Q is the pencil's Q_R exactly; the split count and the block
    eigenvalues are the construction's."""
    from oracle.split import split_nonsym
    a, lam = S.nonsym_problem(n, S.family_seed(6, n))
    reg = {"kind": "unit_disk"}
    r = split_nonsym(a, reg, seed=3)
    p = split_pencil(a, np.eye(n), reg, seed=3)
    k = int((np.abs(lam) > 1).sum())
    assert r.status == OK and r.k == k == p.k
    assert np.array_equal(r.Q, p.Q)
    assert np.abs(r.Q.T @ r.Q - np.eye(n)).max() <= 1e-13
    assert norm1(r.A_hat[k:, :k]) <= 1e-10 * norm1(a)
    ev1 = np.sort_complex(np.linalg.eigvals(r.A_hat[:k, :k]))
    ev2 = np.sort_complex(np.linalg.eigvals(r.A_hat[k:, k:]))
    lam_out = np.sort(lam[np.abs(lam) > 1]).astype(complex)
    lam_in = np.sort(lam[np.abs(lam) < 1]).astype(complex)
    assert np.abs(ev1 - lam_out).max() <= 1e-8 * np.abs(lam).max()
    assert np.abs(ev2 - lam_in).max() <= 1e-8


def test_split_nonsym_complex_pairs_half_plane():
    """A real normal matrix with conjugate pairs, split at Re z < 0: the
    leading block holds the eigenvalues with positive real part."""
    from oracle.split import split_nonsym
    a, ev = S.normal_random_problem(40, S.family_seed(6, 40))
    r = split_nonsym(a, {"kind": "halfplane", "shift": 0.0, "scale": 1.0}, seed=1)
    k = int((ev.real > 0).sum())
    assert r.status == OK and r.k == k
    got = np.sort_complex(np.linalg.eigvals(r.A_hat[:k, :k]))
    assert np.abs(got - np.sort_complex(ev[ev.real > 0])).max() <= 1e-9
