"""One split step: Alg. 4 (RGNEP, pencils) and Alg. 6 (RSEP, symmetric A, B = I).

Steps, in the paper's order:
1. Map the splitting curve to the unit circle (Sec. 3.3): for the half plane
   Re z < sigma with scale s, the pencil (A, B) becomes
   (A - (sigma - s) B, A - (sigma + s) B), i.e. z -> (z - sigma + s)/(z - sigma - s)
   (the paper's map with a = sigma and unit scale, applied to a pencil);
   for the disk |z - c| < r it becomes (A - c B, r B); the unit disk is kept.
2. IRS (Alg. 3) on the mapped pencil -> (A_p, B_p).
3. Right subspace: Q_R = GRURV(2, A_p + B_p, A_p, -1, 1) (Alg. 4 line 2,
   Alg. 6 line 2), the U factor of a rank-revealing factorization of
   (A_p + B_p)^{-1} A_p, which tends to the projector onto the right deflating
   subspace of the eigenvalues OUTSIDE the circle (Sec. 3.2).
4. Pencils only: IRS on the transposed pencil, then
   Q_L = GRURV(2, A_p'^T, (A_p' + B_p')^T, 1, -1) (Alg. 4 lines 3-4).
5. Block form with the ORIGINAL A, B: A_hat = Q_L^T A Q_R (and B_hat), or
   A_hat = Q^T A Q symmetrized for Alg. 6.
6. Split point: the k minimizing ||E21||_1/||A||_1 (+ ||F21||_1/||B||_1),
   E21 = A_hat[k:, :k] (Alg. 4 line 5).

Readings of the paper used here:
* Ordering: the leading k columns of Q (Q_R) span the subspace of the
  eigenvalues outside the unit circle after the map, so A11 holds the outside
  eigenvalues and A22 the inside ones; n_inside = n - k.  (The introduction of
  Sec. 3.1 says "inside" for the leading columns, but the block statement after
  it, the projector of Sec. 3.2 and the algorithms all give "outside".)
* Eigenvalues are those of det(A - lambda B) = 0; after the half-plane map,
  inside the circle means Re lambda < sigma.
* Success: the paper accepts a split when the minimized norm is small enough.
  The oracle also reads the rank off the diagonals of the GRURV factors
  (|diag R| of R1^{m1} R2^{m2}) and requires both answers to agree; a
  disagreement or a large norm is retried with a fresh Gaussian (attempt + 1).
  If every diagonal ratio is tiny (or none is) the eigenvalues all lie on one
  side and the result is NO_SPLIT.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable

import numpy as np

from .irs import irs, norm1, EPS64
from .rurv import grurv2
from .philox import gaussian_matrix

OK, NOT_CONVERGED, NO_SPLIT, RANK_AMBIGUOUS = 0, 1, 2, 3

# |diag R| thresholds for "all inside" / "all outside": rho is scale free
# (it is a diagonal of a rank-revealing factorization of a projector-like
# matrix of norm >= 1), so one absolute threshold separates O(1/n) from
# rounding-level entries.
RHO_ONE_SIDE = 1e-3


def premap(a: np.ndarray, b: np.ndarray, region: dict):
    """Step 1: map the region's boundary to the unit circle (Sec. 3.3)."""
    kind = region.get("kind", "unit_disk")
    if kind == "unit_disk":
        return a.copy(), b.copy()
    if kind == "disk":
        c, r = float(region["center"]), float(region["radius"])
        return a - c * b, r * b
    if kind == "halfplane":
        sigma, s = float(region["shift"]), float(region.get("scale", 1.0))
        return a - (sigma - s) * b, a - (sigma + s) * b
    raise ValueError(kind)


def split_search(a_hat: np.ndarray, norm_a: float, b_hat: np.ndarray | None = None,
                 norm_b: float | None = None):
    """Alg. 4 line 5: for k = 1..n-1, e(k) = ||A_hat[k:, :k]||_1/||A||_1
    (+ the same for B_hat).  Returns (k_star, e(k_star), e as an array indexed
    by k-1).  Ties go to the smallest k."""
    n = a_hat.shape[0]
    if n < 2:
        return 0, np.inf, np.empty(0)

    def e21(x):
        # suf[k, c] = sum_{i >= k} |x_ic|; ||x[k:, :k]||_1 = max_{c < k} suf[k, c]
        suf = np.cumsum(np.abs(x)[::-1, :], axis=0)[::-1, :]
        pre = np.maximum.accumulate(suf, axis=1)
        k = np.arange(1, n)
        return pre[k, k - 1]

    e = e21(a_hat) / norm_a
    if b_hat is not None:
        e = e + e21(b_hat) / norm_b
    k = int(np.argmin(e)) + 1
    return k, float(e[k - 1]), e


def rank_from_rho(rho: np.ndarray):
    """Rank read off |diag| of the GRURV triangular factors.

    Returns (k_rho, gap, side) where side is 'inside' if every entry is tiny
    (projector ~ 0), 'outside' if none is (projector ~ I), else 'split';
    k_rho is the count above the largest gap of the sorted values and gap the
    ratio across it."""
    rho = np.abs(np.asarray(rho, dtype=np.float64))
    n = rho.size
    if rho.max() < RHO_ONE_SIDE:
        return 0, 1.0, "inside"
    if rho.min() > RHO_ONE_SIDE:
        return n, 1.0, "outside"
    srt = np.sort(np.maximum(rho, 1e-300))[::-1]
    ratios = srt[:-1] / srt[1:]
    i = int(np.argmax(ratios))
    return i + 1, float(ratios[i]), "split"


@dataclass
class SplitResult:
    status: int
    k: int                    # leading block size (eigenvalues outside)
    n_inside: int
    Q: np.ndarray             # Q_R (Q for the symmetric case)
    QL: np.ndarray | None
    A_hat: np.ndarray
    B_hat: np.ndarray | None
    e: float                  # the minimized relative norm e(k)
    p_right: int
    p_left: int
    k_rho: int
    rank_gap: float
    attempts: int
    rho: np.ndarray = field(default=None)


GaussSource = Callable[[int, int, int], np.ndarray]  # (n, attempt, side) -> G


def philox_source(seed: int) -> GaussSource:
    """The default Gaussian source: Philox4x32-10 keyed by (seed + attempt),
    tagged by side (0 right, 1 left)."""
    return lambda n, attempt, side: gaussian_matrix(n, seed + attempt, side)


def _defaults(tau, split_tol):
    if tau is None:
        tau = EPS64 ** 0.5
    if split_tol is None:
        split_tol = 1e-10
    return tau, split_tol


def split_sym(a: np.ndarray, region: dict, gauss: GaussSource | None = None, seed: int = 0,
              tau: float | None = None, maxit: int = 60, max_retries: int = 2,
              split_tol: float | None = None) -> SplitResult:
    """Alg. 6 (RSEP) with the map of step 1 (B = I)."""
    tau, split_tol = _defaults(tau, split_tol)
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    gauss = gauss or philox_source(seed)
    a0, b0 = premap(a, np.eye(n), region)
    res = irs(a0, b0, tau=tau, maxit=maxit)
    ap, bp = res.A, res.B
    norm_a = norm1(a)
    best = None
    for attempt in range(max_retries + 1):
        g = gauss(n, attempt, 0)
        q, r1, r2, _ = grurv2(ap + bp, ap, -1, 1, g)
        rho = np.abs(np.diag(r2)) / np.abs(np.diag(r1))
        k_rho, gap, side = rank_from_rho(rho)
        a_hat = q.T @ a @ q
        a_hat = 0.5 * (a_hat + a_hat.T)
        if side != "split":
            k = 0 if side == "inside" else n
            return SplitResult(NO_SPLIT if res.converged else NOT_CONVERGED, k, n - k, q, None,
                               a_hat, None, 0.0, res.p, 0, k_rho, gap, attempt + 1, rho)
        k, e, _ = split_search(a_hat, norm_a)
        cand = SplitResult(OK, k, n - k, q, None, a_hat, None, e, res.p, 0, k_rho, gap,
                           attempt + 1, rho)
        if best is None or e < best.e:
            best = cand
        if e <= split_tol:  # the split is accepted on its backward error (Alg. 4)
            if not res.converged:
                cand.status = NOT_CONVERGED
            return cand
    best.status = NOT_CONVERGED if not res.converged else RANK_AMBIGUOUS
    return best


def split_pencil(a: np.ndarray, b: np.ndarray, region: dict, gauss: GaussSource | None = None,
                 seed: int = 0, tau: float | None = None, maxit: int = 60, max_retries: int = 2,
                 split_tol: float | None = None) -> SplitResult:
    """Alg. 4 (RGNEP) with the map of step 1."""
    tau, split_tol = _defaults(tau, split_tol)
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = a.shape[0]
    gauss = gauss or philox_source(seed)
    a0, b0 = premap(a, b, region)
    right = irs(a0, b0, tau=tau, maxit=maxit)
    left = irs(a0.T, b0.T, tau=tau, maxit=maxit)
    converged = right.converged and left.converged
    ap, bp = right.A, right.B
    alp, blp = left.A, left.B
    norm_a, norm_b = norm1(a), norm1(b)
    best = None
    for attempt in range(max_retries + 1):
        qr_, r1, r2, _ = grurv2(ap + bp, ap, -1, 1, gauss(n, attempt, 0))
        rho_r = np.abs(np.diag(r2)) / np.abs(np.diag(r1))
        ql_, l1, l2, _ = grurv2(alp.T, (alp + blp).T, 1, -1, gauss(n, attempt, 1))
        rho_l = np.abs(np.diag(l1)) / np.abs(np.diag(l2))
        k_rho, gap, side = rank_from_rho(rho_r)
        k_rho_l, gap_l, side_l = rank_from_rho(rho_l)
        a_hat = ql_.T @ a @ qr_
        b_hat = ql_.T @ b @ qr_
        if side != "split" and side == side_l:
            k = 0 if side == "inside" else n
            st = NO_SPLIT if converged else NOT_CONVERGED
            return SplitResult(st, k, n - k, qr_, ql_, a_hat, b_hat, 0.0, right.p, left.p,
                               k_rho, gap, attempt + 1, rho_r)
        if side != side_l:
            # the two sides disagree about the spectrum being one-sided: a
            # bad draw (or iterates short of convergence); try a new draw,
            # and report the rank as unknown (-1) if none agrees
            last = SplitResult(NOT_CONVERGED if not converged else RANK_AMBIGUOUS, -1, -1, qr_, ql_,
                               a_hat, b_hat, np.inf, right.p, left.p, k_rho, gap, attempt + 1, rho_r)
            continue
        k, e, _ = split_search(a_hat, norm_a, b_hat, norm_b)
        cand = SplitResult(OK, k, n - k, qr_, ql_, a_hat, b_hat, e, right.p, left.p, k_rho,
                           min(gap, gap_l), attempt + 1, rho_r)
        if best is None or e < best.e:
            best = cand
        if e <= split_tol:  # the split is accepted on its backward error (Alg. 4)
            if not converged:
                cand.status = NOT_CONVERGED
            return cand
    if best is None:
        return last
    best.status = NOT_CONVERGED if not converged else RANK_AMBIGUOUS
    return best


def split_svd(a: np.ndarray, region: dict, seed: int = 0, **kw):
    """RSVD (the singular value problem, Sec. 3): one symmetric split step
    (Alg. 6) of the embedding E = [0 A; A^T 0], whose eigenvalues are the
    singular values of A, their negatives and |m - n| zeros, with
    eigenvectors [u; v] / sqrt(2).  At a half plane Re z < tau (tau >= 0) the
    leading k columns of E's Q span the pairs of the k singular values above
    tau, so U = sqrt(2) Q[:m, :k] and V = sqrt(2) Q[m:, :k] are orthonormal
    bases of the left and right singular subspaces and
    S11 = Ahat[:k, :k] = U^T A V.  Returns (SplitResult of E, U, V, S11)."""
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    e = np.zeros((m + n, m + n))
    e[:m, m:] = a
    e[m:, :m] = a.T
    res = split_sym(e, region, seed=seed, **kw)
    k = res.k
    u = np.sqrt(2.0) * res.Q[:m, :k]
    v = np.sqrt(2.0) * res.Q[m:, :k]
    s11 = res.A_hat[:k, :k]
    return res, u, v, s11


def split_nonsym(a: np.ndarray, region: dict, gauss: GaussSource | None = None, seed: int = 0,
                 tau: float | None = None, maxit: int = 60, max_retries: int = 2,
                 split_tol: float | None = None) -> SplitResult:
    """RNEP (the non-symmetric standard problem, B = I; the paragraph after
    Alg. 4): the right side of Alg. 4 only, since with B = I the left
    deflating subspace equals the right one: IRS of the mapped (A, I),
    GRURV(2, A_p + B_p, A_p, -1, 1), A_hat = Q^T A Q (not symmetrized), and
    the split point minimizing ||E21||_1 / ||A||_1, the backward error."""
    tau, split_tol = _defaults(tau, split_tol)
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    gauss = gauss or philox_source(seed)
    a0, b0 = premap(a, np.eye(n), region)
    res = irs(a0, b0, tau=tau, maxit=maxit)
    ap, bp = res.A, res.B
    norm_a = norm1(a)
    best = None
    for attempt in range(max_retries + 1):
        g = gauss(n, attempt, 0)
        q, r1, r2, _ = grurv2(ap + bp, ap, -1, 1, g)
        rho = np.abs(np.diag(r2)) / np.abs(np.diag(r1))
        k_rho, gap, side = rank_from_rho(rho)
        a_hat = q.T @ a @ q
        if side != "split":
            k = 0 if side == "inside" else n
            return SplitResult(NO_SPLIT if res.converged else NOT_CONVERGED, k, n - k, q, None,
                               a_hat, None, 0.0, res.p, 0, k_rho, gap, attempt + 1, rho)
        k, e, _ = split_search(a_hat, norm_a)
        cand = SplitResult(OK, k, n - k, q, None, a_hat, None, e, res.p, 0, k_rho, gap,
                           attempt + 1, rho)
        if best is None or e < best.e:
            best = cand
        if e <= split_tol:  # the split is accepted on its backward error (Alg. 4)
            if not res.converged:
                cand.status = NOT_CONVERGED
            return cand
    best.status = NOT_CONVERGED if not res.converged else RANK_AMBIGUOUS
    return best
