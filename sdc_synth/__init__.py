"""Seeded synthetic inputs for the inverse-free split step.

This module builds test and benchmark INPUTS only: matrices with a spectrum
known by construction, and the Gaussian matrices that the randomized
rank-revealing factorization draws.  It holds none of the split method's
arithmetic (no repeated squaring, no rank-revealing factorization, no block
form, no split search).  Both the FP64 oracle and the HIP library consume
these arrays; neither imports the other.

Orthogonal similarity factors are drawn as the Q factor of a Gaussian matrix
with the signs of R's diagonal moved into Q, so that the factor is Haar
distributed.  The QR here is a NumPy library call.

Seeds: base 10113077; a workload family c uses 10113077 + 1000*c and problem i
of that family uses 10113077 + 1000*c + i.
"""
from __future__ import annotations

import math
import numpy as np

BASE_SEED = 10113077


def family_seed(config: int, index: int = 0) -> int:
    return BASE_SEED + 1000 * config + index


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed n x n orthogonal matrix (QR of N(0,1), sign-fixed)."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def gaussian(n: int, seed: int) -> np.ndarray:
    """The N(0,1) n x n matrix that the randomized URV draws (its line 1),
    column-major friendly float64, from numpy's default generator."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, n)))


# ----------------------------------------------------------------------------
# Symmetric problems (B = I): A = Q diag(d) Q^T.
# ----------------------------------------------------------------------------

def sym_problem(n: int, seed: int, gap: float = 0.05, lo: float = -1.0, hi: float = 1.0):
    """Symmetric A = Q diag(d) Q^T with Q Haar and d uniform in [lo, hi]
    excluding |d| < gap.  Returns (A, d, Q).  Half-plane split at 0 puts
    #(d < 0) eigenvalues inside."""
    rng = np.random.default_rng(seed)
    q = haar_orthogonal(n, rng)
    # uniform on [lo,-gap] U [gap,hi] by rejection-free mapping
    neg_len = max(0.0, -gap - lo)
    pos_len = max(0.0, hi - gap)
    u = rng.uniform(0.0, neg_len + pos_len, size=n)
    d = np.where(u < neg_len, lo + u, gap + (u - neg_len))
    a = (q * d[None, :]) @ q.T
    a = 0.5 * (a + a.T)
    return np.asfortranarray(a), d, q


def nonsym_problem(n: int, seed: int, lam_lo: float = 0.1, lam_hi: float = 10.0,
                   circle_gap: float = 0.01, offdiag: float = 0.02):
    """Non-symmetric A = U T U^T with U Haar and T upper triangular: real
    eigenvalues T_ii with |lambda| log-uniform in [lam_lo, lam_hi], random
    signs, | |lambda| - 1 | >= circle_gap; strictly upper part
    N(0,1) offdiag / sqrt(n).  Returns (A, lam)."""
    rng = np.random.default_rng(seed)
    u_ = haar_orthogonal(n, rng)
    lam = np.empty(n)
    for i in range(n):
        while True:
            m = math.exp(rng.uniform(math.log(lam_lo), math.log(lam_hi)))
            if abs(m - 1.0) >= circle_gap:
                break
        lam[i] = m if rng.uniform() < 0.5 else -m
    t = np.triu(rng.standard_normal((n, n)) * (offdiag / math.sqrt(n)), 1)
    t[np.diag_indices(n)] = lam
    return np.asfortranarray(u_ @ t @ u_.T), lam


def svd_problem(m: int, n: int, seed: int, level: float = 1.0, gap: float = 0.05,
                lo: float = 0.1, hi: float = 10.0):
    """m x n A = P diag(sigma) Q^T with P (m x r), Q (n x r) orthonormal
    columns of Haar matrices, r = min(m, n), and sigma log-uniform in [lo, hi]
    excluding [level (1 - gap), level (1 + gap)], in decreasing order.
    Returns (A, sigma, P, Q)."""
    rng = np.random.default_rng(seed)
    r = min(m, n)
    p_ = haar_orthogonal(m, rng)[:, :r]
    q_ = haar_orthogonal(n, rng)[:, :r]
    sig = np.empty(r)
    for i in range(r):
        while True:
            x = math.exp(rng.uniform(math.log(lo), math.log(hi)))
            if abs(x - level) > gap * level:
                break
        sig[i] = x
    sig = np.sort(sig)[::-1]
    a = (p_ * sig[None, :]) @ q_.T
    return np.asfortranarray(a), sig, p_, q_


def clustered_sym_problem(n: int, seed: int):
    """Symmetric, eigenvalues half in [-1,-0.01] and half in [0.01,1], with
    10% of them (5% per side) within 1e-3 of +-0.01, i.e. |d| in
    [0.01, 0.011]; the rest uniform in |d| in [0.011, 1].  Returns (A, d, Q)."""
    rng = np.random.default_rng(seed)
    q = haar_orthogonal(n, rng)
    nneg = n // 2
    npos = n - nneg
    parts = []
    for cnt, sgn in ((nneg, -1.0), (npos, 1.0)):
        ncl = int(math.floor(0.05 * n))
        ncl = min(ncl, cnt)
        mag = np.concatenate([rng.uniform(0.01, 0.011, size=ncl),
                              rng.uniform(0.011, 1.0, size=cnt - ncl)])
        parts.append(sgn * mag)
    d = np.concatenate(parts)
    d = d[rng.permutation(n)]
    a = (q * d[None, :]) @ q.T
    a = 0.5 * (a + a.T)
    return np.asfortranarray(a), d, q


def batch_sizes(count: int, seed: int, nmin: int = 32, nmax: int = 256) -> list[int]:
    """Problem sizes log-uniform in [nmin, nmax] (rounded)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(nmin), math.log(nmax), size=count)
    return [int(round(math.exp(x))) for x in u]


# ----------------------------------------------------------------------------
# Nonsymmetric pencils: A = U T V^T, B = U S V^T with T, S upper triangular.
# ----------------------------------------------------------------------------

def pencil_problem(n: int, seed: int, lam_lo: float = 0.1, lam_hi: float = 10.0,
                   circle_gap: float = 0.01, offdiag: float = 0.02, outside_first: bool = False):
    """Real pencil with real eigenvalues lambda_i = T_ii / S_ii.

    |lambda| is log-uniform in [lam_lo, lam_hi] with a random sign and
    | |lambda| - 1 | >= circle_gap; S_ii is uniform in [0.5, 2] and
    T_ii = lambda_i S_ii.  Strictly upper parts of T and S are
    N(0,1) * offdiag / sqrt(n).  U, V Haar.  With outside_first the
    |lambda| > 1 eigenvalues are placed first on the diagonal, so the leading
    columns of V (of U) span the right (left) deflating subspace of the
    outside eigenvalues.

    Returns dict(A, B, lam, U, V, T, S).
    """
    rng = np.random.default_rng(seed)
    u_ = haar_orthogonal(n, rng)
    v_ = haar_orthogonal(n, rng)
    lo, hi = math.log(lam_lo), math.log(lam_hi)
    mags = np.empty(n)
    for i in range(n):
        while True:
            m = math.exp(rng.uniform(lo, hi))
            if abs(m - 1.0) >= circle_gap:
                break
        mags[i] = m
    signs = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    lam = signs * mags
    if outside_first:
        order = np.argsort(-(np.abs(lam) > 1.0).astype(int), kind="stable")
        lam = lam[order]
    sdiag = rng.uniform(0.5, 2.0, size=n)
    t = np.triu(rng.standard_normal((n, n)) * (offdiag / math.sqrt(n)), 1)
    s = np.triu(rng.standard_normal((n, n)) * (offdiag / math.sqrt(n)), 1)
    t[np.diag_indices(n)] = lam * sdiag
    s[np.diag_indices(n)] = sdiag
    a = u_ @ t @ v_.T
    b = u_ @ s @ v_.T
    return dict(A=np.asfortranarray(a), B=np.asfortranarray(b), lam=lam,
                U=u_, V=v_, T=t, S=s)


# ----------------------------------------------------------------------------
# Constructions of the paper's four numerical experiments (normal matrices,
# eigenvalues near the imaginary axis, a Jordan block).
# ----------------------------------------------------------------------------

def _real_normal_from_eigs(eigs_cplx: list[complex], real_eigs: list[float], rng) -> np.ndarray:
    """Real normal matrix with the given eigenvalues: 2x2 rotation-scaling
    blocks for each conjugate pair, 1x1 for real ones, then a random orthogonal
    similarity."""
    n = 2 * len(eigs_cplx) + len(real_eigs)
    d = np.zeros((n, n))
    i = 0
    for z in eigs_cplx:
        x, y = z.real, z.imag
        d[i:i + 2, i:i + 2] = [[x, y], [-y, x]]
        i += 2
    for x in real_eigs:
        d[i, i] = x
        i += 1
    q = haar_orthogonal(n, rng)
    return q @ d @ q.T


def normal_random_problem(n: int, seed: int, box: float = 1.5):
    """Real normal matrix whose eigenvalues have real and imaginary parts
    uniform in [-box, box] (conjugate pairs; one real eigenvalue if n is odd).
    Returns (A, eigenvalues)."""
    rng = np.random.default_rng(seed)
    pairs = [complex(rng.uniform(-box, box), rng.uniform(-box, box)) for _ in range(n // 2)]
    reals = [float(rng.uniform(-box, box)) for _ in range(n % 2)]
    a = _real_normal_from_eigs(pairs, reals, rng)
    ev = []
    for z in pairs:
        ev += [z, z.conjugate()]
    ev += [complex(x, 0.0) for x in reals]
    return np.asfortranarray(a), np.array(ev)


def near_axis_problem(n: int, seed: int, re_abs: float = 1e-10, box: float = 1.5):
    """Real normal matrix with eigenvalues of real part +-re_abs and imaginary
    part uniform in [-box, box].  Returns (A, eigenvalues)."""
    rng = np.random.default_rng(seed)
    pairs = []
    for _ in range(n // 2):
        sgn = -1.0 if rng.uniform() < 0.5 else 1.0
        pairs.append(complex(sgn * re_abs, rng.uniform(-box, box)))
    reals = [(-1.0 if rng.uniform() < 0.5 else 1.0) * re_abs for _ in range(n % 2)]
    a = _real_normal_from_eigs(pairs, reals, rng)
    ev = []
    for z in pairs:
        ev += [z, z.conjugate()]
    ev += [complex(x, 0.0) for x in reals]
    return np.asfortranarray(a), np.array(ev)


def jordan_problem(n: int, seed: int, jordan_value: float = 0.1):
    """n x n real matrix: n/2 random eigenvalues with negative real part
    (conjugate pairs, Re in [-1.5,-0.1], Im in [-1.5,1.5]) plus an (n/2)x(n/2)
    Jordan block at jordan_value with unit superdiagonal; random orthogonal
    similarity.  Returns A."""
    rng = np.random.default_rng(seed)
    h = n // 2
    d = np.zeros((n, n))
    i = 0
    for _ in range(h // 2):
        x, y = rng.uniform(-1.5, -0.1), rng.uniform(-1.5, 1.5)
        d[i:i + 2, i:i + 2] = [[x, y], [-y, x]]
        i += 2
    if h % 2:
        d[i, i] = rng.uniform(-1.5, -0.1)
        i += 1
    for k in range(n - h):
        d[i + k, i + k] = jordan_value
        if k + 1 < n - h:
            d[i + k, i + k + 1] = 1.0
    q = haar_orthogonal(n, rng)
    return np.asfortranarray(q @ d @ q.T)
