"""Randomized spectral divide-and-conquer (Sec. 3.3-3.5) on top of the split
step, for the oracle.

Strategy, as the paper describes it:
* symmetric A (Sec. 3.4): bound the spectrum by the Gershgorin interval
  [c - R, c + R] and split at a random point x uniform in [c - R/2, c + R/2];
  the two halves inherit [x, c + R] and [c - R, x]; a split that finds every
  eigenvalue on one side still shrinks the interval (progress);
* pencils (Sec. 3.5): split at the unit circle first.  If every eigenvalue
  is inside, try radii 1/2, 1/4, 1/16, ... (2^{-2^k}) until a circle splits
  the spectrum or finds it all outside; then the smallest bounding circle is
  the last radius that had it all inside, and the block is split by lines
  inside that disk.  If every eigenvalue is outside, try radii 2, 4, 16, ...
  (2^{2^k}) until a circle splits it or finds it all inside; then the largest
  circle with the spectrum outside is the last such radius r, and the pair is
  swapped to (B, A), whose eigenvalues are the reciprocals and lie inside
  1/r.  Running out of exponent range ends either search the same way.  A
  block that split at a circle of radius r continues by lines: the inside
  part inside r, the outside part swapped, inside 1/r.  Lines are vertical
  (real arithmetic: a complex-conjugate pair is never separated), random in
  the middle half of the block's interval of real parts.
* A circle or line that hits the pseudospectrum makes the split step fail
  (no convergence, or no split meeting the tolerance); a failed circle is
  retried at a randomly perturbed radius r 2^{u - 1/2}, a failed line at a
  fresh random line.  After repeated failures the block is given up and
  returned as it is, with the bound on its spectrum that the search reached
  (Sec. 3.6: a block Schur form with a bound on each block's
  pseudospectrum).  Repeated failures while no circle at all has worked mean
  that every curve meets the pseudospectrum, which is what a (nearly)
  singular pencil does (Sec. 3.5): the block is then flagged near-singular.
The coupling blocks E21 (and F21) are set to zero after each accepted split,
and the transformations are applied to the rest of the pair and accumulated.
An accepted step divides its block at its split point k and also at every
other k' whose coupling blocks are as small (e(k') <= split_tol): the paper
notes that more than one small pair of blocks may divide the problem into
more than two.  The pieces on either side of k inherit that side's bound.

Each leaf block carries a bound (re_lo, re_hi, radius, inverted): the
eigenvalues mu of the block pair satisfy re_lo <= Re mu <= re_hi and
|mu| <= radius, where mu = 1/lambda when inverted (the block was reached
through a swap) and mu = lambda otherwise.  Infinite entries mean no bound.
"""
from __future__ import annotations

import math

import numpy as np

from .split import split_sym, split_pencil, split_search, norm1, OK, NO_SPLIT

SPLIT_TOL = 1e-10      # the split step's acceptance threshold, also for extra split points
MAX_TRIES = 8          # consecutive failed curves before a block is given up
MAX_CIRCLE_FAILS = 3   # consecutive failed circles before a block is given up (near-singular)
RADIUS_MIN, RADIUS_MAX = 2.0 ** -1000, 2.0 ** 1000   # exponent range of the radius search


def _gershgorin(a: np.ndarray):
    c = np.diag(a)
    r = np.sum(np.abs(a), axis=1) - np.abs(c)
    return float(np.min(c - r)), float(np.max(c + r))


def _lines(blk, lo, hi, swap):
    """Continue a pencil block with lines inside the disk |mu| <= hi (lo = -hi)."""
    return dict(blk, mode="line", lo=lo, hi=hi, radius=hi, swapped=blk["swapped"] ^ swap, tries=0)


def _circle_no_split(blk, all_inside):
    """Next state of a block in circle mode whose circle found every
    eigenvalue on one side (Sec. 3.5).  Returns the new block state."""
    r, rprev, d = blk["radius"], blk["rprev"], blk["dir"]
    if all_inside:
        if d > 0:   # growing: rprev had it all outside -> swap, inside 1/rprev
            return _lines(blk, -1.0 / rprev, 1.0 / rprev, True)
        nr = 0.5 if r >= 1.0 else r * r
        if nr < RADIUS_MIN:  # out of exponent range: bounded by r, go on with lines
            return _lines(blk, -r, r, False)
        return dict(blk, radius=nr, rprev=r, dir=-1, tries=0)
    if d < 0:       # shrinking: rprev had it all inside -> lines inside rprev
        return _lines(blk, -rprev, rprev, False)
    nr = 2.0 if r <= 1.0 else r * r
    if nr > RADIUS_MAX:
        return _lines(blk, -1.0 / r, 1.0 / r, True)
    return dict(blk, radius=nr, rprev=r, dir=1, tries=0)


def _bound(blk, symmetric):
    """(re_lo, re_hi, radius, inverted) of a leaf block."""
    if symmetric:
        return (blk["lo"], blk["hi"], max(abs(blk["lo"]), abs(blk["hi"])), 0)
    if blk["mode"] == "line":
        return (blk["lo"], blk["hi"], blk["radius"], int(blk["swapped"]))
    d, rprev = blk["dir"], blk["rprev"]
    if d < 0:   # every eigenvalue inside rprev
        return (-rprev, rprev, rprev, int(blk["swapped"]))
    if d > 0:   # every eigenvalue outside rprev: reciprocals inside 1/rprev
        return (-1.0 / rprev, 1.0 / rprev, 1.0 / rprev, int(not blk["swapped"]))
    return (-math.inf, math.inf, math.inf, int(blk["swapped"]))


def eig_dc(a: np.ndarray, b: np.ndarray | None = None, symmetric: bool = False, leaf_max: int = 64,
           seed: int = 0):
    """Returns dict(T, S, QL, QR, blocks=[(s, e), ...], bounds=[(re_lo, re_hi,
    radius, inverted), ...] per block, splits, unsplit, near_singular, extra_splits,
    log=[(s, e, mode, curve value, status, k), ...] per split attempt)."""
    a = np.array(a, dtype=np.float64)
    n = a.shape[0]
    t = a.copy()
    s = None if symmetric else np.array(b, dtype=np.float64)
    ql = np.eye(n)
    qr = np.eye(n)
    rng = np.random.default_rng(seed)
    base = dict(s=0, e=n, swapped=False, tries=0, dir=0, rprev=1.0)
    if symmetric:
        lo, hi = _gershgorin(a)
        if not hi > lo:
            hi = lo + 1.0
        work = [dict(base, mode="line", lo=lo, hi=hi, radius=max(abs(lo), abs(hi)))]
    else:
        work = [dict(base, mode="circle", lo=-math.inf, hi=math.inf, radius=1.0)]
    leaves, splits, unsplit, near_singular, extra, log = [], 0, 0, 0, 0, []
    if n <= leaf_max:
        leaves, work = work, []
    while work:
        nxt = []
        for blk in work:
            s0, e0 = blk["s"], blk["e"]
            m = e0 - s0
            if blk["mode"] == "circle":
                region = {"kind": "disk", "center": 0.0, "radius": blk["radius"]}
                curve = blk["radius"]
            else:
                c, r = 0.5 * (blk["lo"] + blk["hi"]), 0.5 * (blk["hi"] - blk["lo"])
                region = {"kind": "halfplane", "shift": c + (rng.uniform() - 0.5) * r, "scale": r if r > 0 else 1.0}
                curve = region["shift"]
            splits += 1
            tb = t[s0:e0, s0:e0]
            if symmetric:
                res = split_sym(tb, region, seed=int(rng.integers(1 << 31)))
                qlb = qrb = res.Q
            else:
                sb = s[s0:e0, s0:e0]
                pa, pb = (sb, tb) if blk["swapped"] else (tb, sb)
                res = split_pencil(pa, pb, region, seed=int(rng.integers(1 << 31)))
                qlb, qrb = res.QL, res.Q
            k = res.k
            log.append((s0, e0, blk["mode"], curve, res.status, k))
            if res.status != OK or not (0 < k < m):
                if res.status == NO_SPLIT:   # progress: the search narrows
                    all_inside = res.n_inside == m
                    if blk["mode"] == "circle":
                        nb = _circle_no_split(blk, all_inside)
                    else:
                        nb = dict(blk, tries=0)
                        if all_inside:
                            nb["hi"] = region["shift"]
                        else:
                            nb["lo"] = region["shift"]
                        if not nb["hi"] > nb["lo"]:
                            nb["tries"] = MAX_TRIES
                else:                        # the curve met the pseudospectrum
                    nb = dict(blk, tries=blk["tries"] + 1)
                    if blk["mode"] == "circle":
                        nb["radius"] = blk["radius"] * 2.0 ** (rng.uniform() - 0.5)
                cap = MAX_CIRCLE_FAILS if nb["mode"] == "circle" else MAX_TRIES
                if nb["tries"] >= cap:
                    unsplit += 1
                    if nb["mode"] == "circle":
                        near_singular += 1
                    leaves.append(dict(nb, unsplit=True))
                else:
                    nxt.append(nb)
                continue
            # accepted: every split point with a small coupling block
            if symmetric:
                _, _, prof = split_search(res.A_hat, norm1(tb))
            else:
                _, _, prof = split_search(res.A_hat, norm1(pa), res.B_hat, norm1(pb))
            cuts = [kk for kk in range(1, m) if kk == k or prof[kk - 1] <= SPLIT_TOL]
            extra += len(cuts) - 1
            # write the split pair, drop the coupling blocks, update the rest
            if symmetric:
                t[s0:e0, s0:e0] = res.A_hat
                for kk in cuts:
                    t[s0 + kk:e0, s0:s0 + kk] = 0.0
                    t[s0:s0 + kk, s0 + kk:e0] = 0.0
            else:
                ah, bh = (res.B_hat, res.A_hat) if blk["swapped"] else (res.A_hat, res.B_hat)
                t[s0:e0, s0:e0] = ah
                s[s0:e0, s0:e0] = bh
                for kk in cuts:
                    t[s0 + kk:e0, s0:s0 + kk] = 0.0
                    s[s0 + kk:e0, s0:s0 + kk] = 0.0
                t[s0:e0, e0:] = qlb.T @ t[s0:e0, e0:]
                s[s0:e0, e0:] = qlb.T @ s[s0:e0, e0:]
                t[:s0, s0:e0] = t[:s0, s0:e0] @ qrb
                s[:s0, s0:e0] = s[:s0, s0:e0] @ qrb
                ql[:, s0:e0] = ql[:, s0:e0] @ qlb
            qr[:, s0:e0] = qr[:, s0:e0] @ qrb
            c1 = dict(blk, tries=0)
            c2 = dict(blk, tries=0)
            if blk["mode"] == "circle":
                r0 = blk["radius"]
                c1 = _lines(c1, -1.0 / r0, 1.0 / r0, True)   # outside r0: reciprocals inside 1/r0
                c2 = _lines(c2, -r0, r0, False)
            else:
                c1["lo"] = region["shift"]
                c2["hi"] = region["shift"]
            for lo, hi in zip([0] + cuts, cuts + [m]):
                c = dict(c1 if hi <= k else c2, s=s0 + lo, e=s0 + hi)
                (leaves if c["e"] - c["s"] <= leaf_max else nxt).append(c)
        work = nxt
    leaves.sort(key=lambda x: x["s"])
    return dict(T=t, S=s, QL=None if symmetric else ql, QR=qr, blocks=[(x["s"], x["e"]) for x in leaves],
                bounds=[_bound(x, symmetric) for x in leaves], unsplit_blocks=[bool(x.get("unsplit")) for x in leaves],
                splits=splits, unsplit=unsplit, near_singular=near_singular, extra_splits=extra, log=log)


def block_eigvals(t: np.ndarray, s: np.ndarray | None, starts, symmetric: bool):
    """Eigenvalues of the diagonal blocks of a block upper-triangular pair,
    the dense method the recursion of Sec. 3.3-3.5 hands its small blocks to.
    Symmetric: each block symmetrized, its eigenvalues ascending (LAPACK
    eigvalsh, a library primitive).  Pencil: the generalized eigenvalues of
    each block pair (LAPACK eigvals), real ones ascending, a complex pair as
    (re, +im), (re, -im).  Returns (wr, wi), each of length n."""
    import scipy.linalg as sla
    n = t.shape[0]
    wr, wi = np.empty(n), np.empty(n)
    for a0, a1 in zip(starts[:-1], starts[1:]):
        blk = np.asarray(t[a0:a1, a0:a1], dtype=np.float64)
        if symmetric:
            wr[a0:a1] = np.linalg.eigvalsh(0.5 * (blk + blk.T))
            wi[a0:a1] = 0.0
            continue
        ev = sla.eigvals(blk, np.asarray(s[a0:a1, a0:a1], dtype=np.float64))
        real = sorted(z.real for z in ev if z.imag == 0.0)
        pairs = sorted((z.real, abs(z.imag)) for z in ev if z.imag > 0.0)
        out = [(x, 0.0) for x in real]
        for x, y in pairs:
            out += [(x, y), (x, -y)]
        wr[a0:a1] = [x for x, _ in out]
        wi[a0:a1] = [y for _, y in out]
    return wr, wi
