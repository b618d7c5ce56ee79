"""Randomized spectral divide-and-conquer (Sec. 3.3-3.5) on top of the split
step, for the oracle.

Strategy, as the paper describes it:
* symmetric A (Sec. 3.4): bound the spectrum by the Gershgorin interval
  [c - R, c + R] and split at a random point x uniform in [c - R/2, c + R/2];
  the two halves inherit [x, c + R] and [c - R, x]; a split that finds every
  eigenvalue on one side still shrinks the interval (progress);
* pencils (Sec. 3.5): split at the unit circle first; if every eigenvalue is
  inside (outside), try circles of radius 2^{-2^k} (2^{2^k}); a block whose
  eigenvalues lie outside a circle of radius r is continued on the swapped
  pair (B, A), whose eigenvalues are the reciprocals and lie inside 1/r;
  inside a known disk, split by random lines through the middle half of the
  interval of real parts (vertical lines only: the oracle keeps real
  arithmetic, so a complex-conjugate pair is never separated).
The coupling blocks E21 (and F21) are set to zero after each accepted split,
and the transformations are applied to the rest of the pair and accumulated.
"""
from __future__ import annotations

import numpy as np

from .split import split_sym, split_pencil, OK, NO_SPLIT

MAX_TRIES = 8


def _gershgorin(a: np.ndarray):
    c = np.diag(a)
    r = np.sum(np.abs(a), axis=1) - np.abs(c)
    return float(np.min(c - r)), float(np.max(c + r))


def eig_dc(a: np.ndarray, b: np.ndarray | None = None, symmetric: bool = False, leaf_max: int = 64,
           seed: int = 0):
    """Returns dict(T, S, QL, QR, blocks=[(s, e), ...], splits, unsplit)."""
    a = np.array(a, dtype=np.float64)
    n = a.shape[0]
    t = a.copy()
    s = None if symmetric else np.array(b, dtype=np.float64)
    ql = np.eye(n)
    qr = np.eye(n)
    rng = np.random.default_rng(seed)
    if symmetric:
        lo, hi = _gershgorin(a)
        work = [dict(s=0, e=n, mode="line", lo=lo, hi=hi, swapped=False, radius=1.0, tries=0)]
    else:
        work = [dict(s=0, e=n, mode="circle", lo=-1.0, hi=1.0, swapped=False, radius=1.0, tries=0)]
    leaves, splits, unsplit = [], 0, 0
    if n <= leaf_max:
        leaves, work = work, []
    while work:
        nxt = []
        for blk in work:
            s0, e0 = blk["s"], blk["e"]
            m = e0 - s0
            if blk["mode"] == "circle":
                region = {"kind": "disk", "center": 0.0, "radius": blk["radius"]}
            else:
                c, r = 0.5 * (blk["lo"] + blk["hi"]), 0.5 * (blk["hi"] - blk["lo"])
                region = {"kind": "halfplane", "shift": c + (rng.uniform() - 0.5) * r, "scale": r if r > 0 else 1.0}
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
            if res.status != OK or not (0 < k < m):
                nb = dict(blk, tries=blk["tries"] + 1)
                if res.status == NO_SPLIT:
                    all_inside = res.n_inside == m
                    if blk["mode"] == "circle":
                        r0 = blk["radius"]
                        nb["radius"] = (0.5 if r0 >= 1 else r0 * r0) if all_inside else (2.0 if r0 <= 1 else r0 * r0)
                        if nb["tries"] >= 6:
                            nb["mode"] = "line"
                            nb["tries"] = 0
                            if all_inside:
                                nb["lo"], nb["hi"] = -r0, r0
                            else:
                                nb["swapped"] = not blk["swapped"]
                                nb["lo"], nb["hi"] = -1.0 / r0, 1.0 / r0
                    else:
                        if all_inside:
                            nb["hi"] = region["shift"]
                        else:
                            nb["lo"] = region["shift"]
                        nb["tries"] = 0 if nb["hi"] > nb["lo"] else MAX_TRIES
                if nb["tries"] >= MAX_TRIES:
                    unsplit += 1
                    leaves.append(blk)
                else:
                    nxt.append(nb)
                continue
            # accepted: write the split pair, drop the coupling blocks, update the rest
            if symmetric:
                t[s0:e0, s0:e0] = res.A_hat
                t[s0 + k:e0, s0:s0 + k] = 0.0
                t[s0:s0 + k, s0 + k:e0] = 0.0
            else:
                ah, bh = (res.B_hat, res.A_hat) if blk["swapped"] else (res.A_hat, res.B_hat)
                t[s0:e0, s0:e0] = ah
                s[s0:e0, s0:e0] = bh
                t[s0 + k:e0, s0:s0 + k] = 0.0
                s[s0 + k:e0, s0:s0 + k] = 0.0
                t[s0:e0, e0:] = qlb.T @ t[s0:e0, e0:]
                s[s0:e0, e0:] = qlb.T @ s[s0:e0, e0:]
                t[:s0, s0:e0] = t[:s0, s0:e0] @ qrb
                s[:s0, s0:e0] = s[:s0, s0:e0] @ qrb
                ql[:, s0:e0] = ql[:, s0:e0] @ qlb
            qr[:, s0:e0] = qr[:, s0:e0] @ qrb
            c1 = dict(blk, e=s0 + k, tries=0)
            c2 = dict(blk, s=s0 + k, tries=0)
            if blk["mode"] == "circle":
                r0 = blk["radius"]
                c1.update(mode="line", swapped=not blk["swapped"], lo=-1.0 / r0, hi=1.0 / r0)
                c2.update(mode="line", lo=-r0, hi=r0)
            else:
                c1["lo"] = region["shift"]
                c2["hi"] = region["shift"]
            for c in (c1, c2):
                (leaves if c["e"] - c["s"] <= leaf_max else nxt).append(c)
        work = nxt
    leaves.sort(key=lambda x: x["s"])
    return dict(T=t, S=s, QL=None if symmetric else ql, QR=qr, blocks=[(x["s"], x["e"]) for x in leaves],
                splits=splits, unsplit=unsplit)


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
