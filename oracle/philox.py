"""Counter-based Gaussian source for RURV's random matrix (Alg. 1 line 1).

Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11): a 4 x 32-bit counter and a 2 x 32-bit key;
each of the ten rounds multiplies counter words 0 and 2 by the constants
0xD2511F53 and 0xCD9E8D57, and mixes the high halves with the other two words
and the key; the key is bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85)
between rounds.

Element (i, j) of the n x n matrix, column-major index e = i + j*n, uses
counter (e mod 2^32, e div 2^32, tag, 0) with tag = side (0 right, 1 left) and
key (seed mod 2^32, seed div 2^32).  The four output words make two 53-bit
uniforms u1 = (hi64(w0, w1) >> 11 + 1/2) 2^-53 in (0, 1) and
u2 = (hi64(w2, w3) >> 11) 2^-53, and the Box-Muller transform
z = sqrt(-2 ln u1) cos(2 pi u2) gives one N(0,1) sample.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Vectorized Philox4x32-10.  ctr: 4 arrays (or ints) of uint32 words,
    key: 2 words.  Returns 4 uint32 arrays."""
    c0, c1, c2, c3 = [np.asarray(x, dtype=np.uint64) & MASK32 for x in ctr]
    k0, k1 = [np.asarray(x, dtype=np.uint64) & MASK32 for x in key]
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + np.uint64(W0)) & MASK32
            k1 = (k1 + np.uint64(W1)) & MASK32
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK32, lo1, (hi0 ^ c3 ^ k1) & MASK32, lo0
    return [c.astype(np.uint32) for c in (c0, c1, c2, c3)]


def gaussian_matrix(n: int, seed: int, tag: int) -> np.ndarray:
    """n x n N(0,1) matrix (float64, Fortran order) from Philox4x32-10."""
    e = np.arange(n * n, dtype=np.uint64)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    w = philox4x32_10((e & MASK32, e >> np.uint64(32), np.full_like(e, tag), np.zeros_like(e)),
                      (seed & 0xFFFFFFFF, seed >> 32))
    w = [x.astype(np.uint64) for x in w]
    x1 = ((w[1] << np.uint64(32)) | w[0]) >> np.uint64(11)
    x2 = ((w[3] << np.uint64(32)) | w[2]) >> np.uint64(11)
    u1 = (x1.astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = x2.astype(np.float64) * 2.0 ** -53
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return np.asfortranarray(z.reshape((n, n), order="F"))
