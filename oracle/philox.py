"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11) and the Gaussian sketch
built from it -- TEST INFRASTRUCTURE ONLY.

Written from the published definition, independently of the device code: a
round maps the counter (c0, c1, c2, c3) with key (k0, k1) to
    (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)),
M0 = 0xD2511F53, M1 = 0xCD9E8D57, and the key is bumped by the Weyl
constants (0x9E3779B9, 0xBB67AE85) between rounds; 10 rounds.

Gaussian sketch element i (row-major over rows x l): counter c = i // 2 =
(c mod 2^32, c div 2^32, 0, 0), key = (seed mod 2^32, seed div 2^32); the
words x0, x1 give u1 = (x0 + 1)/2^32, u2 = x1/2^32 and the Box-Muller pair
(r cos 2 pi u2, r sin 2 pi u2), r = sqrt(-2 ln u1); element 2c is the first,
2c+1 the second.  Values are then rounded to BF16.
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Vectorised over arrays of counters: ctr = (c0, c1, c2, c3), key = (k0, k1)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) for x in ctr)
    k0, k1 = (np.asarray(x, dtype=np.uint64) for x in key)
    for _ in range(10):
        p0 = np.uint64(M0) * c0
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return c0, c1, c2, c3


def gaussian_sketch(rows: int, l: int, seed: int) -> np.ndarray:
    """rows x l standard normals (float64, before BF16 rounding)."""
    total = rows * l
    ncount = (total + 1) // 2
    c = np.arange(ncount, dtype=np.uint64)
    x0, x1, _, _ = philox4x32_10((c & np.uint64(MASK), c >> np.uint64(32), np.zeros_like(c), np.zeros_like(c)),
                                 (np.uint64(seed & MASK), np.uint64((seed >> 32) & MASK)))
    u1 = (x0.astype(np.float64) + 1.0) / 4294967296.0
    u2 = x1.astype(np.float64) / 4294967296.0
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * ncount)
    z[0::2] = r * np.cos(2 * np.pi * u2)
    z[1::2] = r * np.sin(2 * np.pi * u2)
    return z[:total].reshape(rows, l)
