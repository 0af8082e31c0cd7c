"""Oracle: Philox4x32-10 counter-based generator and Box-Muller normals.

TEST INFRASTRUCTURE ONLY.

Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC 2011): ten rounds of two 32x32->64-bit
multiplications with multipliers 0xD2511F53 and 0xCD9E8D57, and a Weyl key
schedule with increments 0x9E3779B9 and 0xBB67AE85.  Normals from the
Box-Muller transform (Box and Muller, 1958).

Channel-noise convention shared with the HIP simulator (each side implements
it from this definition): the complex noise sample with flat index n of the
IQ array uses counter (n mod 2^32, n div 2^32, 0, 0) and key (seed mod 2^32,
seed div 2^32); outputs x0, x1 give u1 = (x0 + 1) / 2^32 and u2 = x1 / 2^32,
and the sample is sigma/sqrt(2) * sqrt(-2 ln u1) * (cos 2 pi u2 + i sin 2 pi u2).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10; all inputs uint32 arrays (broadcastable)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint32) for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint32)
    k1 = np.asarray(k1, dtype=np.uint32)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    c0, c1, c2, c3 = c0.copy(), c1.copy(), c2.copy(), c3.copy()
    k0 = np.broadcast_to(k0, c0.shape).copy()
    k1 = np.broadcast_to(k1, c0.shape).copy()
    with np.errstate(over="ignore"):
        for r in range(10):
            p0 = M0 * c0.astype(np.uint64)
            p1 = M1 * c2.astype(np.uint64)
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & MASK).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & MASK).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
            if r < 9:
                k0 = k0 + W0
                k1 = k1 + W1
    return c0, c1, c2, c3


def channel_noise(n_start: int, count: int, seed: int, sigma: float) -> np.ndarray:
    """Complex128 noise samples for flat indices [n_start, n_start + count)."""
    n = np.arange(n_start, n_start + count, dtype=np.uint64)
    lo = (n & MASK).astype(np.uint32)
    hi = (n >> np.uint64(32)).astype(np.uint32)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    x0, x1, _, _ = philox4x32_10(lo, hi, 0, 0, seed & 0xFFFFFFFF, seed >> 32)
    u1 = (x0.astype(np.float64) + 1.0) / 4294967296.0
    u2 = x1.astype(np.float64) / 4294967296.0
    r = np.sqrt(-2.0 * np.log(u1)) * (sigma / np.sqrt(2.0))
    return r * np.exp(2j * np.pi * u2)
