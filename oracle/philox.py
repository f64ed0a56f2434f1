"""Philox4x32-10 counter-based generator, written from its published
definition (J. Salmon, M. Moraes, R. Dror, D. Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11, Section 4): a 4x32-bit counter is passed through
ten rounds of the Philox S-box, with the 2x32-bit key advanced by the Weyl
constants between rounds.

One round, with counter (c0, c1, c2, c3) and key (k0, k1):
    (hi0, lo0) = M0 * c0,   (hi1, lo1) = M1 * c2      (32x32 -> 64 bit)
    (c0, c1, c2, c3) <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
with M0 = 0xD2511F53, M1 = 0xCD9E8D57; then k0 += 0x9E3779B9 and
k1 += 0xBB67AE85 before the next round.

The paper draws its test matrices in MATLAB without naming a generator; a
counter-based stream lets the GPU regenerate any entry of Omega and Psi from
its indices, so both sides use this published generator.  Vectorised over
NumPy uint64 arrays; pinned by the SC'11 known-answer vectors in
tests/golden/philox4x32_10_kat.txt.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
ROUNDS = 10


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=ROUNDS):
    """Return the four 32-bit output words for counters (c0..c3) (arrays or
    scalars, broadcast together) under key (k0, k1) (Python ints)."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    c0 = c0.copy(); c1 = c1.copy(); c2 = c2.copy(); c3 = c3.copy()
    ka = int(k0) & 0xFFFFFFFF
    kb = int(k1) & 0xFFFFFFFF
    for r in range(rounds):
        if r:
            ka = (ka + W0) & 0xFFFFFFFF
            kb = (kb + W1) & 0xFFFFFFFF
        p0 = M0 * c0                       # exact: both factors < 2^32
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        n0 = hi1 ^ c1 ^ np.uint64(ka)
        n2 = hi0 ^ c3 ^ np.uint64(kb)
        c0, c1, c2, c3 = n0, lo1, n2, lo0
    return c0, c1, c2, c3


def seed_key(seed):
    """Key words from a 64-bit seed: (seed mod 2^32, seed >> 32)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32
