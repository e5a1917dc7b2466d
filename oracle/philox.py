"""Philox4x32-10 counter-based generator, written from its published
definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC 2011, Sec. 3.3 and Table 2).

One round maps a 4-word counter (c0, c1, c2, c3) under a 2-word key (k0, k1)
through two 32x32 -> 64-bit products with the multipliers M0, M1:

    (hi0, lo0) = M0 * c0,   (hi1, lo1) = M1 * c2
    round(c)   = (hi1 ^ c1 ^ k0,  lo1,  hi0 ^ c3 ^ k1,  lo0)

and the key is advanced by the Weyl constants (W0, W1) between rounds.
Ten rounds give Philox4x32-10.

Test infrastructure: this file is part of the CPU oracle.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)

# Stream tags (fourth counter word) that separate the method's random draws.
S_INIT = 0xA    # initial offsets
S_INTEG = 0xB   # integrand parameters
S_PROP = 0xC    # offset proposals of the optimiser
S_PERM = 0xE    # sort keys of the pixel permutation (swap mutation)
S_SWAP = 0xF    # XOR masks of the swap passes


def philox4x32_10(counter, key) -> np.ndarray:
    """Philox4x32-10 of ``counter`` (array [..., 4] of uint32-valued ints)
    under ``key`` = (k0, k1).  Returns uint32 array [..., 4]."""
    ctr = np.asarray(counter, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = (ctr[..., i] for i in range(4))
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    m0, m1 = np.uint64(M0), np.uint64(M1)
    for rnd in range(10):
        if rnd > 0:
            k0 = np.uint64((int(k0) + W0) & 0xFFFFFFFF)
            k1 = np.uint64((int(k1) + W1) & 0xFFFFFFFF)
        p0 = m0 * c0          # < 2**64: exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def seed_key(seed: int):
    """Key words of a 64-bit seed: (low 32 bits, high 32 bits)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def draw(index, word1, problem: int, stream: int, seed: int) -> np.ndarray:
    """Philox output at counters (index, word1, problem, stream)."""
    index = np.asarray(index, dtype=np.uint64)
    word1 = np.broadcast_to(np.asarray(word1, dtype=np.uint64), index.shape)
    ctr = np.stack([index, word1,
                    np.full(index.shape, problem, dtype=np.uint64),
                    np.full(index.shape, stream, dtype=np.uint64)], axis=-1)
    return philox4x32_10(ctr, seed_key(seed))


def q16_pair(words: np.ndarray) -> np.ndarray:
    """Q0.16 offset from the top 16 bits of words 0 and 1: uint16 [..., 2]."""
    return (words[..., :2] >> np.uint32(16)).astype(np.uint16)
