"""Philox4x32-10, vectorised over numpy arrays.

The paper does not name its random generator (Section 2.2 only says selections
use the alias method).  The simulation contract of this project uses the
counter-based Philox4x32 generator with 10 rounds, as published by Salmon,
Moraes, Dror and Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC'11):
a round multiplies counter words 0 and 2 by two fixed 32-bit constants, keeps
both 32-bit halves of each product, and mixes them with words 1 and 3 and the
key; the key is bumped by two Weyl constants between rounds.

Inputs are broadcastable arrays of 32-bit values; outputs are four uint64
arrays holding 32-bit values.
"""
import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_M0 = np.uint64(0xD2511F53)   # multiplier applied to counter word 0
_M1 = np.uint64(0xCD9E8D57)   # multiplier applied to counter word 2
_W0 = 0x9E3779B9              # key bump, word 0 (golden ratio)
_W1 = 0xBB67AE85              # key bump, word 1 (sqrt(3) - 1)
ROUNDS = 10


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=ROUNDS):
    """Return the four 32-bit output words for counter (c0..c3) and key (k0, k1)."""
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + _W0) & 0xFFFFFFFF
            k1 = (k1 + _W1) & 0xFFFFFFFF
        prod0 = _M0 * c0            # < 2^64: exact in uint64
        prod1 = _M1 * c2
        hi0, lo0 = prod0 >> np.uint64(32), prod0 & _MASK
        hi1, lo1 = prod1 >> np.uint64(32), prod1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return c0, c1, c2, c3


def key_of_seed(seed):
    """Key words (low, high) of a 64-bit seed."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32
