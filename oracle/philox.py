"""Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11, Section 3.2 and Table 2).

The generator maps a 128-bit counter (c0, c1, c2, c3) and a 64-bit key
(k0, k1) to four 32-bit words.  One round multiplies c0 and c2 by two fixed
odd constants, keeps both halves of each 64-bit product, and mixes the high
halves with the other two counter words and the key; between rounds the key
is advanced by two Weyl constants.  Ten rounds are applied.

Two independent implementations live here: ``philox_scalar`` uses Python's
unbounded integers and is used for tiny cross-checks; ``philox`` is the same
definition on numpy uint64 arrays (32x32 -> 64-bit products cannot overflow
uint64), used everywhere else.

Pinned by: bit-equality with rocRAND's philox4x32_10 engine (a third-party
implementation, called through its public API from a host program in the
test-suite), bit-equality between the two implementations here and the C
oracle, and uniformity / independence statistics of the derived hash.
"""
from __future__ import annotations

import numpy as np

# Round multipliers and key increments (SC'11, Table 2 / Section 3.2).
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
ROUNDS = 10

_MASK32 = 0xFFFFFFFF


def philox_scalar(ctr, key):
    """Philox4x32-10 of one counter, Python integers.  ctr: 4 ints, key: 2 ints."""
    c0, c1, c2, c3 = (int(v) & _MASK32 for v in ctr)
    k0, k1 = (int(v) & _MASK32 for v in key)
    for r in range(ROUNDS):
        if r:
            k0 = (k0 + PHILOX_W0) & _MASK32
            k1 = (k1 + PHILOX_W1) & _MASK32
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 32, p0 & _MASK32
        hi1, lo1 = p1 >> 32, p1 & _MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return (c0, c1, c2, c3)


def philox(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.

    All arguments broadcast against each other (numpy integer arrays or ints,
    values taken modulo 2**32).  Returns four uint32 arrays.
    """
    m = np.uint64(_MASK32)
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(
        *(np.asarray(v, dtype=np.uint64) & m for v in (c0, c1, c2, c3, k0, k1)))
    c0, c1, c2, c3 = (v.copy() for v in (c0, c1, c2, c3))
    k0 = k0.copy()
    k1 = k1.copy()
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    sh = np.uint64(32)
    for r in range(ROUNDS):
        if r:
            k0 = (k0 + np.uint64(PHILOX_W0)) & m
            k1 = (k1 + np.uint64(PHILOX_W1)) & m
        p0 = c0 * m0
        p1 = c2 * m1
        hi0, lo0 = p0 >> sh, p0 & m
        hi1, lo1 = p1 >> sh, p1 & m
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(v.astype(np.uint32) for v in (c0, c1, c2, c3))


def split64(v):
    """(lo32, hi32) of a 64-bit unsigned value or array."""
    v = np.asarray(v, dtype=np.uint64)
    return v & np.uint64(_MASK32), v >> np.uint64(32)
