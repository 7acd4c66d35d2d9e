"""Philox4x64-10 counter-based generator, vectorised over numpy uint64 arrays.

Written from the published definition (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11): a 4 x 64-bit counter and a
2 x 64-bit key; each of the ten rounds multiplies counter words 0 and 2 by two
fixed odd constants, keeps the high and low halves of the 128-bit products,
and recombines them with the other counter words and the key by XOR; between
rounds the key is bumped by two Weyl constants.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np

_U64 = np.uint64
MUL0 = _U64(0xD2E7470EE14C6C93)
MUL1 = _U64(0xCA5A826395121157)
WEYL0 = _U64(0x9E3779B97F4A7C15)
WEYL1 = _U64(0xBB67AE8584CAA73B)
_LO32 = _U64(0xFFFFFFFF)
_S32 = _U64(32)


def mulhilo64(a, b):
    """Full 64 x 64 -> 128-bit product of uint64 arrays, as (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    with np.errstate(over="ignore"):
        lo = a * b
        a_lo, a_hi = a & _LO32, a >> _S32
        b_lo, b_hi = b & _LO32, b >> _S32
        ll = a_lo * b_lo
        lh = a_lo * b_hi
        hl = a_hi * b_lo
        hh = a_hi * b_hi
        mid = (ll >> _S32) + (lh & _LO32) + (hl & _LO32)
        hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x64 rounds on broadcastable uint64 arrays; returns 4 arrays."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64)
    k1 = np.asarray(k1, dtype=np.uint64)
    for rnd in range(10):
        if rnd:
            with np.errstate(over="ignore"):
                k0 = k0 + WEYL0
                k1 = k1 + WEYL1
        hi0, lo0 = mulhilo64(MUL0, c0)
        hi1, lo1 = mulhilo64(MUL1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3
