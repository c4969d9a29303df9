"""Philox counter-based generator, written from its published definition.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Philox-N x W-R (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11, Section 3 and Table 2) maps a counter of N words of
W bits and a key of N/2 words to N output words through R rounds.  Each round
multiplies two of the counter words by fixed odd multipliers, keeps the high
and low halves of the double-width products, xors the high halves with the
other two counter words and the round key, and permutes the words.  The key is
bumped by the two Weyl constants after every round.

The paper (Sketch 'n Solve) draws its sketch from "random" signs and
positions without naming a generator; this implementation fixes Philox4x32-10
as the generator for every random quantity of the method (reading C-1 in the
design notes).  The multipliers and Weyl constants are the ones the SC'11
paper tabulates for Philox4x32 and Philox4x64.

The structure is written once, generically over the word width, so that the
64-bit instance can be checked against an independent implementation
(numpy.random.Philox, which is Philox4x64-10) and that check covers the round
function and key schedule that the 32-bit instance shares.  The 32-bit
instance, with its own multipliers and Weyl constants, is checked block for
block against PyTorch's header-only Philox4x32-10 engine, a second
implementation that shares no code with this one.
"""
from __future__ import annotations

import numpy as np

# SC'11 Table 2 constants.
PHILOX_M4x32 = (0xD2511F53, 0xCD9E8D57)
PHILOX_W32 = (0x9E3779B9, 0xBB67AE85)  # golden ratio, sqrt(3) - 1
PHILOX_M4x64 = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
PHILOX_W64 = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)


def _round(ctr, key, M, mulhilo, xor):
    """One Philox-4 round: (c0,c1,c2,c3) -> (hi1^c1^k0, lo1, hi0^c3^k1, lo0)."""
    c0, c1, c2, c3 = ctr
    k0, k1 = key
    hi0, lo0 = mulhilo(M[0], c0)
    hi1, lo1 = mulhilo(M[1], c2)
    return (xor(xor(hi1, c1), k0), lo1, xor(xor(hi0, c3), k1), lo0)


def _philox4(ctr, key, rounds, M, W, mulhilo, xor, add):
    ctr = tuple(ctr)
    key = tuple(key)
    for r in range(rounds):
        if r > 0:
            key = (add(key[0], W[0]), add(key[1], W[1]))
        ctr = _round(ctr, key, M, mulhilo, xor)
    return ctr


# ---- 32-bit words on numpy uint32 arrays (vectorised over counters) --------

def _mulhilo32(a, b):
    p = np.uint64(a) * np.asarray(b, dtype=np.uint64)
    return (p >> np.uint64(32)).astype(np.uint32), (p & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def _xor32(a, b):
    return np.bitwise_xor(np.asarray(a, dtype=np.uint32), np.asarray(b, dtype=np.uint32))


def _add32(a, b):
    return np.uint32((int(a) + int(b)) & 0xFFFFFFFF)


def philox4x32(c0, c1, c2, c3, k0, k1, rounds: int = 10):
    """Philox4x32-R on arrays of counters; returns four uint32 arrays."""
    ctr = tuple(np.asarray(c, dtype=np.uint32) for c in (c0, c1, c2, c3))
    key = (np.uint32(k0), np.uint32(k1))
    return _philox4(ctr, key, rounds, PHILOX_M4x32, PHILOX_W32, _mulhilo32, _xor32, _add32)


# ---- 64-bit words on Python integers (used to pin the structure) ----------

_MASK64 = (1 << 64) - 1


def _mulhilo64(a, b):
    p = int(a) * int(b)
    return (p >> 64) & _MASK64, p & _MASK64


def philox4x64(ctr, key, rounds: int = 10):
    """Philox4x64-R on one counter (four Python ints) and key (two ints)."""
    return _philox4(tuple(int(c) for c in ctr), tuple(int(k) for k in key), rounds,
                    PHILOX_M4x64, PHILOX_W64, _mulhilo64,
                    lambda a, b: (int(a) ^ int(b)) & _MASK64,
                    lambda a, b: (int(a) + int(b)) & _MASK64)
