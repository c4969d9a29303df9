"""Pins of the oracle's Philox generator (SC'11 definition).

The round function and key schedule are written once, generically over the
word width; the 64-bit instance is compared with numpy.random.Philox (an
independent Philox4x64-10), which pins the shared structure.  The 32-bit
instance is then pinned by evaluating it both vectorised on numpy uint32
arrays and on plain Python integers.
"""
import numpy as np
import pytest

from oracle import philox as P


def _numpy_blocks(key, counter, nblocks):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(counter, dtype=np.uint64))
    raw = bg.random_raw(4 * nblocks)
    return [tuple(int(v) for v in raw[4 * t:4 * t + 4]) for t in range(nblocks)]


def _bump(ctr, k):
    v = sum(int(c) << (64 * j) for j, c in enumerate(ctr)) + k
    v &= (1 << 256) - 1
    return tuple((v >> (64 * j)) & ((1 << 64) - 1) for j in range(4))


@pytest.mark.parametrize("key,counter", [
    ((0, 0), (0, 0, 0, 0)),
    ((1, 2), (3, 4, 5, 6)),
    ((0xFFFFFFFFFFFFFFFF, 0x0123456789ABCDEF), (0xFFFFFFFFFFFFFFFE, 0xFFFFFFFFFFFFFFFF, 7, 0)),
])
def test_philox4x64_matches_numpy(key, counter):
    # numpy bumps the 256-bit counter before producing each block
    blocks = _numpy_blocks(key, counter, 5)
    for t, blk in enumerate(blocks):
        assert P.philox4x64(_bump(counter, t + 1), key) == blk


def _philox4x32_scalar(ctr, key, rounds=10):
    m32 = (1 << 32) - 1
    return P._philox4(tuple(ctr), tuple(key), rounds, P.PHILOX_M4x32, P.PHILOX_W32,
                      lambda a, b: (((a * b) >> 32) & m32, (a * b) & m32),
                      lambda a, b: (a ^ b) & m32, lambda a, b: (a + b) & m32)


def test_philox4x32_vectorised_equals_integer_evaluation():
    rng = np.random.default_rng(7)
    c = rng.integers(0, 2**32, size=(4, 64), dtype=np.uint64).astype(np.uint32)
    k0, k1 = 0xDEADBEEF, 0x01234567
    w = P.philox4x32(c[0], c[1], c[2], c[3], k0, k1)
    for t in range(64):
        ref = _philox4x32_scalar(tuple(int(c[j, t]) for j in range(4)), (k0, k1))
        assert tuple(int(w[j][t]) for j in range(4)) == ref


def test_philox4x32_rounds_and_key_matter():
    c = np.arange(16, dtype=np.uint32)
    z = np.zeros(16, np.uint32)
    a = P.philox4x32(c, z, z, z, 1, 2)
    b = P.philox4x32(c, z, z, z, 1, 3)
    r7 = P.philox4x32(c, z, z, z, 1, 2, rounds=7)
    assert not np.array_equal(a[0], b[0])
    assert not np.array_equal(a[0], r7[0])


def test_philox4x32_output_bits_balanced_and_avalanche():
    n = 1 << 16
    c0 = np.arange(n, dtype=np.uint32)
    z = np.zeros(n, np.uint32)
    w = P.philox4x32(c0, z, z, z, 42, 0)
    bits = np.unpackbits(np.stack(w).view(np.uint8))
    assert abs(bits.mean() - 0.5) < 0.002
    # flipping one counter bit flips about half of the 128 output bits
    w2 = P.philox4x32(c0 ^ np.uint32(1 << 13), z, z, z, 42, 0)
    flips = np.unpackbits((np.stack(w) ^ np.stack(w2)).view(np.uint8)).reshape(-1).mean()
    assert abs(flips - 0.5) < 0.002
