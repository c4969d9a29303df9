"""Pins of the oracle's Philox generator (SC'11 definition).

The round function and key schedule are written once, generically over the
word width; the 64-bit instance is compared with numpy.random.Philox (an
independent Philox4x64-10), which pins the shared structure.  The 32-bit
instance, with its own multipliers and Weyl constants, is compared with
PyTorch's header-only Philox4x32-10 engine (ATen/core/PhiloxRNGEngine.h,
compiled here with g++ into a small known-answer program), an implementation
that shares no code with the oracle; it is also evaluated both vectorised on
numpy uint32 arrays and on plain Python integers.
"""
import os
import shutil
import subprocess

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


_KAT_SRC = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
// argv: triples (key, counter words 2-3, counter words 0-1) as 64-bit numbers;
// prints the four 32-bit output words of each block
int main(int argc, char** argv) {
  for (int a = 1; a + 2 < argc; a += 3) {
    at::Philox4_32 e(strtoull(argv[a], 0, 0), strtoull(argv[a + 1], 0, 0),
                     strtoull(argv[a + 2], 0, 0));
    unsigned w[4];
    for (int j = 0; j < 4; ++j) w[j] = e();
    std::printf("%u %u %u %u\n", w[0], w[1], w[2], w[3]);
  }
  return 0;
}
"""


def _torch_philox_blocks(tmp_path, triples):
    """Philox4x32-10 blocks from PyTorch's engine: key = (k0, k1) = the 64-bit
    seed, counter = (c0, c1, c2, c3) = (offset lo, offset hi, subsequence lo,
    subsequence hi)."""
    torch = pytest.importorskip("torch")
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    hdr = os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(hdr):
        pytest.skip("g++ or PyTorch's Philox header not available")
    src = tmp_path / "kat.cpp"
    exe = tmp_path / "kat"
    src.write_text(_KAT_SRC)
    subprocess.run([gxx, "-O1", "-std=c++17", "-I", inc, str(src), "-o", str(exe)], check=True,
                   capture_output=True)
    args = [str(v) for t in triples for v in t]
    out = subprocess.run([str(exe)] + args, check=True, capture_output=True, text=True).stdout
    return [tuple(int(v) for v in line.split()) for line in out.splitlines()]


def _kat_triples():
    rng = np.random.default_rng(2024)
    m64 = (1 << 64) - 1
    t = [(0, 0, 0), (m64, m64, m64), (0xDEADBEEF01234567, 5, 7),
         (0x243F6A8885A308D3, 0x299F31D0A4093822, 0x0370734413198A2E)]
    for _ in range(124):
        t.append(tuple(int(v) * 2 + 1 for v in rng.integers(0, 2**63, size=3, dtype=np.int64)))
    return t


def _oracle_block(key, sub, off, mod=P):
    a = lambda v: np.array([v & 0xFFFFFFFF], dtype=np.uint32)
    w = mod.philox4x32(a(off), a(off >> 32), a(sub), a(sub >> 32), key & 0xFFFFFFFF, key >> 32)
    return tuple(int(x[0]) for x in w)


def test_philox4x32_matches_pytorch_engine(tmp_path):
    triples = _kat_triples()
    ref = _torch_philox_blocks(tmp_path, triples)
    assert len(ref) == len(triples)
    for (key, sub, off), blk in zip(triples, ref):
        assert _oracle_block(key, sub, off) == blk, (key, sub, off)


@pytest.mark.parametrize("which,idx", [("PHILOX_M4x32", 0), ("PHILOX_M4x32", 1),
                                       ("PHILOX_W32", 0), ("PHILOX_W32", 1)])
def test_philox4x32_known_answers_catch_a_wrong_constant(tmp_path, monkeypatch, which, idx):
    """A constant changed in the oracle (one bit of one multiplier or Weyl
    constant) no longer matches the independent engine."""
    triples = _kat_triples()[:8]
    ref = _torch_philox_blocks(tmp_path, triples)
    good = list(getattr(P, which))
    good[idx] ^= 1 << 9
    monkeypatch.setattr(P, which, tuple(good))
    assert any(_oracle_block(k, q, o) != blk for (k, q, o), blk in zip(triples, ref))
