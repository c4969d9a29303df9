"""Writes the stored fixtures under tests/golden/ from the oracle alone.

    python tests/golden/make_golden.py

Fixtures (all derived from the readings of the paper fixed in the oracle):
  gaussian_table_bf16.txt   T[q] of the Gaussian sketch (Sec. 1.2.1), q = 0..255,
                            as bfloat16 bit patterns and decimal values.
  hash_seed42_d200.txt      CountSketch bucket and sign (Sec. 1.2.2) of rows
                            0..255 and 2^32-2 .. 2^32+1 for seed 42, d = 200.
  sketch_small.txt          SA, Sb of a 64 x 3 integer matrix (seed 5, d = 8):
                            exact integers, so any summation order reproduces them.
"""
import os
import struct
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import sketch as S  # noqa: E402


def bf16_bits(v: float) -> int:
    return struct.unpack("<I", struct.pack("<f", np.float32(v)))[0] >> 16


def small_integer_problem():
    rng = np.random.default_rng(123)
    A = rng.integers(-9, 10, size=(64, 3)).astype(np.float64)
    b = rng.integers(-9, 10, size=64).astype(np.float64)
    return A, b


def main():
    T = S.gaussian_table()
    with open(os.path.join(HERE, "gaussian_table_bf16.txt"), "w") as f:
        f.write("# q bf16_bits value  (T[q] = bf16_rne(Phi^-1((q + 1/2) / 256)))\n")
        for q in range(256):
            f.write(f"{q} 0x{bf16_bits(T[q]):04x} {float(T[q])!r}\n")
    rows = list(range(256)) + [2**32 - 2, 2**32 - 1, 2**32, 2**32 + 1]
    with open(os.path.join(HERE, "hash_seed42_d200.txt"), "w") as f:
        f.write("# row h s  (seed 42, d 200)\n")
        for i in rows:
            h, s = S.countsketch_hash(42, 200, i, 1)
            f.write(f"{i} {int(h[0])} {int(s[0])}\n")
    A, b = small_integer_problem()
    SA, Sb = S.countsketch_apply(A, b, 5, 8)
    with open(os.path.join(HERE, "sketch_small.txt"), "w") as f:
        f.write("# SA | Sb rows for the 64x3 integer problem of make_golden.small_integer_problem, seed 5, d 8\n")
        for k in range(8):
            f.write(" ".join(str(int(v)) for v in list(SA[k]) + [Sb[k]]) + "\n")


if __name__ == "__main__":
    main()
