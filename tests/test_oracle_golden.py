"""The oracle still reproduces the stored fixtures of tests/golden/."""
import os
import struct

import numpy as np

from oracle import sketch as S

G = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(G, name)) as f:
        return [ln.split() for ln in f if not ln.startswith("#")]


def test_gaussian_table_fixture():
    T = S.gaussian_table()
    for q, bits, val in _rows("gaussian_table_bf16.txt"):
        assert float(val) == T[int(q)]
        f32 = struct.unpack("<f", struct.pack("<I", int(bits, 16) << 16))[0]
        assert f32 == T[int(q)]


def test_hash_fixture():
    for i, h, s in _rows("hash_seed42_d200.txt"):
        hh, ss = S.countsketch_hash(42, 200, int(i), 1)
        assert int(hh[0]) == int(h) and int(ss[0]) == int(s)


def test_sketch_fixture():
    import importlib.util
    spec = importlib.util.spec_from_file_location("mg", os.path.join(G, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    A, b = mg.small_integer_problem()
    SA, Sb = S.countsketch_apply(A, b, 5, 8)
    ref = np.array([[float(v) for v in r] for r in _rows("sketch_small.txt")])
    assert np.array_equal(np.column_stack([SA, Sb]), ref)
