"""The C ABI library loads, exports every symbol include/sns.h declares, and
rejects bad arguments on the host (no device work is enqueued for them)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sns.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sns_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    import paper_2409_14309_amd as sns
    lib = sns.load()
    decl = _declared()
    assert "sns_lstsq" in decl and "sns_sketch_apply" in decl
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) <= set(sns.exported_symbols())


def test_status_strings_and_version():
    import paper_2409_14309_amd as sns
    assert sns.sns_status_string(0) == "SNS_OK"
    assert sns.sns_status_string(4) == "SNS_ERR_RANK_DEFICIENT"
    assert sns.sns_version() >= 100


def test_host_side_argument_checks():
    import paper_2409_14309_amd as sns
    lib = sns.load()
    nb = C.c_size_t()
    sk = sns.Sketch(0, 64, 1)
    fake = 0x1000  # never dereferenced: every call below fails validation first
    cases = [
        (sns.Matrix(1000, 0, 0, 0, fake, 0, None, None, 0), sk, 2),       # n = 0
        (sns.Matrix(1000, 100, 0, 0, fake, 100, None, None, 0), sk, 2),   # d < n
        (sns.Matrix(50, 10, 0, 0, fake, 10, None, None, 0), sk, 2),       # m < d
        (sns.Matrix(1000, 10, 0, 0, fake, 5, None, None, 0), sk, 2),      # ld < n
        (sns.Matrix(1000, 10, 7, 0, fake, 10, None, None, 0), sk, 3),     # bad dtype
        (sns.Matrix(1000, 10, 0, 0, None, 10, None, None, 0), sk, 1),     # null values
        (sns.Matrix(1000, 10, 1, 0, fake, 10, None, None, 0), sns.Sketch(1, 64, 1), 3),  # gaussian f64
        (sns.Matrix(1000, 10, 0, 0, fake, 10, None, None, 0), sns.Sketch(5, 64, 1), 1),  # bad kind
        (sns.Matrix(0, 10, 0, 0, fake, 10, None, None, 0), sk, 2),         # m = 0
        (sns.Matrix(100000, 10, 0, 0, fake, 10, None, None, 0), sns.Sketch(0, 16385, 1), 2),  # d > 16384
        (sns.Matrix(1000, 10, 0, 0, fake, 10, None, None, 0), sns.Sketch(0, 0, 1), 2),       # d = 0
    ]
    csr = dict(row_ptr=fake, col_idx=fake)
    cases += [
        (sns.Matrix(1000, 10, 0, 1, fake, 0, None, csr["col_idx"], 5), sk, 1),             # no row_ptr
        (sns.Matrix(10000, 4097, 0, 1, fake, 0, csr["row_ptr"], csr["col_idx"], 5),
         sns.Sketch(0, 5000, 1), 2),                                                      # CSR too wide
        (sns.Matrix(1000, 10, 0, 1, fake, 0, csr["row_ptr"], csr["col_idx"], 5),
         sns.Sketch(1, 64, 1), 3),                                                        # gaussian CSR
        (sns.Matrix(1000, 10, 0, 1, fake, 0, csr["row_ptr"], csr["col_idx"], -1), sk, 2),  # nnz < 0
    ]
    for A, s, want in cases:
        assert lib.sns_sketch_workspace_size(C.byref(s), C.byref(A), C.byref(nb)) == want
        assert lib.sns_sketch_apply(C.byref(s), C.byref(A), None, C.c_void_p(fake), None, None,
                                    C.c_void_p(fake), 1 << 30, None) == want
    A = sns.Matrix(1000, 10, 0, 0, fake, 10, None, None, 0)
    assert lib.sns_sketch_workspace_size(C.byref(sk), C.byref(A), C.byref(nb)) == 0 and nb.value > 0
    # b without Sb
    assert lib.sns_sketch_apply(C.byref(sk), C.byref(A), C.c_void_p(fake), C.c_void_p(fake), None,
                                None, C.c_void_p(fake), 1 << 30, None) == 1
    # workspace too small
    assert lib.sns_sketch_apply(C.byref(sk), C.byref(A), None, C.c_void_p(fake), None, None,
                                C.c_void_p(fake), 16, None) == 7
    # the largest sketch the bucket sort takes is accepted; the QR takes d <= 8192
    Aw = sns.Matrix(100000, 10, 0, 0, fake, 10, None, None, 0)
    assert lib.sns_sketch_workspace_size(C.byref(sns.Sketch(0, 16384, 1)), C.byref(Aw),
                                         C.byref(nb)) == 0
    o0 = sns.opts()
    assert lib.sns_lstsq_workspace_size(C.byref(sns.Sketch(0, 8192, 1)), C.byref(Aw), C.byref(o0),
                                        C.byref(nb)) == 0
    assert lib.sns_lstsq_workspace_size(C.byref(sns.Sketch(0, 8193, 1)), C.byref(Aw), C.byref(o0),
                                        C.byref(nb)) == 2
    o = sns.opts(refine=1, max_iters=-1)
    assert lib.sns_lstsq(C.byref(sk), C.byref(A), C.c_void_p(fake), C.c_void_p(fake), C.byref(o),
                         C.c_void_p(fake), 1 << 30, None, None) == 1
    Ac = sns.Matrix(1000, 10, 0, 1, fake, 0, csr["row_ptr"], csr["col_idx"], 50)
    assert lib.sns_sketch_workspace_size(C.byref(sk), C.byref(Ac), C.byref(nb)) == 0 and nb.value > 0
    o = sns.opts(refine=1, max_iters=5)
    assert lib.sns_lstsq(C.byref(sk), C.byref(Ac), C.c_void_p(fake), C.c_void_p(fake), C.byref(o),
                         C.c_void_p(fake), 1 << 30, None, None) == 3                  # CSR refine
    assert lib.sns_qr_solve(10, 20, 0, C.c_void_p(fake), 20, C.c_void_p(fake), C.c_void_p(fake),
                            None, None, C.c_void_p(fake), 1 << 30, None) == 2
    assert lib.sns_hash(1, 0, 0, 10, C.c_void_p(fake), None, None) == 2
    # sparse sign embedding: zeta in 1..64, dense only, zeta * m < 2^31
    Ad = sns.Matrix(1000, 10, 0, 0, fake, 10, None, None, 0)
    for z, want in ((0, 1), (65, 1), (64, 0), (1, 0)):
        ss = sns.Sketch(2, 64, 1, z)
        assert lib.sns_sketch_workspace_size(C.byref(ss), C.byref(Ad), C.byref(nb)) == want
    assert lib.sns_sketch_workspace_size(C.byref(sns.Sketch(2, 64, 1, 4)), C.byref(Ac),
                                         C.byref(nb)) == 3
    Abig = sns.Matrix((1 << 31) - 1, 10, 0, 0, fake, 10, None, None, 0)
    assert lib.sns_sketch_workspace_size(C.byref(sns.Sketch(2, 64, 1, 2)), C.byref(Abig),
                                         C.byref(nb)) == 2
    # Hadamard sketch: dense only, m <= 2^26; workspace holds the m' x (n + 1) buffers
    sh = sns.Sketch(3, 64, 1, 0)
    assert lib.sns_sketch_workspace_size(C.byref(sh), C.byref(Ad), C.byref(nb)) == 0
    assert nb.value >= 1024 * 11 * 4
    assert lib.sns_sketch_workspace_size(C.byref(sh), C.byref(Ac), C.byref(nb)) == 3
    Ahuge = sns.Matrix((1 << 26) + 1, 10, 0, 0, fake, 10, None, None, 0)
    assert lib.sns_sketch_workspace_size(C.byref(sh), C.byref(Ahuge), C.byref(nb)) == 2
    # fp32 column tiles are 64 wide: n = 63 keeps b as column n of m' x 64
    # buffers; n = 64 moves b to m'-vectors beside m' x 64 buffers (one buffer
    # of each for m' = 2^10, two from m' = 2^17 on, where a second pass runs)
    for m, n, want in [(1000, 63, 1024 * 64 * 4), (1000, 64, 1024 * 64 * 4 + 1024 * 4),
                       (70000, 63, 2 * (1 << 17) * 64 * 4),
                       (70000, 64, 2 * ((1 << 17) * 64 * 4 + (1 << 17) * 4))]:
        Ah = sns.Matrix(m, n, 0, 0, fake, n, None, None, 0)
        assert lib.sns_sketch_workspace_size(C.byref(sh), C.byref(Ah), C.byref(nb)) == 0
        assert nb.value == want, (m, n, nb.value, want)
    # refine outside 0..2; SAA-SAS and non-sparse sketches are rejected by batches
    Aa = sns.Matrix(1000, 10, 0, 0, fake, 12, None, None, 0)  # 16-byte rows for refinement
    o3 = sns.opts(refine=3, max_iters=5)
    assert lib.sns_lstsq_workspace_size(C.byref(sk), C.byref(Aa), C.byref(o3), C.byref(nb)) == 1
    o2 = sns.opts(refine=2, max_iters=5)
    assert lib.sns_lstsq_workspace_size(C.byref(sk), C.byref(Aa), C.byref(o2), C.byref(nb)) == 0
    assert nb.value >= 1000 * 12 * 4  # holds Y
    assert lib.sns_lstsq_workspace_size(C.byref(sk), C.byref(Ad), C.byref(o2), C.byref(nb)) == 2
    probs = (sns.Problem * 1)(sns.Problem(sk, Aa, fake, fake, o2))
    assert lib.sns_lstsq_batched_workspace_size(probs, 1, C.byref(nb)) == 1
    probs = (sns.Problem * 1)(sns.Problem(sh, Aa, fake, fake, sns.opts(refine=1, max_iters=5)))
    assert lib.sns_lstsq_batched_workspace_size(probs, 1, C.byref(nb)) == 3


def test_device_gaussian_table_matches_oracle_bits():
    """The library builds its own table (host inverse normal + bf16 rounding);
    it must equal the oracle's table bit for bit."""
    import struct

    import paper_2409_14309_amd as sns
    from oracle.sketch import gaussian_table
    got = sns.sns_gaussian_table()
    ref = np.array([struct.unpack("<I", struct.pack("<f", np.float32(v)))[0] >> 16
                    for v in gaussian_table()], dtype=np.uint16)
    assert np.array_equal(got, ref)


def test_tuning_table_round_trip(tmp_path):
    """Host-only: entries survive save/clear/load; bad entries and malformed
    files are refused and leave the table unchanged."""
    import paper_2409_14309_amd as sns
    sns.load()
    sns.sns_tune_clear()
    a = sns.TuneEntry(0, 256, 1, 1 << 20, 16, 4, 512, 1, 123.5)
    b = sns.TuneEntry(1, 50, 4096, 65535, 16, 1, 64, 2, 7.25, 8)
    sns.sns_tune_set(a)
    sns.sns_tune_set(b)
    sns.sns_tune_set(sns.TuneEntry(0, 256, 1, 1 << 20, 32, 4, 1024, 2, 99.0))  # replaces a
    sns.sns_tune_gather_set(sns.TuneGatherEntry(0, 50, 200, 1, 1 << 22, 8, 4, 60.5))
    sns.sns_tune_gather_set(sns.TuneGatherEntry(0, 50, 200, 1, 1 << 22, 16, 2, 55.0))  # replaces
    sns.sns_tune_qr_set(sns.TuneQrEntry(1, 512, 1, 128, 0, 1, 300.25))
    sns.sns_tune_qr_set(sns.TuneQrEntry(513, 4096, 1, 256, 3, 2, 800.0))
    p1 = tmp_path / "t1.txt"
    sns.sns_tune_save(str(p1))
    sns.sns_tune_clear()
    sns.sns_tune_load(str(p1))
    p2 = tmp_path / "t2.txt"
    sns.sns_tune_save(str(p2))
    assert p1.read_text() == p2.read_text()
    rows = [ln.split() for ln in p1.read_text().splitlines() if not ln.startswith("#")]
    assert rows == [["0", "256", "1", "1048576", "32", "4", "1024", "2", "99.000", "4"],
                    ["1", "50", "4096", "65535", "16", "1", "64", "2", "7.250", "8"],
                    ["G", "0", "50", "200", "1", "4194304", "16", "2", "55.000"],
                    ["Q", "1", "512", "1", "128", "0", "1", "300.250"],
                    ["Q", "513", "4096", "1", "256", "3", "2", "800.000"]]
    import pytest
    with pytest.raises(sns.SnsError):
        sns.sns_tune_set(sns.TuneEntry(0, 64, 1, 10, 8, 2, 64, 1, 0.0))  # (8, 2) not a pass shape
    with pytest.raises(sns.SnsError):  # 6 waves per work-group
        sns.sns_tune_set(sns.TuneEntry(0, 64, 1, 10, 16, 4, 64, 1, 0.0, 6))
    with pytest.raises(sns.SnsError):  # 24 lanes per row: not a power of two
        sns.sns_tune_gather_set(sns.TuneGatherEntry(0, 50, 200, 1, 10, 24, 1, 0.0))
    with pytest.raises(sns.SnsError):  # 128 segments
        sns.sns_tune_gather_set(sns.TuneGatherEntry(0, 50, 200, 1, 10, 16, 128, 0.0))
    with pytest.raises(sns.SnsError):  # configuration 0 holds at most 512 rows
        sns.sns_tune_qr_set(sns.TuneQrEntry(1, 600, 1, 128, 0, 1, 0.0))
    with pytest.raises(sns.SnsError):  # three trailing columns
        sns.sns_tune_qr_set(sns.TuneQrEntry(1, 500, 1, 128, 0, 3, 0.0))
    for text in ("0 64 1 10 16 4 64 1 1.0\n0 64 oops\n",
                 "0 64 1 10 16 4 64 1 1.0 8\n0 64 11 20 16 4 64 1 1.0 2\n",
                 "G 0 50 200 1 10 16 2 1.0\nG 0 50 200 1 10 12 2 1.0\n",
                 "Q 1 512 1 128 0 1 1.0\nQ 1 9000 1 128 4 1 1.0\n",
                 "Q 1 512 1 128\n"):
        bad = tmp_path / "bad.txt"
        bad.write_text(text)
        with pytest.raises(sns.SnsError):
            sns.sns_tune_load(str(bad))
    p3 = tmp_path / "t3.txt"
    sns.sns_tune_save(str(p3))
    assert p3.read_text() == p1.read_text()
    sns.sns_tune_clear()
    if os.path.exists(sns._binding.TUNING_PATH):
        sns.sns_tune_load(sns._binding.TUNING_PATH)


def test_qr_solve_noalloc_host_checks():
    """The allocation-free QR solve rejects bad arguments and sizes whose
    workspace exceeds its 64 MiB static array before touching the device."""
    import paper_2409_14309_amd as sns
    lib = sns.load()
    fake = 0x1000
    f = lib.sns_qr_solve_noalloc
    assert f(200, 50, 1, None, 50, fake, fake, None, None, None) == 1      # null SA
    assert f(200, 50, 1, fake, 50, fake, None, None, None, None) == 1      # null x0
    assert f(200, 50, 7, fake, 50, fake, fake, None, None, None) == 3      # bad dtype
    assert f(40, 50, 1, fake, 50, fake, fake, None, None, None) == 2       # d < n
    assert f(200, 50, 1, fake, 40, fake, fake, None, None, None) == 2      # ld < n
    assert f(8192, 1000, 1, fake, 1000, fake, fake, None, None, None) == 7  # over 64 MiB
    need = C.c_size_t()
    assert lib.sns_qr_solve_workspace_size(4096, 1000, C.byref(need)) == 0
    assert need.value <= 64 << 20  # the size the header promises fits
