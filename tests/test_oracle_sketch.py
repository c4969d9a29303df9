"""Pins of the oracle's CountSketch (Sec. 1.2.2) and Gaussian sketch (Sec. 1.2.1).

CountSketch: S has exactly one +-1 per column (checked on the materialised S),
the sparse-product oracle equals a dense product with S built entry by entry
and an explicit row loop, sketching the identity returns S itself, the map is
linear, row blocks sketched with global offsets add up to the whole, and
E||Sx||^2 = ||x||^2 (statistical).  Hash statistics: bucket counts uniform
(chi-square), signs balanced, consecutive rows independent.
Sparse sign embedding: zeta = 1 is the CountSketch itself; S is the sum of
zeta matrices with one +-1 per column (built here entry by entry from the
per-k hashes), the sparse product equals that dense product and an explicit
loop, the hashes of different k are independent (collision rate 1/d), and
E||Sx||^2 = zeta ||x||^2 (statistical).
Hadamard sketch (SRHT): the popcount sign rows equal scipy.linalg.hadamard
(Sylvester construction) entry for entry; S A equals the product built with
scipy's full Hadamard matrix on the zero-padded, sign-flipped A; sampled rows
are uniform and signs balanced; E||Sx||^2 = ||x||^2 (statistical).
Gaussian table: symmetric, monotone, every entry the bfloat16 rounding of the
normal quantile computed independently by bisection on math.erfc; bfloat16
rounding agrees with torch's float32 -> bfloat16 conversion.
Gaussian apply: the d^{-1/2} scale by E[S^T S] = var(T) I over seeds (a 1/d
scale or none fails it); A and b rounded to bfloat16 exactly as torch rounds
them, and b sketched as one more column of A.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy import stats

from oracle import sketch as S
from workloads import dense_gaussian, sparse_csr


# ---------------------------------------------------------------- hash ----

def test_hash_range_and_offsets():
    for d in (1, 2, 3, 200, 1024, 4000, (1 << 31) - 1):
        h, s = S.countsketch_hash(42, d, 0, 5000)
        assert h.dtype == np.uint32 and s.dtype == np.int8
        assert int(h.max()) < d
        assert set(np.unique(s)) <= {-1, 1}
    h, s = S.countsketch_hash(7, 1000, 0, 10001)
    h2, s2 = S.countsketch_hash(7, 1000, 3333, 5000)   # odd offset: lane parity shifts
    assert np.array_equal(h[3333:8333], h2) and np.array_equal(s[3333:8333], s2)
    h3, _ = S.countsketch_hash(8, 1000, 0, 10001)
    assert np.mean(h3 == h) < 0.01
    e = S.countsketch_hash(7, 1000, 10, 0)
    assert e[0].size == 0


def test_hash_large_row_index():
    # rows beyond 2^33 use the high counter word
    i0 = (1 << 33) + 5
    h, s = S.countsketch_hash(3, 997, i0, 64)
    hlo, _ = S.countsketch_hash(3, 997, 5, 64)
    assert not np.array_equal(h, hlo)


def test_hash_bucket_uniformity_and_sign_balance():
    m, d = 1 << 20, 1000
    h, s = S.countsketch_hash(42, d, 0, m)
    counts = np.bincount(h, minlength=d)
    chi2 = ((counts - m / d) ** 2 / (m / d)).sum()
    p = stats.chi2.sf(chi2, d - 1)
    assert 1e-4 < p < 1 - 1e-4
    assert abs(s.astype(np.int64).sum()) < 5 * math.sqrt(m)
    # consecutive rows (same Philox block) are independent
    a, b = h[0::2] % 8, h[1::2] % 8
    joint = np.bincount(a * 8 + b, minlength=64)
    chi2 = ((joint - joint.sum() / 64) ** 2 / (joint.sum() / 64)).sum()
    assert stats.chi2.sf(chi2, 63) > 1e-4
    assert abs(np.mean(s[0::2].astype(float) * s[1::2])) < 5 / math.sqrt(m / 2)


# --------------------------------------------------------- CountSketch ----

def _dense_S_entrywise(seed, d, m):
    h, s = S.countsketch_hash(seed, d, 0, m)
    M = np.zeros((d, m))
    for i in range(m):
        M[int(h[i]), i] = float(s[i])
    return M


def test_materialised_S_one_signed_entry_per_column():
    M = S.countsketch_matrix(42, 50, 3000).toarray()
    assert np.all((M != 0).sum(axis=0) == 1)
    assert set(np.unique(M[M != 0])) <= {-1.0, 1.0}


def test_countsketch_equals_dense_product_and_loop():
    p = dense_gaussian(700, 9, seed=1)
    SA, Sb = S.countsketch_apply(p.A, p.b, 42, 31)
    M = _dense_S_entrywise(42, 31, 700)
    np.testing.assert_allclose(SA, M @ p.A, rtol=0, atol=1e-12)
    np.testing.assert_allclose(Sb, M @ p.b, rtol=0, atol=1e-12)
    SAl, Sbl = S.countsketch_apply_loop(p.A, p.b, 42, 31)
    np.testing.assert_allclose(SA, SAl, rtol=0, atol=1e-12)
    np.testing.assert_allclose(Sb, Sbl, rtol=0, atol=1e-12)


def test_sketch_of_identity_is_S():
    m, d = 400, 17
    SA, _ = S.countsketch_apply(np.eye(m), None, 5, d)
    assert np.array_equal(SA, _dense_S_entrywise(5, d, m))


def test_linearity_and_augmented_column():
    rng = np.random.default_rng(0)
    A1, A2 = rng.standard_normal((500, 6)), rng.standard_normal((500, 6))
    b = rng.standard_normal(500)
    s1, _ = S.countsketch_apply(A1, None, 9, 40)
    s2, _ = S.countsketch_apply(A2, None, 9, 40)
    s3, _ = S.countsketch_apply(2.0 * A1 - 3.0 * A2, None, 9, 40)
    np.testing.assert_allclose(s3, 2.0 * s1 - 3.0 * s2, atol=1e-12)
    SAb, _ = S.countsketch_apply(np.column_stack([A1, b]), None, 9, 40)
    SA, Sb = S.countsketch_apply(A1, b, 9, 40)
    np.testing.assert_allclose(SAb, np.column_stack([SA, Sb]), atol=1e-13)


def test_row_blocks_with_global_offsets_sum_to_whole():
    rng = np.random.default_rng(1)
    m, n, d, seed = 1000, 5, 23, 77
    A = rng.standard_normal((m, n))
    SA, _ = S.countsketch_apply(A, None, seed, d)
    acc = np.zeros((d, n))
    for r0, r1 in [(0, 333), (333, 334), (334, 1000)]:
        h, s = S.countsketch_hash(seed, d, r0, r1 - r0)
        Sblk = sp.csr_matrix((s.astype(float), (h.astype(int), np.arange(r1 - r0))), shape=(d, r1 - r0))
        acc += Sblk @ A[r0:r1]
    np.testing.assert_allclose(acc, SA, atol=1e-12)


def test_integer_inputs_are_exact():
    rng = np.random.default_rng(2)
    A = rng.integers(-8, 9, size=(3000, 7)).astype(np.float64)
    SA, _ = S.countsketch_apply(A, None, 11, 50)
    assert np.array_equal(SA, np.round(SA))
    assert np.array_equal(SA, _dense_S_entrywise(11, 50, 3000) @ A)


def test_unbiased_norm():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(300)
    vals = []
    for seed in range(400):
        sx, _ = S.countsketch_apply(x[:, None], None, seed, 20)
        vals.append(float(np.sum(sx ** 2)))
    vals = np.array(vals)
    assert abs(vals.mean() - x @ x) < 5 * vals.std() / math.sqrt(len(vals))


def test_csr_input_matches_dense():
    p = sparse_csr(5000, 40, seed=4, nnz_per_col=30, dense_block=40)
    SA, Sb = S.countsketch_apply(p.A, p.b, 42, 160)
    SAd, Sbd = S.countsketch_apply(p.A.toarray(), p.b, 42, 160)
    np.testing.assert_allclose(SA, SAd, atol=1e-12)
    np.testing.assert_allclose(Sb, Sbd, atol=1e-12)


# ------------------------------------------------------------ bfloat16 ----

def test_bf16_round_matches_torch_on_float32_values():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.uniform(-5, 5, 20000),
                        # exact ties between bf16 neighbours
                        (np.arange(1, 400) * 2 + 1).astype(np.float64) * 2.0 ** -8])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    got = S.bf16_round(x32.astype(np.float64))
    assert np.array_equal(got, ref)


def _inv_normal_bisect(p):
    lo, hi = -10.0, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if 0.5 * math.erfc(-mid / math.sqrt(2.0)) < p:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_gaussian_table():
    T = S.gaussian_table()
    assert T.shape == (256,)
    assert np.all(np.diff(T) >= 0)
    assert np.array_equal(T[::-1], -T)
    for q in range(256):
        z = _inv_normal_bisect((q + 0.5) / 256.0)
        ulp = 2.0 ** (math.floor(math.log2(abs(z))) - 7)
        assert abs(T[q] - z) <= 0.5 * ulp + 1e-15
    assert abs(T.mean()) == 0.0
    assert 0.95 < np.mean(T ** 2) < 1.0


def test_gaussian_codes_uniform_and_offsets():
    q = S.gaussian_codes(42, 48, 0, 4000)
    counts = np.bincount(q.ravel(), minlength=256)
    chi2 = ((counts - q.size / 256) ** 2 / (q.size / 256)).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4
    q2 = S.gaussian_codes(42, 48, 1000, 500)
    assert np.array_equal(q[:, 1000:1500], q2)
    q3 = S.gaussian_codes(42, 40, 0, 4000)
    assert np.array_equal(q3, q[:40])


def test_gaussian_sketch_isotropy():
    # E[(G^T G) / d] = var(T) I over the columns of G
    d, m = 2048, 48
    G = S.gaussian_matrix(9, d, m)
    C = G.T @ G / d
    var = np.mean(S.gaussian_table() ** 2)
    assert np.max(np.abs(np.diag(C) - var)) < 6 * var * math.sqrt(2.0 / d)
    off = C - np.diag(np.diag(C))
    assert np.max(np.abs(off)) < 6 * var / math.sqrt(d)


def test_gaussian_apply_scale_by_expected_gram():
    # Sec. 1.2.1: S = d^{-1/2} G, so E[S^T S] = var(T) I.  Sketching the
    # identity (exact in bf16) returns S; its Gram matrix averaged over seeds
    # must show var(T) on the diagonal.  A 1/d scale or no scale misses it by
    # a factor d or 1/d.
    m, d, seeds = 24, 64, 120
    var = float(np.mean(S.gaussian_table() ** 2))
    acc = np.zeros((m, m))
    for sd in range(seeds):
        SA, _ = S.gaussian_apply(np.eye(m), None, 1000 + sd, d)
        acc += SA.T @ SA
    acc /= seeds
    # each diagonal entry is a mean of seeds * d squared table values / d
    sd_diag = var * math.sqrt(2.0 / (d * seeds))
    assert np.max(np.abs(np.diag(acc) - var)) < 6 * sd_diag
    off = acc - np.diag(np.diag(acc))
    assert np.max(np.abs(off)) < 6 * var / math.sqrt(d * seeds)


def test_gaussian_apply_rounds_a_and_b_like_torch_bfloat16():
    # The product is taken with bf16(A) and bf16(b), round to nearest even;
    # torch's float32 -> bfloat16 conversion is an independent rounding.
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(17)
    m, n, d, seed = 300, 5, 32, 77
    A = rng.standard_normal((m, n)).astype(np.float32).astype(np.float64)
    b = rng.standard_normal(m).astype(np.float32).astype(np.float64)
    SA, Sb = S.gaussian_apply(A, b, seed, d)
    G = S.gaussian_matrix(seed, d, m)
    Ab = torch.from_numpy(A.astype(np.float32)).bfloat16().double().numpy()
    bb = torch.from_numpy(b.astype(np.float32)).bfloat16().double().numpy()
    np.testing.assert_allclose(SA, (G @ Ab) / math.sqrt(d), rtol=0, atol=1e-12)
    np.testing.assert_allclose(Sb, (G @ bb) / math.sqrt(d), rtol=0, atol=1e-12)
    # b is treated like a column of A: [A | b] sketched together gives Sb
    SAb, _ = S.gaussian_apply(np.column_stack([A, b]), None, seed, d)
    assert np.array_equal(SAb[:, n], Sb)
    # and the rounding matters at this scale (unrounded b differs)
    assert np.max(np.abs(Sb - (G @ b) / math.sqrt(d))) > 1e-6


# ------------------------------------------------------ sparse sign ----

def test_sparse_sign_zeta_one_is_countsketch():
    p = dense_gaussian(900, 7, seed=5)
    a = S.countsketch_apply(p.A, p.b, 13, 40)
    c = S.sparse_sign_apply(p.A, p.b, 13, 40, 1)
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    h0, s0 = S.countsketch_hash(13, 40, 0, 900)
    h1, s1 = S.sparse_sign_hash(13, 40, 0, 900, 0)
    assert np.array_equal(h0, h1) and np.array_equal(s0, s1)


@pytest.mark.parametrize("zeta", [2, 3, 8])
def test_sparse_sign_structure_product_and_loop(zeta):
    m, d, n, seed = 600, 37, 5, 21
    rng = np.random.default_rng(zeta)
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    # entry by entry: column i gets s_k(i) at row h_k(i) for each k
    M = np.zeros((d, m))
    per_k = []
    for k in range(zeta):
        h, sg = S.sparse_sign_hash(seed, d, 0, m, k)
        Mk = np.zeros((d, m))
        for i in range(m):
            Mk[h[i], i] = sg[i]
        assert np.all((Mk != 0).sum(axis=0) == 1)
        per_k.append(Mk)
        M += Mk
    assert np.array_equal(S.sparse_sign_matrix(seed, d, m, zeta).toarray(), M)
    SA, Sb = S.sparse_sign_apply(A, b, seed, d, zeta)
    np.testing.assert_allclose(SA, M @ A, rtol=0, atol=1e-12)
    np.testing.assert_allclose(Sb, M @ b, rtol=0, atol=1e-12)
    # explicit loop over columns of S (rows of A), all k of a row in turn
    SAl = np.zeros((d, n))
    for i in range(m):
        for Mk in per_k:
            r = int(np.flatnonzero(Mk[:, i])[0])
            SAl[r] += Mk[r, i] * A[i]
    np.testing.assert_allclose(SA, SAl, rtol=0, atol=1e-12)


def test_sparse_sign_hashes_independent_across_k():
    d, m = 64, 200000
    h0, s0 = S.sparse_sign_hash(3, d, 0, m, 0)
    h1, s1 = S.sparse_sign_hash(3, d, 0, m, 1)
    rate = float(np.mean(h0 == h1))
    assert abs(rate - 1.0 / d) < 5 * math.sqrt((1.0 / d) / m)
    agree = float(np.mean(s0 == s1))
    assert abs(agree - 0.5) < 5 * math.sqrt(0.25 / m)


def test_sparse_sign_norm_scales_with_zeta():
    rng = np.random.default_rng(6)
    x = rng.standard_normal(300)
    vals = []
    for seed in range(300):
        sx, _ = S.sparse_sign_apply(x[:, None], None, seed, 20, 4)
        vals.append(float(np.sum(sx ** 2)))
    vals = np.array(vals)
    assert abs(vals.mean() - 4 * (x @ x)) < 5 * vals.std() / math.sqrt(len(vals))


# ----------------------------------------------------------- hadamard ----

@pytest.mark.parametrize("mp", [1, 2, 8, 64, 256])
def test_hadamard_sign_rows_equal_sylvester(mp):
    import scipy.linalg as sla
    H = S.hadamard_sign_matrix(np.arange(mp), mp)
    assert np.array_equal(H, sla.hadamard(mp).astype(np.float64))


@pytest.mark.parametrize("m,n,d", [(1000, 7, 40), (1024, 3, 1024), (5, 2, 3), (300, 1, 64)])
def test_hadamard_apply_equals_full_transform(m, n, d):
    import scipy.linalg as sla
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    SA, Sb = S.hadamard_apply(A, b, 17, d)
    mp = S.hadamard_padded_rows(m)
    assert mp >= m and mp < 2 * max(m, 1) + 1 and (mp & (mp - 1)) == 0
    Ap = np.zeros((mp, n + 1))
    Ap[:m, :n] = A
    Ap[:m, n] = b
    Ap[:m] *= S.hadamard_signs(17, m)[:, None]
    full = sla.hadamard(mp).astype(np.float64) @ Ap
    ref = full[S.hadamard_rows(17, d, mp)] / math.sqrt(d)
    np.testing.assert_allclose(np.column_stack([SA, Sb]), ref, rtol=0, atol=1e-10)


def test_hadamard_rows_uniform_and_signs_balanced():
    rows = S.hadamard_rows(5, 64000, 64)
    assert rows.min() >= 0 and rows.max() < 64
    counts = np.bincount(rows, minlength=64)
    assert stats.chisquare(counts).pvalue > 1e-4
    sg = S.hadamard_signs(5, 100000).astype(np.int64)
    assert abs(sg.mean()) < 5 / math.sqrt(100000)


def test_hadamard_unbiased_norm():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(200)
    vals = []
    for seed in range(300):
        sx, _ = S.hadamard_apply(x[:, None], None, seed, 16)
        vals.append(float(np.sum(sx ** 2)))
    vals = np.array(vals)
    assert abs(vals.mean() - x @ x) < 5 * vals.std() / math.sqrt(len(vals))
