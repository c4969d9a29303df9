"""GPU parity of the CountSketch over CSR rows (Sec. 1.2.2 applied to a
sparse A) against the oracle, and of plain sketch-and-solve on a CSR matrix.

Bars: integer-valued inputs give bit-exact SA and Sb; random values agree to
a relative Frobenius error of 1e-5 (fp32) / 1e-12 (fp64) and componentwise
within 128 u sum |S||A|; repeated calls are bit-identical; the CSR and dense
forms of one matrix give the same sketch; at the 16,777,216 x 1000 size
(d = 4000) sampled buckets of SA and all of Sb are checked against the oracle.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import sketch as OS
from oracle import solve as OSV
from workloads import sparse_csr

pytestmark = pytest.mark.gpu


def _dev(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _csr_dev(sns, torch, A):
    return sns.CsrMatrix(_dev(A.indptr.astype(np.int32), torch), _dev(A.indices.astype(np.int32), torch),
                         _dev(A.data, torch), A.shape)


def _random_csr(m, n, density, seed, dt, integer=False, long_rows=0):
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=density, format="csr", random_state=rng, dtype=np.float64)
    if long_rows:  # a few full rows (longer than one 64-lane batch)
        A = A.tolil()
        for i in rng.choice(m, size=long_rows, replace=False):
            A[i, :] = rng.standard_normal(n) + 0.5
        A = A.tocsr()
    A.sort_indices()
    if integer:
        A.data = rng.integers(-8, 9, size=A.nnz).astype(np.float64)
        A.data[A.data == 0] = 1.0
    else:
        A.data = rng.standard_normal(A.nnz)
    A = sp.csr_matrix((A.data.astype(dt), A.indices.astype(np.int32), A.indptr.astype(np.int32)),
                      shape=(m, n))
    b = (rng.integers(-8, 9, size=m) if integer else rng.standard_normal(m)).astype(dt)
    return A, b


CASES = [
    # m, n, d, density, dtype, long rows
    (20000, 50, 200, 0.02, np.float32, 0),
    (20000, 50, 200, 0.02, np.float64, 3),
    (100000, 300, 1024, 0.002, np.float32, 5),    # mostly empty rows
    (5000, 700, 800, 0.05, np.float64, 2),
    (4099, 129, 130, 0.3, np.float32, 0),          # ragged, dense-ish
    (70000, 16, 64, 0.2, np.float32, 0),           # few long buckets
    (3000, 1, 5, 0.5, np.float64, 0),              # single column
    (9000, 4096, 4096, 0.0005, np.float32, 1),     # widest CSR row supported
]


def _run(sns, torch, A, b, d, seed, acc64=False):
    SA, Sb = sns.sketch(_csr_dev(sns, torch, A), None if b is None else _dev(b, torch), "count", d,
                        seed, accum_fp64=acc64)
    torch.cuda.synchronize()
    return SA.cpu().numpy(), (None if Sb is None else Sb.cpu().numpy())


@pytest.mark.parametrize("m,n,d,dens,dt,lr", CASES)
def test_csr_integer_bit_exact(gpu_lib, m, n, d, dens, dt, lr):
    import torch
    A, b = _random_csr(m, n, dens, m + n, dt, integer=True, long_rows=lr)
    SA, Sb = _run(gpu_lib, torch, A, b, d, 42)
    SAr, Sbr = OS.countsketch_apply(A, b, 42, d)
    assert np.array_equal(SA.astype(np.float64), SAr)
    assert np.array_equal(Sb.astype(np.float64), Sbr)


@pytest.mark.parametrize("m,n,d,dens,dt,lr", CASES)
@pytest.mark.parametrize("acc64", [False, True])
def test_csr_random_within_tolerance(gpu_lib, m, n, d, dens, dt, lr, acc64):
    import torch
    if acc64 and dt == np.float64:
        pytest.skip("fp64 always accumulates in fp64")
    A, b = _random_csr(m, n, dens, 3 * m + n, dt, long_rows=lr)
    SA, Sb = _run(gpu_lib, torch, A, b, d, 1234, acc64)
    SAr, Sbr = OS.countsketch_apply(A, b, 1234, d)
    tol = 1e-12 if dt == np.float64 else 1e-5
    full = np.column_stack([SA, Sb]).astype(np.float64)
    ref = np.column_stack([SAr, Sbr])
    assert np.linalg.norm(full - ref) <= tol * np.linalg.norm(ref)
    absS = abs(OS.countsketch_matrix(1234, d, m))
    absA = abs(A.astype(np.float64))
    bound = np.column_stack([(absS @ absA).toarray(), absS @ np.abs(b.astype(np.float64))])
    u = np.finfo(dt).eps / 2
    assert np.all(np.abs(full - ref) <= 128 * u * bound + 1e-300)
    if dt == np.float32:
        # the CSR sketch sums in fp64 whatever accum_fp64 says: each entry is
        # the fp32 rounding of a sum whose own error is fp64-sized
        u64 = np.finfo(np.float64).eps / 2
        assert np.all(np.abs(full - ref) <= u * np.abs(ref) + 128 * u64 * bound + 1e-300)


def test_csr_matches_dense_form(gpu_lib):
    import torch
    sns = gpu_lib
    A, b = _random_csr(30000, 64, 0.05, 8, np.float32, integer=True)
    SAc, Sbc = _run(sns, torch, A, b, 256, 77)
    SAd, Sbd = sns.sketch(_dev(A.toarray(), torch), _dev(b, torch), "count", 256, 77)
    torch.cuda.synchronize()
    assert np.array_equal(SAc, SAd.cpu().numpy()) and np.array_equal(Sbc, Sbd.cpu().numpy())


def test_csr_deterministic_repeat(gpu_lib):
    import torch
    A, b = _random_csr(60000, 200, 0.01, 4, np.float32, long_rows=4)
    r1 = _run(gpu_lib, torch, A, b, 512, 5)
    r2 = _run(gpu_lib, torch, A, b, 512, 5)
    assert np.array_equal(r1[0].view(np.uint32), r2[0].view(np.uint32))
    assert np.array_equal(r1[1].view(np.uint32), r2[1].view(np.uint32))


def test_csr_edge_cases(gpu_lib):
    import torch
    sns = gpu_lib
    # no nonzeros at all: SA is zero, Sb still sketches every row of b
    m, n, d = 5000, 10, 40
    A = sp.csr_matrix((np.zeros(0, np.float32), np.zeros(0, np.int32), np.zeros(m + 1, np.int32)),
                      shape=(m, n))
    b = np.random.default_rng(1).integers(-4, 5, size=m).astype(np.float32)
    SA, Sb = _run(sns, torch, A, b, d, 3)
    assert not SA.any()
    assert np.array_equal(Sb.astype(np.float64), OS.countsketch_apply(A, b, 3, d)[1])
    # no b
    A, _ = _random_csr(8000, 30, 0.05, 2, np.float64, integer=True)
    SA, Sb = _run(sns, torch, A, None, 90, 11)
    assert Sb is None
    assert np.array_equal(SA, OS.countsketch_apply(A, None, 11, 90)[0])
    # columns outside [0, n) are ignored
    A, b = _random_csr(6000, 20, 0.1, 5, np.float32, integer=True)
    bad = A.copy()
    bad.indices = bad.indices.copy()
    bad.indices[::7] += 1000
    keep = A.copy()
    keep.data = keep.data.copy()
    keep.data[::7] = 0
    SA, Sb = _run(sns, torch, bad, b, 60, 9)
    assert np.array_equal(SA.astype(np.float64), OS.countsketch_apply(keep, b, 9, 60)[0])


def test_csr_rejects_wide_rows(gpu_lib):
    import torch
    sns = gpu_lib
    A, b = _random_csr(9000, 4097, 0.0005, 1, np.float32)
    with pytest.raises(sns.SnsError):
        _run(sns, torch, A, b, 4097, 1)


@pytest.mark.parametrize("dt,tol", [(np.float64, 1e-12), (np.float32, 1e-5)])
def test_csr_plain_solve_matches_oracle(gpu_lib, dt, tol):
    import torch
    sns = gpu_lib
    p = sparse_csr(200000, 100, seed=21, nnz_per_col=300, dense_block=100, dtype=dt)
    x, info = sns.lstsq(_csr_dev(sns, torch, p.A), _dev(p.b, torch), "count", 400, 42,
                        accum_fp64=True)
    assert info.status == 0
    xr = OSV.sketch_and_solve(p.A, p.b, "count", 42, 400).x
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg - xr) <= tol * np.linalg.norm(xr)


def test_csr_refine_rejected(gpu_lib):
    import torch
    sns = gpu_lib
    A, b = _random_csr(5000, 10, 0.1, 1, np.float32)
    with pytest.raises(sns.SnsError):
        sns.lstsq(_csr_dev(sns, torch, A), _dev(b, torch), "count", 40, 1, refine=True)


def test_csr_full_size_sampled(gpu_lib):
    """The 16,777,216 x 1000 sparse workload with d = 4000: sampled buckets of
    SA (every row hashed to them summed by the oracle) and all of Sb."""
    import torch
    sns = gpu_lib
    m, n, d, seed = 1 << 24, 1000, 4000, 42
    p = sparse_csr(m, n, seed=1002)
    A = p.A
    SA, Sb = _run(sns, torch, A, p.b, d, seed)
    h, s = OS.countsketch_hash(seed, d, 0, m)
    rng = np.random.default_rng(0)
    ks = np.unique(np.concatenate([rng.choice(d, 24, replace=False), [0, d - 1]]))
    for k in ks:
        rows = np.nonzero(h == k)[0]
        ref = np.asarray((sp.csr_matrix(s[rows].astype(np.float64)) @ A[rows].astype(np.float64)).todense()).ravel()
        assert np.linalg.norm(SA[k] - ref) <= 1e-5 * max(np.linalg.norm(ref), 1e-30)
    S = sp.csr_matrix((s.astype(np.float64), (h.astype(np.int64), np.arange(m))), shape=(d, m))
    Sbr = S @ p.b.astype(np.float64)
    assert np.linalg.norm(Sb - Sbr) <= 1e-5 * np.linalg.norm(Sbr)
