"""GPU parity of the CountSketch hash and apply (Sec. 1.2.2) against the oracle.

Bar: hash indices and signs bit-exact; integer-valued inputs give bit-exact
SA and Sb (every partial sum is an exactly representable integer, so any
summation order agrees); random inputs agree to a relative Frobenius error
of 1e-5 (fp32) / 1e-12 (fp64); repeated calls are bit-identical.
"""
import numpy as np
import pytest

from oracle import sketch as OS

pytestmark = pytest.mark.gpu


def _dev(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("seed", [0, 42, (1 << 40) + 3])
@pytest.mark.parametrize("d", [1, 7, 200, 1024, 4000, (1 << 31) - 1])
@pytest.mark.parametrize("i0,count", [(0, 1000), (1, 999), ((1 << 32) - 3, 64), (5, 1), (0, 0)])
def test_hash_bit_exact(gpu_lib, seed, d, i0, count):
    import torch
    sns = gpu_lib
    h = torch.empty(max(count, 1), dtype=torch.int32, device="cuda")
    s = torch.empty(max(count, 1), dtype=torch.int8, device="cuda")
    sns.sns_hash(seed, d, i0, count, h, s)
    torch.cuda.synchronize()
    hr, sr = OS.countsketch_hash(seed, d, i0, count)
    assert np.array_equal(h.cpu().numpy()[:count].view(np.uint32), hr)
    assert np.array_equal(s.cpu().numpy()[:count], sr)


CASES = [
    # m, n, d, dtype
    (5000, 13, 50, np.float32),
    (20000, 50, 200, np.float64),
    (70000, 256, 1024, np.float32),
    (3000, 300, 400, np.float32),      # two column tiles
    (100000, 16, 64, np.float32),      # few long buckets: segmented reduction
    (1000, 1, 1000, np.float64),       # d = m, single column
    (4099, 129, 130, np.float64),      # ragged fp64, two column tiles
    (777, 3, 5, np.float32),
    (40000, 64, 2048, np.float64),     # staged placing with 96 KB of LDS per work-group
]


def _run(sns, torch, A, b, d, seed, acc64=False, ld_pad=0):
    if ld_pad:
        full = np.zeros((A.shape[0], A.shape[1] + ld_pad), dtype=A.dtype)
        full[:, :A.shape[1]] = A
        Ad = _dev(full, torch)[:, :A.shape[1]]
    else:
        Ad = _dev(A, torch)
    bd = _dev(b, torch)
    SA, Sb = sns.sketch(Ad, bd, "count", d, seed, accum_fp64=acc64)
    torch.cuda.synchronize()
    return SA.cpu().numpy(), Sb.cpu().numpy()


@pytest.mark.parametrize("m,n,d,dt", CASES)
def test_integer_inputs_bit_exact(gpu_lib, m, n, d, dt):
    import torch
    rng = np.random.default_rng(m + n)
    A = rng.integers(-8, 9, size=(m, n)).astype(dt)
    b = rng.integers(-8, 9, size=m).astype(dt)
    SA, Sb = _run(gpu_lib, torch, A, b, d, 42)
    SAr, Sbr = OS.countsketch_apply(A, b, 42, d)
    assert np.array_equal(SA.astype(np.float64), SAr)
    assert np.array_equal(Sb.astype(np.float64), Sbr)


@pytest.mark.parametrize("m,n,d,dt", CASES)
@pytest.mark.parametrize("acc64", [False, True])
def test_random_inputs_within_tolerance(gpu_lib, m, n, d, dt, acc64):
    import torch
    if acc64 and dt == np.float64:
        pytest.skip("fp64 always accumulates in fp64")
    rng = np.random.default_rng(7 * m + n)
    A = rng.standard_normal((m, n)).astype(dt)
    b = rng.standard_normal(m).astype(dt)
    SA, Sb = _run(gpu_lib, torch, A, b, d, 1234)
    SAr, Sbr = OS.countsketch_apply(A, b, 1234, d)
    tol = 1e-12 if dt == np.float64 else 1e-5
    full = np.column_stack([SA, Sb]).astype(np.float64)
    ref = np.column_stack([SAr, Sbr])
    assert np.linalg.norm(full - ref) <= tol * np.linalg.norm(ref)
    # componentwise guard: error within (depth) u sum |S||A|
    absS = abs(OS.countsketch_matrix(1234, d, m))
    bound = np.column_stack([absS @ np.abs(A.astype(np.float64)), absS @ np.abs(b.astype(np.float64))])
    u = np.finfo(dt).eps / 2
    assert np.all(np.abs(full - ref) <= 128 * u * bound + 1e-300)


def test_padded_leading_dimension(gpu_lib):
    import torch
    rng = np.random.default_rng(3)
    A = rng.integers(-5, 6, size=(6000, 37)).astype(np.float32)
    b = rng.integers(-5, 6, size=6000).astype(np.float32)
    SA, Sb = _run(gpu_lib, torch, A, b, 100, 9, ld_pad=3)
    SAr, Sbr = OS.countsketch_apply(A, b, 9, 100)
    assert np.array_equal(SA.astype(np.float64), SAr) and np.array_equal(Sb.astype(np.float64), Sbr)


def test_deterministic_repeat(gpu_lib):
    import torch
    rng = np.random.default_rng(4)
    A = rng.standard_normal((50000, 64)).astype(np.float32)
    b = rng.standard_normal(50000).astype(np.float32)
    r1 = _run(gpu_lib, torch, A, b, 256, 5)
    r2 = _run(gpu_lib, torch, A, b, 256, 5)
    assert np.array_equal(r1[0].view(np.uint32), r2[0].view(np.uint32))
    assert np.array_equal(r1[1].view(np.uint32), r2[1].view(np.uint32))


def test_sketch_without_b(gpu_lib):
    import torch
    sns = gpu_lib
    rng = np.random.default_rng(5)
    A = rng.integers(-3, 4, size=(3000, 20)).astype(np.float64)
    SA, Sb = sns.sketch(_dev(A, torch), None, "count", 60, 77)
    torch.cuda.synchronize()
    assert Sb is None
    assert np.array_equal(SA.cpu().numpy(), OS.countsketch_apply(A, None, 77, 60)[0])


def test_largest_sketch_size(gpu_lib):
    """d = 16384, the most buckets the sort's LDS histograms take: integer
    inputs give bit-exact SA and Sb."""
    import torch
    m, n, d = 200000, 8, 16384
    rng = np.random.default_rng(16384)
    A = rng.integers(-8, 9, size=(m, n)).astype(np.float32)
    b = rng.integers(-8, 9, size=m).astype(np.float32)
    SA, Sb = _run(gpu_lib, torch, A, b, d, 11)
    SAr, Sbr = OS.countsketch_apply(A, b, 11, d)
    assert np.array_equal(SA.astype(np.float64), SAr)
    assert np.array_equal(Sb.astype(np.float64), Sbr)


def test_staged_and_direct_placing_agree(gpu_lib):
    """The bucket sort places a work-group's keys through LDS when they fit
    (at most 1024 keys per wave-block) and scatters them directly otherwise,
    one form for a whole batch.  A problem solved alone (staged) and next to
    a 5,000,000-row problem (whose 1280-key wave-blocks put the batch on the
    direct scatter) gives the same bits: either way the rows of a bucket are
    summed in ascending row order."""
    import torch
    sns = gpu_lib
    rng = np.random.default_rng(99)
    As = _dev(rng.standard_normal((100003, 16)).astype(np.float32), torch)
    bs = _dev(rng.standard_normal(100003).astype(np.float32), torch)
    Ab = _dev(rng.standard_normal((5_000_000, 1)).astype(np.float32), torch)
    bb = _dev(rng.standard_normal(5_000_000).astype(np.float32), torch)
    x_solo, i_solo = sns.lstsq(As, bs, "count", 64, 21)
    xs, infos = sns.lstsq_batched([As, Ab], [bs, bb], [64, 8], [21, 5], refine=False)
    assert i_solo.status == 0 and infos[0].status == 0 and infos[1].status == 0
    assert np.array_equal(x_solo.cpu().numpy().view(np.uint64), xs[0].cpu().numpy().view(np.uint64))
    assert i_solo.sketch_resid == infos[0].sketch_resid
    x_big, _ = sns.lstsq(Ab, bb, "count", 8, 5)
    assert np.array_equal(x_big.cpu().numpy().view(np.uint64), xs[1].cpu().numpy().view(np.uint64))
