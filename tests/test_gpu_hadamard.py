"""GPU parity of the Hadamard sketch (SRHT, Sec. 1.2.1) against the oracle.

The device transforms D [A | b] in passes of 8 index bits (registers and
one LDS exchange per block of 256 rows), then forms each sampled row from
the untransformed top bits with fp64 sums; b is column n of the work buffers,
or, when n fills whole column tiles (a multiple of 64 fp32 / 32 fp64
columns), a vector of its own with its own first pass (m' >= 256) and view
passes.  Bars: integer inputs
with d a power of four (so d^{-1/2} is a power of two) give bit-exact SA and
Sb; random inputs agree to a relative Frobenius error of 1e-5 (fp32) / 1e-12
(fp64), and every entry lies within (2 L + 16) u d^{-1/2} sum_i |[A | b]_i|
of the oracle (L = log2 m', the depth of the transform); at 2^21 + 5 rows
(m' = 2^22) sampled rows of SA are recomputed by the oracle one by one; a
solve with the SRHT reaches RE <= 1e-6.
"""
import math

import numpy as np
import pytest

from oracle import metrics as OM
from oracle import sketch as OS
from workloads import dense_gaussian, dense_ill_conditioned

pytestmark = pytest.mark.gpu


def _dev(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


CASES = [
    # m, n, d, dtype
    (1000, 7, 40, np.float64),
    (1024, 3, 1024, np.float32),
    (5, 2, 4, np.float32),
    (4097, 33, 130, np.float32),      # m' = 8192: two levels of the transform
    (20000, 64, 256, np.float64),     # m' = 32768
    (3000, 300, 300, np.float32),     # many column tiles
    (1, 1, 1, np.float64),
]


def _sketch(sns, torch, A, b, d, seed):
    SA, Sb = sns.sketch(_dev(A, torch), _dev(b, torch), "hadamard", d, seed)
    torch.cuda.synchronize()
    return SA.cpu().numpy().astype(np.float64), Sb.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("m,n,d,dt", [
    (1000, 7, 64, np.float64), (4097, 33, 256, np.float32), (5, 2, 4, np.float64),
    # b as a vector of its own: first pass only (m' = 2^15, 2^9), first pass
    # and one view pass (m' = 2^17), and m' < 256 (the view of pass 1)
    (20000, 64, 1024, np.float32), (300, 32, 64, np.float64), (70000, 64, 256, np.float32),
    (100, 64, 64, np.float32)])
def test_integer_inputs_bit_exact(gpu_lib, m, n, d, dt):
    import torch
    rng = np.random.default_rng(m + n)
    A = rng.integers(-8, 9, size=(m, n)).astype(dt)
    b = rng.integers(-8, 9, size=m).astype(dt)
    SA, Sb = _sketch(gpu_lib, torch, A, b, d, 42)
    SAr, Sbr = OS.hadamard_apply(A, b, 42, d)
    assert np.array_equal(SA, SAr)
    assert np.array_equal(Sb, Sbr)


@pytest.mark.parametrize("m,n,d,dt", CASES)
def test_random_inputs_within_tolerance(gpu_lib, m, n, d, dt):
    import torch
    rng = np.random.default_rng(7 * m + n)
    A = rng.standard_normal((m, n)).astype(dt)
    b = rng.standard_normal(m).astype(dt)
    SA, Sb = _sketch(gpu_lib, torch, A, b, d, 7)
    SAr, Sbr = OS.hadamard_apply(A, b, 7, d)
    full, ref = np.column_stack([SA, Sb]), np.column_stack([SAr, Sbr])
    tol = 1e-5 if dt == np.float32 else 1e-12
    assert np.linalg.norm(full - ref) <= tol * np.linalg.norm(ref)
    u = 2.0 ** -24 if dt == np.float32 else 2.0 ** -53
    L = max(0, (m - 1).bit_length())
    colsum = np.abs(np.column_stack([A, b]).astype(np.float64)).sum(axis=0) / math.sqrt(d)
    assert np.all(np.abs(full - ref) <= (2 * L + 16) * u * colsum[None, :] + 1e-300)


@pytest.mark.parametrize("n", [32, 64])
def test_full_depth_sampled_rows(gpu_lib, n):
    """2^21 + 5 rows (m' = 2^22: two full passes, 64 rows summed per sampled
    row); n = 32 keeps b as column n, n = 64 transforms it as a vector."""
    import torch
    m, d = (1 << 21) + 5, 1024
    p = dense_gaussian(m, n, seed=51, dtype=np.float32)
    SA, Sb = _sketch(gpu_lib, torch, p.A, p.b, d, 3)
    mp = OS.hadamard_padded_rows(m)
    rows = OS.hadamard_rows(3, d, mp)
    signs = OS.hadamard_signs(3, m).astype(np.float64)
    Ab = np.column_stack([p.A, p.b]).astype(np.float64)
    # b's entry on its own, within the entrywise bound of the random cases
    L = (mp - 1).bit_length()
    bbound = (2 * L + 16) * 2.0 ** -24 * np.abs(p.b.astype(np.float64)).sum() / math.sqrt(d)
    for k in (0, 1, 511, 1023):
        h = OS.hadamard_sign_matrix(rows[k:k + 1], mp)[0, :m]
        ref = (h * signs) @ Ab / math.sqrt(d)
        got = np.concatenate([SA[k], [Sb[k]]])
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref), k
        assert abs(float(Sb[k]) - ref[-1]) <= bbound, k


def test_hadamard_solve_reaches_target(gpu_lib):
    import torch
    p = dense_ill_conditioned(1 << 17, 64, seed=52, cond=1e6)
    x, info = gpu_lib.lstsq(_dev(p.A, torch), _dev(p.b, torch), "hadamard", 256, 42, refine=True,
                            max_iters=100, rtol=1e-6)
    assert info.status == 0
    xs = OM.lstsq_exact(p.A, p.b)
    assert OM.metrics(p.A, p.b, x.cpu().numpy(), xs)["RE"] <= 1e-6


@pytest.mark.parametrize("off,extra", [(1, 3), (0, 1), (2, 4)])
def test_strided_views_of_A(gpu_lib, off, extra):
    """A given as a column window of a wider array (row stride n + extra,
    first column at offset off): odd strides and offsets take the
    elementwise reads of the first pass, even ones the paired reads."""
    import torch
    m, n, d = 5000, 37, 256  # d a power of four: integer inputs give exact results
    rng = np.random.default_rng(off * 10 + extra)
    big = rng.integers(-8, 9, size=(m, n + extra)).astype(np.float32)
    A = big[:, off:off + n]
    b = rng.integers(-8, 9, size=m).astype(np.float32)
    Adev = _dev(big, torch)[:, off:off + n]
    assert Adev.stride(0) == n + extra
    SA, Sb = gpu_lib.sketch(Adev, _dev(b, torch), "hadamard", d, 5)
    torch.cuda.synchronize()
    SAr, Sbr = OS.hadamard_apply(np.ascontiguousarray(A), b, 5, d)
    assert np.array_equal(SA.cpu().numpy().astype(np.float64), SAr)
    assert np.array_equal(Sb.cpu().numpy().astype(np.float64), Sbr)
