"""GPU parity of the Gaussian sketch on the matrix cores (Sec. 1.2.1).

The device multiplies the same bf16 values the oracle uses (table values of G
and bf16(A), bf16(b)), so products are exact and only the fp32 accumulation
order differs: SA and Sb agree to a relative Frobenius error of 1e-5, and
every entry lies within (K-terms) u32 sum |G| |bf16(A)| of the oracle.  At
the full 262144 x 512, d = 2048 size, sampled rows of SA are checked one by
one.  The sketch-and-precondition solve with this sketch reaches the
residual-error target.
"""
import math

import numpy as np
import pytest

from oracle import metrics as OM
from oracle import sketch as OS
from oracle import solve as OSV
from workloads import dense_scaled_columns

pytestmark = pytest.mark.gpu


def _dev(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("m,n,d", [(4096, 64, 256), (10000, 100, 200), (3000, 257, 300), (777, 5, 130),
                                   (50000, 512, 1024), (40013, 512, 1000), (20011, 1100, 1160)])
def test_gaussian_sketch_matches_oracle(gpu_lib, m, n, d):
    import torch
    rng = np.random.default_rng(m + n + d)
    A = rng.standard_normal((m, n)).astype(np.float32)
    b = rng.standard_normal(m).astype(np.float32)
    SA, Sb = gpu_lib.sketch(_dev(A, torch), _dev(b, torch), "gaussian", d, 99)
    torch.cuda.synchronize()
    SA, Sb = SA.cpu().numpy().astype(np.float64), Sb.cpu().numpy().astype(np.float64)
    SAr, Sbr = OS.gaussian_apply(A, b, 99, d)
    full, ref = np.column_stack([SA, Sb]), np.column_stack([SAr, Sbr])
    assert np.linalg.norm(full - ref) <= 1e-5 * np.linalg.norm(ref)
    G = OS.gaussian_matrix(99, d, m)
    bound = (np.abs(G) @ np.abs(np.column_stack([OS.bf16_round(A), OS.bf16_round(b)]))) / math.sqrt(d)
    u = 2.0 ** -24
    assert np.all(np.abs(full - ref) <= (m / 8 + 64) * u * bound + 1e-30)


def test_gaussian_sketch_deterministic_and_seed_dependent(gpu_lib):
    import torch
    rng = np.random.default_rng(5)
    A = _dev(rng.standard_normal((20000, 96)).astype(np.float32), torch)
    b = _dev(rng.standard_normal(20000).astype(np.float32), torch)
    s1 = gpu_lib.sketch(A, b, "gaussian", 384, 7)
    s2 = gpu_lib.sketch(A, b, "gaussian", 384, 7)
    s3 = gpu_lib.sketch(A, b, "gaussian", 384, 8)
    torch.cuda.synchronize()
    assert torch.equal(s1[0], s2[0]) and torch.equal(s1[1], s2[1])
    assert not torch.equal(s1[0], s3[0])


def test_gaussian_sketch_full_size_sampled_rows(gpu_lib):
    """262144 x 512 fp32, d = 2048: rows of SA checked one by one."""
    import torch
    p = dense_scaled_columns(262144, 512, seed=1003)
    SA, Sb = gpu_lib.sketch(_dev(p.A, torch), _dev(p.b, torch), "gaussian", 2048, 42)
    torch.cuda.synchronize()
    rows = [0, 1, 127, 128, 1000, 2047]
    G = OS.gaussian_matrix(42, 2048, 262144, rows=rows)
    A16 = OS.bf16_round(p.A)
    ref = (G @ A16) / math.sqrt(2048)
    refb = (G @ OS.bf16_round(p.b)) / math.sqrt(2048)
    got = SA.cpu().numpy()[rows].astype(np.float64)
    gotb = Sb.cpu().numpy()[rows].astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
    assert np.linalg.norm(gotb - refb) <= 1e-5 * np.linalg.norm(refb)


def test_gaussian_sap_sas_reaches_target(gpu_lib):
    import torch
    p = dense_scaled_columns(65536, 128, seed=31)
    x, info = gpu_lib.lstsq(_dev(p.A, torch), _dev(p.b, torch), "gaussian", 512, 42, refine=True,
                            max_iters=100, rtol=1e-6)
    assert info.status == 0
    xs = OM.lstsq_exact(p.A, p.b)
    met = OM.metrics(p.A, p.b, x.cpu().numpy(), xs)
    assert met["RE"] <= 1e-6, met
    r = OSV.sap_sas(p.A, p.b, "gaussian", 42, 512, 100, rtol=1e-6)
    assert abs(info.iters - r.iters) <= 2


def test_gaussian_plain_sketch_and_solve_parity(gpu_lib):
    import torch
    p = dense_scaled_columns(30000, 40, seed=32)
    x, info = gpu_lib.lstsq(_dev(p.A, torch), _dev(p.b, torch), "gaussian", 160, 42)
    r = OSV.sketch_and_solve(p.A, p.b, "gaussian", 42, 160)
    # fp32 sketch of a column-scaled A: x0 agrees to kappa(SA) * 1e-6 or so
    assert np.linalg.norm(x.cpu().numpy() - r.x) <= 1e-3 * np.linalg.norm(r.x)


def test_gaussian_plain_solve_well_conditioned_parity(gpu_lib):
    """N(0,1) FP32 A with d = 4n: x0 from the MFMA sketch within 1e-5 of the
    oracle's sketch-and-solve on the same bf16 values, element by element
    (scaled by max|x0|) and in norm."""
    import torch
    from workloads import dense_gaussian
    p = dense_gaussian(30000, 40, seed=33, dtype=np.float32)
    x, info = gpu_lib.lstsq(_dev(p.A, torch), _dev(p.b, torch), "gaussian", 160, 42)
    assert info.status == 0
    r = OSV.sketch_and_solve(p.A, p.b, "gaussian", 42, 160)
    xg = x.cpu().numpy()
    assert np.max(np.abs(xg - r.x)) <= 1e-5 * np.max(np.abs(r.x)), np.max(np.abs(xg - r.x))
    assert np.linalg.norm(xg - r.x) <= 1e-5 * np.linalg.norm(r.x)
