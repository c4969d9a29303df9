"""The benchmark workloads at their full sizes, in the configuration the
benchmark times: the 4,194,304 x 256 FP32 ill-conditioned problem with the
CountSketch (d = 1024, seed 42), the 262,144 x 512 FP32 problem with the
Gaussian sketch (d = 2048), and the Sec. 3.1 family at 1,000,000 x 1000 FP64
(d = 4000), each solved by SAP-SAS or SAA-SAS to rtol 1e-6; and the
16,777,216 x 1000 CSR problem (d = 4000) by plain sketch-and-solve, against
the oracle's sketch-and-solve element by element.

The oracle recomputes sampled buckets of SA one by one (every row the hash
sends to the bucket, signed, summed in fp64) and all of Sb; the refined
answer is checked against the least-squares solution of the same data taken
from one FP64 Householder QR of [A | b] on the host (x* = R^{-1} c and the
optimal residual norm |rho| from the last diagonal entry).
"""
import numpy as np
import pytest

from oracle import sketch as OS
import workloads
from oracle import solve as OSV
from workloads import dense_ill_conditioned, dense_scaled_columns, sparse_csr

# generating the data (about 8 s) and the host QR of [A | b] (about a minute)
# dominate the time
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(400)]

M, N, D, SEED = 4194304, 256, 1024, 42


@pytest.fixture(scope="module")
def problem():
    return dense_ill_conditioned(M, N, seed=1001)


def _dev(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_sketch_sampled_buckets(gpu_lib, problem):
    import torch
    p = problem
    SA, Sb = gpu_lib.sketch(_dev(p.A, torch), _dev(p.b, torch), "count", D, SEED)
    torch.cuda.synchronize()
    SA, Sb = SA.cpu().numpy().astype(np.float64), Sb.cpu().numpy().astype(np.float64)
    h, s = OS.countsketch_hash(SEED, D, 0, M)
    s = s.astype(np.float64)
    # Sb: every bucket
    Sbr = np.bincount(h, weights=s * p.b.astype(np.float64), minlength=D)
    absb = np.bincount(h, weights=np.abs(p.b.astype(np.float64)), minlength=D)
    u = 2.0 ** -24
    assert np.all(np.abs(Sb - Sbr) <= 128 * u * absb + 1e-300)
    # SA: sampled buckets, each recomputed from its own rows
    rng = np.random.default_rng(7)
    for k in [0, 1, 511, 1023] + list(rng.choice(D, size=12, replace=False)):
        rows = np.nonzero(h == k)[0]
        block = p.A[rows].astype(np.float64)
        ref = (s[rows, None] * block).sum(axis=0)
        bound = 128 * u * np.abs(block).sum(axis=0)
        assert np.all(np.abs(SA[k] - ref) <= bound + 1e-300), int(k)


def _lstsq_by_qr(A, b):
    """x* and the optimal residual norm from one FP64 Householder QR of [A | b]
    (LAPACK): R = [[R11, c], [0, rho]] gives x* = R11^{-1} c, |rho| = ||b - A x*||."""
    m, n = A.shape
    Ab = np.empty((m, n + 1), dtype=np.float64)
    Ab[:, :n] = A
    Ab[:, n] = b
    R = np.linalg.qr(Ab, mode="r")
    del Ab
    return np.linalg.solve(np.triu(R[:n, :n]), R[:n, n]), abs(R[n, n])


def _residual_error(A, dx, rho, blk=1 << 18):
    """||A dx|| / rho, with A taken to FP64 one row block at a time."""
    ss = sum(float(np.sum((A[i:i + blk].astype(np.float64) @ dx) ** 2)) for i in range(0, A.shape[0], blk))
    return np.sqrt(ss) / rho


def test_refined_solve_reaches_target(gpu_lib, problem):
    import torch
    p = problem
    x, info = gpu_lib.lstsq(_dev(p.A, torch), _dev(p.b, torch), "count", D, SEED, refine=True,
                            max_iters=100, rtol=1e-6)
    assert info.status == 0
    assert info.iters <= 40
    xs, rho = _lstsq_by_qr(p.A, p.b)
    re = _residual_error(p.A, x.cpu().numpy() - xs, rho)
    assert re <= 1e-6, re


def test_gaussian_full_size_solve(gpu_lib):
    """262,144 x 512 FP32, columns scaled over three decades, Gaussian sketch
    d = 2048 on the bf16 matrix cores, SAP-SAS to rtol 1e-6."""
    import torch
    p = dense_scaled_columns(262144, 512, seed=1003)
    x, info = gpu_lib.lstsq(_dev(p.A, torch), _dev(p.b, torch), "gaussian", 2048, SEED, refine=True,
                            max_iters=100, rtol=1e-6)
    assert info.status == 0
    xs, rho = _lstsq_by_qr(p.A, p.b)
    re = _residual_error(p.A, x.cpu().numpy() - xs, rho)
    assert re <= 1e-6, re


@pytest.fixture(scope="module")
def paper_problem(gpu_lib):
    """Sec. 3.1 family, 1,000,000 x 1000 FP64: kappa 1e10, optimal residual
    beta = 1e-10, drawn on the device; x is the least-squares solution by
    construction (b - A x is beta times a unit vector orthogonal to range A)."""
    import torch
    A, b, x = workloads.paper_benchmark_device(1000000, 1000, 1005, device=torch.device("cuda:0"))
    torch.cuda.synchronize()
    return A, b, x


@pytest.mark.parametrize("kind,refine,zeta", [("count", "sap", 1), ("count", "saa", 1),
                                              ("hadamard", "sap", 1), ("sparse", "sap", 4)])
def test_paper_family_full_size(gpu_lib, paper_problem, kind, refine, zeta):
    import torch
    A, b, xs = paper_problem
    x, info = gpu_lib.lstsq(A, b, kind, 4000, SEED, refine=refine, max_iters=100, rtol=1e-6,
                            zeta=zeta)
    assert info.status == 0
    dx = x - xs
    re = float(torch.linalg.norm(A @ dx)) / 1e-10
    fe = float(torch.linalg.norm(dx) / torch.linalg.norm(xs))
    assert re <= 1e-6, (re, fe)
    # sigma_min = 1e-10 = beta and ||x|| = 1, so ||dx|| <= ||A dx|| / sigma_min
    # gives FE <= RE
    assert fe <= 1e-6, (re, fe)


@pytest.fixture(scope="module")
def csr_problem(gpu_lib):
    """16,777,216 x 1000 CSR (d = 4000) and the oracle's sketch-and-solve x0."""
    p = sparse_csr(1 << 24, 1000, seed=1002)
    return p, OSV.sketch_and_solve(p.A, p.b, "count", SEED, 4000).x


def test_csr_full_size_plain_solve(gpu_lib, csr_problem):
    """Plain sketch-and-solve at full size, the benchmark's setting: the CSR
    sketch accumulates in FP64 and rounds SA and Sb to FP32, then the FP64
    QR.  kappa(SA) is about 4, so x0 moves by a few times FP32 rounding.
    Every element of x0 is within 1e-5 of the oracle's, scaled by its largest
    entry, and the accum_fp64 flag (meaningful for dense A only) changes no
    bit."""
    import torch
    p, xr = csr_problem
    A = p.A
    M = gpu_lib.CsrMatrix(_dev(A.indptr.astype(np.int32), torch), _dev(A.indices.astype(np.int32), torch),
                          _dev(A.data, torch), A.shape)
    b = _dev(p.b, torch)
    x, info = gpu_lib.lstsq(M, b, "count", 4000, SEED)
    assert info.status == 0
    xg = x.cpu().numpy()
    assert np.max(np.abs(xg - xr)) <= 1e-5 * np.max(np.abs(xr)), np.max(np.abs(xg - xr))
    assert np.linalg.norm(xg - xr) <= 1e-5 * np.linalg.norm(xr)
    x2, _ = gpu_lib.lstsq(M, b, "count", 4000, SEED, accum_fp64=True)
    assert np.array_equal(x2.cpu().numpy(), xg)
