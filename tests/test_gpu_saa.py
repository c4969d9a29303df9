"""GPU parity of SAA-SAS (Sec. 2.1: the sketch-and-apply solver) against the
oracle, through sns_lstsq with refine = 2.

The device forms Y = A R^{-1} (fp64 products, stored in A's dtype) and runs
LSQR on Y from r0 = b - A x0.  Bars: with fp64 data and a fixed iteration
count the answer agrees with the oracle's saa_sas to 1e-9 relative (the same
bar as SAP-SAS: kappa(R) ~ 1e3 amplifies the rounding of the sketch); shapes
with ragged row and column tiles of the Y product (n = 2, 130, 200, 300, m
below one tile) are covered (refinement needs 16-byte rows, so n is even).
With fp32 data the oracle rounds its Y to fp32 as the device stores it, and
the forward error agrees to 1e-5 on a well-conditioned problem.  On the ill-conditioned fp32 problem (kappa 1e6) the criterion is
the residual error RE <= 1e-6 against the fp64 least-squares solution, and
SAA and SAP take the same number of iterations within 2 (they are the same
method in exact arithmetic).  Batched calls and the server reject refine = 2.
"""
import numpy as np
import pytest

from oracle import metrics as OM
from oracle import solve as OSV
from workloads import dense_gaussian, dense_ill_conditioned, paper_benchmark

pytestmark = pytest.mark.gpu


def _dev(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("m,n,d", [(20000, 64, 256), (10007, 200, 800), (5000, 130, 520),
                                   (3000, 2, 8), (120, 20, 80), (40000, 300, 1200),
                                   (12000, 256, 1024), (12000, 258, 1032), (12000, 512, 2048),
                                   (12000, 514, 2056)])
def test_saa_fp64_fixed_iterations_matches_oracle(gpu_lib, m, n, d):
    import torch
    p = dense_gaussian(m, n, seed=m + n)
    k = 6
    x, info = gpu_lib.lstsq(_dev(p.A, torch), _dev(p.b, torch), "count", d, 42, refine="saa",
                            max_iters=k, rtol=0.0)
    r = OSV.saa_sas(p.A, p.b, "count", 42, d, k)
    assert info.status == 0
    assert info.iters == r.iters
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg - r.x) <= 1e-9 * np.linalg.norm(r.x)


def test_saa_fp32_well_conditioned_fixed_iterations(gpu_lib):
    import torch
    p = dense_gaussian(50000, 64, seed=22, dtype=np.float32)
    x, info = gpu_lib.lstsq(_dev(p.A, torch), _dev(p.b, torch), "count", 256, 42, refine="saa",
                            max_iters=3, rtol=0.0)
    r = OSV.saa_sas(p.A, p.b, "count", 42, 256, 3, y_dtype=np.float32)
    assert info.iters == 3
    assert np.linalg.norm(x.cpu().numpy() - r.x) <= 1e-5 * np.linalg.norm(r.x)


@pytest.mark.parametrize("m,n,d", [(1 << 17, 64, 256), (200000, 100, 400)])
def test_saa_fp32_illconditioned_stop_rule(gpu_lib, m, n, d):
    import torch
    p = dense_ill_conditioned(m, n, seed=23, cond=1e6)
    A, b = _dev(p.A, torch), _dev(p.b, torch)
    x, info = gpu_lib.lstsq(A, b, "count", d, 42, refine="saa", max_iters=100, rtol=1e-6)
    assert info.status == 0
    xs = OM.lstsq_exact(p.A, p.b)
    met = OM.metrics(p.A, p.b, x.cpu().numpy(), xs)
    assert met["RE"] <= 1e-6, met
    _, info_sap = gpu_lib.lstsq(A, b, "count", d, 42, refine="sap", max_iters=100, rtol=1e-6)
    assert abs(info.iters - info_sap.iters) <= 2


def test_saa_paper_benchmark_fp64(gpu_lib):
    """Sec. 3.1 family (kappa 1e10, beta 1e-10) at a small m: SAA and SAP
    agree with each other and with the oracle's SAA-SAS."""
    import torch
    p = paper_benchmark(20000, 200, seed=31)
    A, b = _dev(p.A, torch), _dev(p.b, torch)
    k = 30
    xa, ia = gpu_lib.lstsq(A, b, "count", 800, 42, refine="saa", max_iters=k, rtol=0.0)
    xp, ip = gpu_lib.lstsq(A, b, "count", 800, 42, refine="sap", max_iters=k, rtol=0.0)
    r = OSV.saa_sas(p.A, p.b, "count", 42, 800, k)
    xa, xp = xa.cpu().numpy(), xp.cpu().numpy()
    # compare in the residual norm: A dx relative to ||b|| (x itself has kappa 1e10 sensitivity)
    nb = np.linalg.norm(p.b)
    assert np.linalg.norm(p.A @ (xa - r.x)) <= 1e-12 * nb
    assert np.linalg.norm(p.A @ (xa - xp)) <= 1e-12 * nb
    xs = OM.lstsq_exact(p.A, p.b)
    assert np.linalg.norm(p.A @ (xa - xs)) <= 1e-12 * nb


def test_saa_rejected_by_batched_calls(gpu_lib):
    import torch
    sns = gpu_lib
    p = dense_gaussian(4000, 16, seed=5, dtype=np.float32)
    with pytest.raises(sns.SnsError):
        sns.lstsq_batched([_dev(p.A, torch)], [_dev(p.b, torch)], [64], [1], refine=2)
