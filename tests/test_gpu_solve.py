"""GPU parity of the QR solve (Sec. 1.2 step 3) and of sns_lstsq (SAS and
SAP-SAS, Secs. 1.2, 1.3, 2.1) against the oracle.

Bars: fp64 R and x0 from the same SA agree to 1e-12 relative (the LAPACK sign
convention is shared, so R is compared entry by entry); the plain fp64 solve
of the 20000 x 50 workload agrees to 1e-12; fp64 refinement with a fixed
iteration count agrees to 1e-9 (kappa(R) ~ 1e3 amplifies rounding); fp32
refinement on a well-conditioned problem agrees to 1e-5 in forward error;
on the ill-conditioned fp32 problem (kappa 1e6) the criterion is the residual
error RE <= 1e-6 against the fp64 least-squares solution, reached by the
device stop rule.
"""
import numpy as np
import pytest

from oracle import metrics as OM
from oracle import qr as OQ
from oracle import solve as OSV
from workloads import dense_gaussian, dense_ill_conditioned

pytestmark = pytest.mark.gpu


def _dev(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _qr_gpu(sns, torch, SA, Sb):
    d, n = SA.shape
    ws = torch.empty(sns.sns_qr_solve_workspace_size(d, n), dtype=torch.uint8, device="cuda")
    x0 = torch.empty(n, dtype=torch.float64, device="cuda")
    R = torch.empty((n, n), dtype=torch.float64, device="cuda")
    info = sns.Info()
    sns.sns_qr_solve(d, n, _dev(SA, torch), _dev(Sb, torch), x0, R, ws, info)
    torch.cuda.synchronize()
    return x0.cpu().numpy(), R.cpu().numpy(), info


def _check_r_x0(R, Rr, x0, xr, tol=1e-12):
    """Element by element: every entry of column j of R within tol times the
    column's norm (Householder QR is backward stable column by column, and
    ||R[:, j]|| = ||SA[:, j]||), every entry of x0 within tol times max|x0|
    (times kappa(R) / 1e3 when R is worse conditioned than that); the
    strictly lower part of R is exactly zero."""
    cn = np.linalg.norm(Rr, axis=0)
    assert np.all(np.abs(R - Rr) <= tol * cn[None, :]), np.max(np.abs(R - Rr) / cn[None, :])
    assert np.all(np.tril(R, -1) == 0.0)
    amp = max(1.0, np.linalg.cond(Rr) / 1e3)
    assert np.max(np.abs(x0 - xr)) <= tol * amp * np.max(np.abs(xr)), np.max(np.abs(x0 - xr))
    assert np.linalg.norm(x0 - xr) <= tol * amp * np.linalg.norm(xr)


@pytest.mark.parametrize("d,n", [(200, 50), (1024, 256), (600, 600), (2100, 130), (80, 1),
                                 (513, 17), (4000, 97), (512, 16), (1025, 300), (4097, 40),
                                 (8192, 70), (257, 19), (4000, 1000), (8192, 600)])
def test_qr_solve_matches_oracle(gpu_lib, d, n):
    import torch
    rng = np.random.default_rng(d * 7 + n)
    SA = rng.standard_normal((d, n))
    Sb = rng.standard_normal(d)
    x0, R, info = _qr_gpu(gpu_lib, torch, SA, Sb)
    Rr, c, rho, _, _ = OQ.householder_qr_augmented(SA, Sb)
    xr = OQ.back_substitution(Rr, c)
    assert info.status == 0
    _check_r_x0(R, Rr, x0, xr)
    assert abs(info.sketch_resid - rho) <= 1e-12 * max(rho, 1.0)


def test_qr_solve_largest_shape(gpu_lib):
    """The largest QR the library takes, d = 8192 and n = 4096 (a trailing
    step then has 4097 column groups for 256 resident work-groups, so every
    work-group takes about 16 in turn).  The oracle's column loop is too slow
    at this size; the reference is LAPACK's Householder QR of [SA | Sb]
    (numpy), whose R the oracle's pins show equal to the oracle's entry by
    entry with the same sign convention.  R is compared element by element,
    x0 = R^{-1} c and rho = |R[n, n]| from the same factorisation."""
    import torch
    from scipy.linalg import solve_triangular
    d, n = 8192, 4096
    rng = np.random.default_rng(8192)
    SA = rng.standard_normal((d, n))
    Sb = rng.standard_normal(d)
    x0, R, info = _qr_gpu(gpu_lib, torch, SA, Sb)
    Ra = np.linalg.qr(np.column_stack([SA, Sb]), mode="r")
    Rr, c = Ra[:n, :n], Ra[:n, n]
    xr = solve_triangular(Rr, c)
    assert info.status == 0
    _check_r_x0(R, Rr, x0, xr)
    assert abs(info.sketch_resid - abs(Ra[n, n])) <= 1e-12 * abs(Ra[n, n])


def test_qr_solve_fp32_input_and_rank_deficiency(gpu_lib):
    import torch
    rng = np.random.default_rng(11)
    SA = rng.standard_normal((300, 40)).astype(np.float32)
    Sb = rng.standard_normal(300).astype(np.float32)
    x0, R, info = _qr_gpu(gpu_lib, torch, SA, Sb)
    Rr, c, rho, _, _ = OQ.householder_qr_augmented(SA.astype(np.float64), Sb.astype(np.float64))
    _check_r_x0(R, Rr, x0, OQ.back_substitution(Rr, c))
    SA = rng.standard_normal((300, 40))
    SA[:, 7] = SA[:, 3]
    _, _, info = _qr_gpu(gpu_lib, torch, SA, rng.standard_normal(300))
    assert info.status == 4  # SNS_ERR_RANK_DEFICIENT


def test_plain_fp64_20000x50(gpu_lib):
    """The plain FP64 sketch-and-solve workload at full size."""
    import torch
    sns = gpu_lib
    p = dense_gaussian(20000, 50, seed=1000)
    x, info = sns.lstsq(_dev(p.A, torch), _dev(p.b, torch), "count", 200, 42)
    r = OSV.sketch_and_solve(p.A, p.b, "count", 42, 200)
    xg = x.cpu().numpy()
    assert info.status == 0 and info.iters == 0
    assert np.max(np.abs(xg - r.x)) <= 1e-12 * np.max(np.abs(r.x))
    assert np.linalg.norm(xg - r.x) <= 1e-12 * np.linalg.norm(r.x)
    assert abs(info.sketch_resid - r.rho) <= 1e-12 * r.rho
    # accuracy of the method itself (reported, not a parity bar)
    xs = OM.lstsq_exact(p.A, p.b)
    fe = np.linalg.norm(xg - xs) / np.linalg.norm(xs)
    assert fe < 1e-3


def test_refine_fp64_fixed_iterations(gpu_lib):
    import torch
    sns = gpu_lib
    p = dense_ill_conditioned(30000, 40, seed=21, cond=1e3, dtype=np.float64)
    for k in (1, 3, 8):
        x, info = sns.lstsq(_dev(p.A, torch), _dev(p.b, torch), "count", 160, 42, refine=True,
                            max_iters=k, rtol=0.0)
        r = OSV.sap_sas(p.A, p.b, "count", 42, 160, k)
        assert info.iters == k
        xg = x.cpu().numpy()
        assert np.linalg.norm(xg - r.x) <= 1e-9 * np.linalg.norm(r.x), k


def test_refine_fp32_well_conditioned_fixed_iterations(gpu_lib):
    import torch
    sns = gpu_lib
    p = dense_gaussian(50000, 64, seed=22, dtype=np.float32)
    x, info = sns.lstsq(_dev(p.A, torch), _dev(p.b, torch), "count", 256, 42, refine=True,
                        max_iters=3, rtol=0.0)
    r = OSV.sap_sas(p.A, p.b, "count", 42, 256, 3)
    xg = x.cpu().numpy()
    assert info.iters == 3
    assert np.linalg.norm(xg - r.x) <= 1e-5 * np.linalg.norm(r.x)


@pytest.mark.parametrize("m,n,d", [(1 << 17, 64, 256), (200000, 100, 400)])
def test_refine_fp32_illconditioned_stop_rule(gpu_lib, m, n, d):
    import torch
    sns = gpu_lib
    p = dense_ill_conditioned(m, n, seed=23, cond=1e6)
    x, info = sns.lstsq(_dev(p.A, torch), _dev(p.b, torch), "count", d, 42, refine=True,
                        max_iters=100, rtol=1e-6)
    assert info.status == 0
    xs = OM.lstsq_exact(p.A, p.b)
    met = OM.metrics(p.A, p.b, x.cpu().numpy(), xs)
    assert met["RE"] <= 1e-6, met
    r = OSV.sap_sas(p.A, p.b, "count", 42, d, 100, rtol=1e-6)
    assert abs(info.iters - r.iters) <= 2
    assert info.rel_resid_est <= 1e-6


def test_refine_zero_iterations_returns_sketch_solution(gpu_lib):
    import torch
    sns = gpu_lib
    p = dense_gaussian(8000, 20, seed=24)
    x0, _ = sns.lstsq(_dev(p.A, torch), _dev(p.b, torch), "count", 80, 3)
    x1, info = sns.lstsq(_dev(p.A, torch), _dev(p.b, torch), "count", 80, 3, refine=True,
                         max_iters=0, rtol=0.0)
    assert info.iters == 0
    assert np.array_equal(x0.cpu().numpy(), x1.cpu().numpy())


def test_exact_recovery(gpu_lib):
    import torch
    sns = gpu_lib
    p = dense_gaussian(10000, 30, seed=25)
    b = p.A @ p.x_true
    x, info = sns.lstsq(_dev(p.A, torch), _dev(b, torch), "count", 120, 9)
    assert np.linalg.norm(x.cpu().numpy() - p.x_true) <= 1e-11 * np.linalg.norm(p.x_true)


def test_concurrent_solves_on_two_streams_from_one_thread(gpu_lib):
    """Two refined solves issued back to back on two streams from one host
    thread: the first returns with iterations possibly still in flight while
    the second polls the same ring of pinned host slots.  Each must give the
    answer of the same solve run alone."""
    import torch
    sns = gpu_lib
    probs = [dense_ill_conditioned(200000, 64, seed=61, cond=1e6),
             dense_ill_conditioned(150000, 48, seed=62, cond=1e6)]
    devs = [(_dev(p.A, torch), _dev(p.b, torch)) for p in probs]
    solo = [sns.lstsq(A, b, "count", 4 * A.shape[1], 7, refine=True, max_iters=100, rtol=1e-6)
            for A, b in devs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    torch.cuda.synchronize()
    for (A, b), st in zip(devs, streams):
        sk = sns.sketch_desc("count", 4 * A.shape[1], 7)
        M = sns.dense(A)
        o = sns.opts(1, 100, 1e-6)
        ws = torch.empty(sns.sns_lstsq_workspace_size(sk, M, o), dtype=torch.uint8, device="cuda")
        x = torch.empty(A.shape[1], dtype=torch.float64, device="cuda")
        buf = torch.zeros(64, dtype=torch.uint8).pin_memory()
        info = sns.Info.from_address(buf.data_ptr())
        outs.append((x, info, buf, ws))
        sns.sns_lstsq(sk, M, b, x, o, ws, info, st)
    torch.cuda.synchronize()
    for (x, info, _, _), (xs, info_s) in zip(outs, solo):
        assert info.status == 0 and info_s.status == 0
        assert info.iters == info_s.iters
        assert torch.equal(x, xs)


# ------------------------------------------------------- failure statuses --
# Numerical outcomes arrive in sns_info.status (SNS_ERR_NUMERICAL = 6,
# SNS_ERR_NOT_CONVERGED = 5); every kernel runs its fixed trip counts on
# non-finite data, so these cases end normally.

@pytest.mark.parametrize("refine", [False, True])
def test_nan_in_b_reports_numerical(gpu_lib, refine):
    import torch
    p = dense_gaussian(20000, 32, seed=41, dtype=np.float32)
    b = p.b.copy()
    b[1234] = np.nan
    x, info = gpu_lib.lstsq(_dev(p.A, torch), _dev(b, torch), "count", 128, 42, refine=refine,
                            max_iters=10, rtol=1e-6)
    assert info.status == 6, info.status


@pytest.mark.parametrize("refine", [False, True])
def test_inf_in_a_reports_numerical(gpu_lib, refine):
    import torch
    p = dense_gaussian(20000, 32, seed=42, dtype=np.float64)
    A = p.A.copy()
    A[777, 5] = np.inf
    x, info = gpu_lib.lstsq(_dev(A, torch), _dev(p.b, torch), "count", 128, 42, refine=refine,
                            max_iters=10, rtol=1e-6)
    assert info.status == 6, info.status


def test_max_iters_before_stop_rule_reports_not_converged(gpu_lib):
    """rtol = 1e-12 cannot be met in two iterations: status NOT_CONVERGED
    with the iterate after max_iters returned, the same bits as a run of
    exactly two iterations (rtol = 0), and within the FP64 fixed-iteration
    bar of the oracle's two-step SAP-SAS."""
    import torch
    p = dense_ill_conditioned(40000, 48, seed=43, cond=1e3, dtype=np.float64)
    A, b = _dev(p.A, torch), _dev(p.b, torch)
    x, info = gpu_lib.lstsq(A, b, "count", 192, 42, refine=True, max_iters=2, rtol=1e-12)
    assert info.status == 5 and info.iters == 2, (info.status, info.iters)
    x2, info2 = gpu_lib.lstsq(A, b, "count", 192, 42, refine=True, max_iters=2, rtol=0.0)
    assert info2.status == 0 and info2.iters == 2
    assert np.array_equal(x.cpu().numpy(), x2.cpu().numpy())
    r = OSV.sap_sas(p.A, p.b, "count", 42, 192, 2)
    assert np.linalg.norm(x.cpu().numpy() - r.x) <= 1e-9 * np.linalg.norm(r.x)
