"""GPU checks of the autotuner: the tuner returns a valid plan with a
measured time; a solve under a tuned plan still matches the oracle (the plan
only regroups partial sums), and batched solves stay bit-identical to solo
ones under it."""
import numpy as np
import pytest

from oracle import solve as OSV
from workloads import dense_gaussian

pytestmark = pytest.mark.gpu


def test_tune_pass_and_tuned_solve(gpu_lib):
    import torch
    sns = gpu_lib
    p = dense_gaussian(60000, 64, seed=12, dtype=np.float64)
    A = torch.from_numpy(p.A).cuda()
    b = torch.from_numpy(p.b).cuda()
    M = sns.dense(A)
    ws = torch.empty(sns.sns_tune_workspace_size(M), dtype=torch.uint8, device="cuda")
    e = sns.sns_tune_pass(M, 3, ws)
    assert e.us > 0 and e.lpr * e.nch * 2 >= 64 and 64 <= e.grid <= 4096 and e.unroll in (1, 2)
    assert e.waves in (4, 8)
    assert e.m_lo == e.m_hi == 60000 and e.n == 64 and e.dtype == sns.SNS_F64
    # force an unusual plan for this shape (8-wave work-groups), then solve
    forced = sns.TuneEntry(sns.SNS_F64, 64, 50000, 70000, 64, 1, 96, 2, 0.0, 8)
    sns.sns_tune_set(forced)
    try:
        x, info = sns.lstsq(A, b, "count", 256, 5, refine=True, max_iters=8, rtol=0.0)
        r = OSV.sap_sas(p.A, p.b, "count", 5, 256, 8, rtol=0.0)
        assert info.iters == 8
        assert np.linalg.norm(x.cpu().numpy() - r.x) <= 1e-9 * np.linalg.norm(r.x)
        xs, infos = sns.lstsq_batched([A, A[:30000]], [b, b[:30000]], [256, 128], [5, 6],
                                      max_iters=8, rtol=0.0)
        x2, _ = sns.lstsq(A[:30000], b[:30000], "count", 128, 6, refine=True, max_iters=8, rtol=0.0)
        assert np.array_equal(xs[0].cpu().numpy(), x.cpu().numpy())
        assert np.array_equal(xs[1].cpu().numpy(), x2.cpu().numpy())
    finally:
        sns.sns_tune_clear()
        import os
        if os.path.exists(sns._binding.TUNING_PATH):
            sns.sns_tune_load(sns._binding.TUNING_PATH)


def _restore_table(sns):
    import os
    sns.sns_tune_clear()
    if os.path.exists(sns._binding.TUNING_PATH):
        sns.sns_tune_load(sns._binding.TUNING_PATH)


def _pow2(v, lo, hi):
    return lo <= v <= hi and v & (v - 1) == 0


def test_tune_gather_and_forced_gather_shapes(gpu_lib):
    """The gather tuner returns a valid (lanes per row, segments) pair with a
    measured time.  Every forced shape gives an SA equal to the oracle's bit
    for bit on integer-valued data (every partial sum is exact, so any order
    agrees) and to 1e-5 relative on N(0,1) data; a solve under a forced shape
    matches the oracle's sketch-and-solve."""
    import torch
    from oracle import sketch as OS
    sns = gpu_lib
    m, n, d, seed = 200003, 50, 200, 7
    rng = np.random.default_rng(31)
    Ai = rng.integers(-3, 4, size=(m, n)).astype(np.float32)
    bi = rng.integers(-3, 4, size=m).astype(np.float32)
    Ag = torch.from_numpy(Ai).cuda()
    bg = torch.from_numpy(bi).cuda()
    M = sns.dense(Ag)
    ws = torch.empty(sns.sns_tune_gather_workspace_size(M, d), dtype=torch.uint8, device="cuda")
    e = sns.sns_tune_gather(M, bg, d, seed, 3, ws)
    assert e.us > 0 and _pow2(e.lpr, 4, 64) and _pow2(e.nseg, 1, 64)
    assert e.nseg == 1 or e.nseg * d * 256 <= m
    assert (e.dtype, e.n, e.d, e.m_lo, e.m_hi) == (sns.SNS_F32, n, d, m, m)
    SAr, Sbr = OS.countsketch_apply(Ai.astype(np.float64), bi.astype(np.float64), seed, d)
    p = dense_gaussian(m, n, seed=32, dtype=np.float32)
    Ad, bd = torch.from_numpy(p.A).cuda(), torch.from_numpy(p.b).cuda()
    SAg, Sbg = OS.countsketch_apply(p.A.astype(np.float64), p.b.astype(np.float64), seed, d)
    try:
        for lpr, nseg in [(4, 1), (4, 16), (8, 2), (16, 64), (64, 4)]:
            sns.sns_tune_gather_set(sns.TuneGatherEntry(sns.SNS_F32, n, d, m, m, lpr, nseg, 0.0))
            SA, Sb = sns.sketch(Ag, bg, "count", d, seed)
            torch.cuda.synchronize()
            assert np.array_equal(SA.cpu().numpy(), SAr.astype(np.float32)), (lpr, nseg)
            assert np.array_equal(Sb.cpu().numpy(), Sbr.astype(np.float32)), (lpr, nseg)
            SA, Sb = sns.sketch(Ad, bd, "count", d, seed)
            err = np.linalg.norm(SA.cpu().numpy().astype(np.float64) - SAg) / np.linalg.norm(SAg)
            assert err <= 1e-5, (lpr, nseg, err)
        x, info = sns.lstsq(Ad, bd, "count", d, seed)
        r = OSV.sketch_and_solve(p.A.astype(np.float64), p.b.astype(np.float64), "count", seed, d)
        assert info.status == 0
        assert np.linalg.norm(x.cpu().numpy() - r.x0) <= 1e-4 * np.linalg.norm(r.x0)
    finally:
        _restore_table(sns)


@pytest.mark.parametrize("d,n", [(200, 50), (700, 100), (1500, 375)])
def test_tune_qr_and_forced_panel_shapes(gpu_lib, d, n):
    """The QR tuner returns a configuration that holds d; under every forced
    configuration and trailing width the QR solve matches the oracle's
    Householder QR (R column by column and x0 to 1e-12)."""
    import torch
    from oracle import qr as OQ
    sns = gpu_lib
    rng = np.random.default_rng(d + n)
    SA = rng.standard_normal((d, n))
    Sb = rng.standard_normal(d)
    SAd, Sbd = torch.from_numpy(SA).cuda(), torch.from_numpy(Sb).cuda()
    ws = torch.empty(sns.sns_tune_qr_workspace_size(d, n), dtype=torch.uint8, device="cuda")
    e = sns.sns_tune_qr(SAd, Sbd, 3, ws)
    cap = {0: 512, 1: 1024, 2: 2048, 3: 4096, 4: 8192}
    assert e.us > 0 and cap[e.cfg] >= d and e.cb in (1, 2)
    assert (e.d_lo, e.d_hi, e.n_lo, e.n_hi) == (d, d, n, n)
    Rr, c, rho, _, _ = OQ.householder_qr_augmented(SA, Sb)
    xr = OQ.back_substitution(Rr, c)
    cn = np.linalg.norm(Rr, axis=0)
    qws = torch.empty(sns.sns_qr_solve_workspace_size(d, n), dtype=torch.uint8, device="cuda")
    try:
        for cfg in [k for k in cap if cap[k] >= d]:
            for cb in (1, 2):
                sns.sns_tune_qr_set(sns.TuneQrEntry(d, d, n, n, cfg, cb, 0.0))
                x0 = torch.empty(n, dtype=torch.float64, device="cuda")
                R = torch.empty((n, n), dtype=torch.float64, device="cuda")
                info = sns.Info()
                sns.sns_qr_solve(d, n, SAd, Sbd, x0, R, qws, info)
                torch.cuda.synchronize()
                Rg, xg = R.cpu().numpy(), x0.cpu().numpy()
                assert info.status == 0
                assert np.all(np.abs(Rg - Rr) <= 1e-12 * cn[None, :]), (cfg, cb)
                assert np.max(np.abs(xg - xr)) <= 1e-12 * np.max(np.abs(xr)), (cfg, cb)
                assert abs(info.sketch_resid - rho) <= 1e-12 * max(rho, 1.0)
    finally:
        _restore_table(sns)
