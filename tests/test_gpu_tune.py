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
    assert e.m_lo == e.m_hi == 60000 and e.n == 64 and e.dtype == sns.SNS_F64
    # force an unusual plan for this shape, then solve
    forced = sns.TuneEntry(sns.SNS_F64, 64, 50000, 70000, 64, 1, 96, 2, 0.0)
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
