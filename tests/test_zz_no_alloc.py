"""The allocation-free QR solve (workspace in the library's static device
array) gives the same bits as sns_qr_solve with a caller workspace, on two
calls in a row (the second smaller, so it runs over what the first left in
the array), for FP64 and FP32 input."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _solve_both(sns, torch, SA, Sb):
    d, n = SA.shape
    A = torch.from_numpy(np.ascontiguousarray(SA)).cuda()
    b = torch.from_numpy(np.ascontiguousarray(Sb)).cuda()
    ws = torch.empty(sns.sns_qr_solve_workspace_size(d, n), dtype=torch.uint8, device="cuda")
    out = []
    for noalloc in (False, True):
        x0 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        R = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
        info = sns.Info()
        torch.cuda.synchronize()
        if noalloc:
            sns.sns_qr_solve_noalloc(d, n, A, b, x0, R, info)
        else:
            sns.sns_qr_solve(d, n, A, b, x0, R, ws, info)
        torch.cuda.synchronize()
        out.append((x0.cpu().numpy(), R.cpu().numpy(), info.status, info.sketch_resid))
    return out


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_noalloc_qr_matches_workspace_qr_twice(gpu_lib, dt):
    import torch
    rng = np.random.default_rng(5)
    for d, n in ((2048, 513), (300, 37)):
        SA = rng.standard_normal((d, n)).astype(dt)
        Sb = rng.standard_normal(d).astype(dt)
        (x_ws, R_ws, st_ws, rho_ws), (x_na, R_na, st_na, rho_na) = _solve_both(gpu_lib, torch, SA, Sb)
        assert st_ws == 0 and st_na == 0
        assert np.array_equal(x_ws, x_na), (d, n)
        assert np.array_equal(R_ws, R_na), (d, n)
        assert rho_ws == rho_na


def test_noalloc_rejects_oversize(gpu_lib):
    import torch
    fake = torch.zeros(8, dtype=torch.float64, device="cuda")
    st = gpu_lib.load().sns_qr_solve_noalloc(8192, 1000, 1, fake.data_ptr(), 1000, fake.data_ptr(),
                                             fake.data_ptr(), None, None, None)
    assert st == 7  # SNS_ERR_OUT_OF_MEMORY, nothing enqueued
