"""GPU checks of the batched solve (many uneven problems per launch).

Bars: every problem of a batch gives x and info bit-identical to its solo
sns_lstsq call (the batch runs the same per-problem arithmetic), with and
without the HIP graph for the refinement chunks, on repeated replays with
other device work in between; FP32 refined results reach RE <= 1e-6 against
the FP64 least-squares solution; FP64 batches with a fixed iteration count
agree with the oracle's SAP-SAS to 1e-9.
"""
import numpy as np
import pytest

from oracle import metrics as OM
from oracle import solve as OSV
from workloads import dense_gaussian

pytestmark = pytest.mark.gpu

MIX = [  # m, n (d = 4 n), the serving mix's shapes at test sizes
    (4096, 16), (70000, 64), (5000, 256), (30000, 32), (150000, 128), (9000, 16),
    (4500, 128), (120000, 256), (20000, 64), (6000, 32),
]


def _dev(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _problems(torch, dt=np.float32, mix=MIX, seed0=500):
    out = []
    for k, (m, n) in enumerate(mix):
        p = dense_gaussian(m, n, seed=seed0 + k, dtype=dt)
        out.append((p, _dev(p.A, torch), _dev(p.b, torch), 4 * n, 1000 + k))
    return out


def _solo(sns, probs, refine, max_iters, rtol):
    res = []
    for p, A, b, d, seed in probs:
        x, info = sns.lstsq(A, b, "count", d, seed, refine=refine, max_iters=max_iters, rtol=rtol)
        res.append((x.cpu().numpy(), info))
    return res


def _batch(sns, probs, refine, max_iters, rtol, use_graph):
    xs, infos = sns.lstsq_batched([q[1] for q in probs], [q[2] for q in probs],
                                  [q[3] for q in probs], [q[4] for q in probs], refine=refine,
                                  max_iters=max_iters, rtol=rtol, use_graph=use_graph)
    return [(x.cpu().numpy(), i) for x, i in zip(xs, infos)]


def _same(a, b):
    for (xa, ia), (xb, ib) in zip(a, b):
        assert np.array_equal(xa.view(np.uint64), xb.view(np.uint64))
        assert (ia.status, ia.iters) == (ib.status, ib.iters)
        assert ia.rel_resid_est == ib.rel_resid_est and ia.sketch_resid == ib.sketch_resid


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_equals_solo_fp32_refined(gpu_lib, use_graph):
    import torch
    sns = gpu_lib
    probs = _problems(torch)
    solo = _solo(sns, probs, True, 80, 1e-6)
    _same(_batch(sns, probs, True, 80, 1e-6, use_graph), solo)
    for (p, *_), (x, info) in zip(probs, solo):
        assert info.status == 0
        met = OM.metrics(p.A, p.b, x, OM.lstsq_exact(p.A, p.b))
        assert met["RE"] <= 1e-6, met


def test_graph_replays_with_eager_work_between(gpu_lib):
    import torch
    sns = gpu_lib
    probs = _problems(torch, mix=MIX[:6], seed0=900)
    solo = _solo(sns, probs, True, 60, 1e-6)
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        junk = junk * 1.0001 + float(rep)  # unrelated eager work on the same stream
        torch.cuda.synchronize()
        _same(_batch(sns, probs, True, 60, 1e-6, True), solo)


def test_batch_mixed_plain_and_refined(gpu_lib):
    import torch
    sns = gpu_lib
    probs = _problems(torch, mix=MIX[:5], seed0=700)
    plain = _solo(sns, probs, False, 0, 0.0)
    refined = _solo(sns, probs, True, 50, 1e-6)
    import paper_2409_14309_amd as P
    xs, pr = [], []
    for k, (p, A, b, d, seed) in enumerate(probs):
        x = torch.empty(A.shape[1], dtype=torch.float64, device="cuda")
        ref = k % 2 == 1
        o = P.opts(int(ref), 50 if ref else 0, 1e-6 if ref else 0.0)
        pr.append(P.problem(P.sketch_desc("count", d, seed), P.dense(A), b, x, o))
        xs.append(x)
    ws = torch.empty(P.sns_lstsq_batched_workspace_size(pr), dtype=torch.uint8, device="cuda")
    infos = (P.Info * len(pr))()
    P.sns_lstsq_batched(pr, ws, infos, True)
    torch.cuda.synchronize()
    for k in range(len(probs)):
        want = refined[k] if k % 2 == 1 else plain[k]
        _same([(xs[k].cpu().numpy(), infos[k])], [want])


def test_batch_fp64_fixed_iterations_matches_oracle(gpu_lib):
    import torch
    sns = gpu_lib
    mix = [(3000, 16), (12000, 48), (5000, 100), (20000, 8)]
    probs = _problems(torch, dt=np.float64, mix=mix, seed0=300)
    got = _batch(sns, probs, True, 6, 0.0, True)
    _same(got, _solo(sns, probs, True, 6, 0.0))
    for (p, A, b, d, seed), (x, info) in zip(probs, got):
        r = OSV.sap_sas(p.A, p.b, "count", seed, d, 6, rtol=0.0)
        assert info.iters == 6
        assert np.linalg.norm(x - r.x) <= 1e-9 * np.linalg.norm(r.x)


def test_batch_rejects_mixed_dtypes(gpu_lib):
    import torch
    sns = gpu_lib
    a = dense_gaussian(5000, 16, seed=1, dtype=np.float32)
    b = dense_gaussian(5000, 16, seed=2, dtype=np.float64)
    with pytest.raises(sns.SnsError):
        sns.lstsq_batched([_dev(a.A, torch), _dev(b.A, torch)], [_dev(a.b, torch), _dev(b.b, torch)],
                          [64, 64], [1, 2])


def test_batch_straddles_fused_step_limit(gpu_lib):
    """Problems with n <= 256 run the LSQR step inside the reduction kernel,
    larger ones in the separate step kernels; one batch holding both kinds
    (and widths near 512) matches the solo calls bit for bit, and FP64
    results with a fixed iteration count agree with the oracle's SAP-SAS on
    both sides of the limit."""
    import torch
    sns = gpu_lib
    mix = [(6000, 256), (6500, 258), (5000, 254), (7000, 300), (4000, 16),  # rows of 16 bytes
           (8000, 510), (8000, 512), (8500, 514)]
    probs = _problems(torch, dt=np.float64, mix=mix, seed0=1300)
    got = _batch(sns, probs, True, 6, 0.0, True)
    _same(got, _solo(sns, probs, True, 6, 0.0))
    for (p, A, b, d, seed), (x, info) in zip(probs, got):
        r = OSV.sap_sas(p.A, p.b, "count", seed, d, 6, rtol=0.0)
        assert info.iters == 6
        assert np.linalg.norm(x - r.x) <= 1e-9 * np.linalg.norm(r.x)
    probs32 = _problems(torch, mix=[(40000, 256), (40000, 260), (20000, 64), (60000, 512),
                                    (60000, 516)], seed0=1400)
    solo = _solo(sns, probs32, True, 80, 1e-6)
    _same(_batch(sns, probs32, True, 80, 1e-6, True), solo)
    for (p, *_), (x, info) in zip(probs32, solo):
        assert info.status == 0
        assert OM.metrics(p.A, p.b, x, OM.lstsq_exact(p.A, p.b))["RE"] <= 1e-6
