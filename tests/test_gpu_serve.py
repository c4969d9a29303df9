"""GPU checks of the continuous-batching server.

Bars: a request's x and info are bit-identical whether it runs alone or in a
mix of requests that arrive while it runs, and equal to its solo sns_lstsq
call; admission never holds more workspace than the pool; every submitted
request completes (also when the server is destroyed right away); refined
FP32 results reach RE <= 1e-6 against the FP64 least-squares solution.
"""
import time

import numpy as np
import pytest

from oracle import metrics as OM
from workloads import dense_gaussian

pytestmark = pytest.mark.gpu

SHAPES = [(4096, 16), (60000, 64), (5000, 256), (25000, 32), (120000, 128), (8000, 16),
          (4500, 128), (90000, 256), (15000, 64), (6000, 32), (40000, 16), (7000, 64)]


def _dev(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _reqs(torch, shapes=SHAPES, seed0=40):
    out = []
    for k, (m, n) in enumerate(shapes):
        p = dense_gaussian(m, n, seed=seed0 + k, dtype=np.float32)
        out.append((p, _dev(p.A, torch), _dev(p.b, torch), 4 * n, 77 + k))
    return out


def _same(xa, ia, xb, ib):
    assert np.array_equal(xa.view(np.uint64), xb.view(np.uint64))
    assert (ia.status, ia.iters, ia.rel_resid_est, ia.sketch_resid) == \
        (ib.status, ib.iters, ib.rel_resid_est, ib.sketch_resid)


def test_alone_equals_in_mix_equals_solo(gpu_lib):
    import torch
    sns = gpu_lib
    reqs = _reqs(torch)
    torch.cuda.synchronize()
    srv = sns.Server(1 << 30, max_slots=8, chunk_iters=3)
    try:
        # request 1 alone
        p, A, b, d, seed = reqs[1]
        x_alone, i_alone = srv.wait(srv.submit(A, b, d, seed, max_iters=80))
        x_alone = x_alone.cpu().numpy()
        # the same request again, submitted in the middle of a stream of others
        tickets = []
        for k, (_, A2, b2, d2, s2) in enumerate(reqs):
            tickets.append((k, srv.submit(A2, b2, d2, s2, max_iters=80)))
            if k % 3 == 2:
                time.sleep(0.002)  # let rounds start while requests keep arriving
        got = {k: srv.wait(t) for k, t in tickets}
        st = srv.stats()
    finally:
        srv.close()
    x_mix, i_mix = got[1]
    _same(x_mix.cpu().numpy(), i_mix, x_alone, i_alone)
    assert st.completed == len(reqs) + 1 and st.peak_slots <= 8 and st.rounds >= 2
    for k, (p, A, b, d, seed) in enumerate(reqs):
        xs, infs = sns.lstsq(A, b, "count", d, seed, refine=True, max_iters=80, rtol=1e-6)
        x, info = got[k]
        _same(x.cpu().numpy(), info, xs.cpu().numpy(), infs)
        assert info.status == 0
        met = OM.metrics(p.A, p.b, x.cpu().numpy(), OM.lstsq_exact(p.A, p.b))
        assert met["RE"] <= 1e-6, (k, met)


def test_admission_bounded_by_pool(gpu_lib):
    import torch
    import paper_2409_14309_amd as P
    sns = gpu_lib
    reqs = _reqs(torch, shapes=[(60000, 128)] * 6, seed0=60)
    probe = P.problem(P.sketch_desc("count", 512, 1), P.dense(reqs[0][1]), reqs[0][2],
                      torch.empty(128, dtype=torch.float64, device="cuda"), P.opts(1, 80, 1e-6))
    one = P.sns_lstsq_workspace_size(probe.sketch, probe.A, probe.opts)
    # the pool holds the server's tables and about two request workspaces
    srv = sns.Server(int(2.5 * one) + (3 * (4 * 4096 + 16384) + 8 * 4 + 4096), max_slots=4)
    try:
        ts = [srv.submit(A, b, d, s, max_iters=80) for _, A, b, d, s in reqs]
        res = [srv.wait(t) for t in ts]
        st = srv.stats()
    finally:
        srv.close()
    assert st.peak_slots <= 2 and st.completed == 6
    for (p, A, b, d, s), (x, info) in zip(reqs, res):
        xs, infs = sns.lstsq(A, b, "count", d, s, refine=True, max_iters=80, rtol=1e-6)
        _same(x.cpu().numpy(), info, xs.cpu().numpy(), infs)


def test_plain_requests_and_destroy_drains(gpu_lib):
    import torch
    sns = gpu_lib
    reqs = _reqs(torch, shapes=SHAPES[:6], seed0=80)
    srv = sns.Server(1 << 30, max_slots=3, chunk_iters=2)
    xs = []
    for k, (_, A, b, d, s) in enumerate(reqs):
        x = torch.full((A.shape[1],), float("nan"), dtype=torch.float64, device="cuda")
        srv.submit(A, b, d, s, refine=(k % 2 == 0), max_iters=60, x=x)
        xs.append(x)
    srv.close()  # completes everything that was submitted
    torch.cuda.synchronize()
    for k, (_, A, b, d, s) in enumerate(reqs):
        ref, _ = sns.lstsq(A, b, "count", d, s, refine=(k % 2 == 0), max_iters=60, rtol=1e-6)
        assert np.array_equal(xs[k].cpu().numpy(), ref.cpu().numpy())


def test_submit_errors(gpu_lib):
    import torch
    sns = gpu_lib
    srv = sns.Server(1 << 22, max_slots=1, queue_capacity=1)
    try:
        p = dense_gaussian(5000, 16, seed=3, dtype=np.float64)
        with pytest.raises(sns.SnsError):  # server is fp32
            srv.submit(_dev(p.A, torch), _dev(p.b, torch), 64, 1)
        with pytest.raises(sns.SnsError):  # unknown ticket
            sns.sns_serve_poll(srv.handle, 123456)
        big = dense_gaussian(400000, 64, seed=4, dtype=np.float32)
        with pytest.raises(sns.SnsError):  # workspace larger than the pool
            srv.submit(_dev(big.A, torch), _dev(big.b, torch), 256, 1)
    finally:
        srv.close()
