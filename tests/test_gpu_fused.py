"""GPU parity of the persistent fused sketch + QR launch: every CountSketch
problem with d <= 256, n <= 64 and m (n + 1) <= 2^21 (dense) has its sketch
(Sec. 1.2 steps 1-2) and its Householder QR and x0 (step 3) computed there,
in every entry point (single solve, batch, server), once sns_fused_enable(1)
has switched it on (the default is the blocked path).

Bars: FP64 x0 agrees with the oracle's sketch-and-solve entry by entry to
1e-12 (times kappa(SA) / 1e3 when that is larger), and the sketched
residual rho to 1e-12 ||Sb||; FP32 inputs (summed in FP64 by the kernel) agree to 1e-10 with
the oracle run on the same FP32 values; the shapes cover one chunk, several
4096-row sub-blocks, chunk counts that need the two-level sum, ragged m,
m = d, n = 1 and d = n.  Which launch ran is read from the library's kernel
timing hooks.  A batch of uneven problems gives the same bits as the solo
calls; rank deficiency and a NaN in b are reported as on the blocked path.
"""
import numpy as np
import pytest

from oracle import solve as OSV
from workloads import dense_gaussian

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def fused_on(gpu_lib):
    """The fused form is off by default: every test here switches it on and
    restores the default afterwards."""
    gpu_lib.sns_fused_enable(True)
    yield
    gpu_lib.sns_fused_enable(False)

SHAPES = [  # m, n, d
    (4096, 16, 64),      # one chunk, one sub-block
    (3001, 50, 200),     # ragged single sub-block
    (20000, 50, 200),    # the 20000 x 50 workload: one chunk of 5 sub-blocks
    (30001, 64, 256),    # the widest system held in LDS
    (600007, 2, 8),      # 74 chunks of 8192 rows: group sums and the top sum
    (256, 64, 256),      # m = d
    (5000, 1, 4),        # one column
    (40000, 8, 8),       # d = n
]


def _dev(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _ran_fused(sns, fn):
    sns.sns_timing_reset()
    sns.sns_timing_select(["fused_sq", "qr_panel", "cs_gather"])
    sns.sns_timing_enable(True)
    try:
        out = fn()
    finally:
        sns.sns_timing_enable(False)
        sns.sns_timing_select(None)
    kt = sns.sns_timing_summary()
    return out, kt


def _check_x0(xg, r, SA, tol):
    amp = max(1.0, np.linalg.cond(SA) / 1e3)
    assert np.max(np.abs(xg - r.x0)) <= tol * amp * np.max(np.abs(r.x0)), np.max(np.abs(xg - r.x0))


@pytest.mark.parametrize("m,n,d", SHAPES)
def test_fused_plain_solve_matches_oracle_fp64(gpu_lib, m, n, d):
    import torch
    sns = gpu_lib
    p = dense_gaussian(m, n, seed=m + n + d)
    A, b = _dev(p.A, torch), _dev(p.b, torch)
    (x, info), kt = _ran_fused(sns, lambda: sns.lstsq(A, b, "count", d, 77))
    assert "fused_sq" in kt and "qr_panel" not in kt and "cs_gather" not in kt, kt
    r = OSV.sketch_and_solve(p.A, p.b, "count", 77, d)
    SA, Sb = OSV.sketch(p.A, p.b, "count", 77, d)
    assert info.status == 0 and info.iters == 0
    _check_x0(x.cpu().numpy(), r, SA, 1e-12)
    # rho is the norm of a residual (far below ||Sb|| when the fit is good):
    # its rounding error scales with ||Sb||, the size of what was subtracted
    assert abs(info.sketch_resid - r.rho) <= 1e-12 * np.linalg.norm(Sb)


@pytest.mark.parametrize("m,n,d", [(20000, 50, 200), (30001, 64, 256), (600007, 2, 8)])
def test_fused_plain_solve_matches_oracle_fp32(gpu_lib, m, n, d):
    import torch
    sns = gpu_lib
    p = dense_gaussian(m, n, seed=3 * m + n, dtype=np.float32)
    A, b = _dev(p.A, torch), _dev(p.b, torch)
    (x, info), kt = _ran_fused(sns, lambda: sns.lstsq(A, b, "count", d, 5))
    assert "fused_sq" in kt
    A64, b64 = p.A.astype(np.float64), p.b.astype(np.float64)
    r = OSV.sketch_and_solve(A64, b64, "count", 5, d)
    SA, _ = OSV.sketch(A64, b64, "count", 5, d)
    assert info.status == 0
    _check_x0(x.cpu().numpy(), r, SA, 1e-10)


@pytest.mark.parametrize("m,n,d", [(20000, 65, 260), (40000, 64, 256)])
def test_fused_larger_problems_keep_the_blocked_path(gpu_lib, m, n, d):
    """n > 64, or m (n + 1) > 2^21: the blocked path."""
    import torch
    sns = gpu_lib
    p = dense_gaussian(m, n, seed=9)
    A, b = _dev(p.A, torch), _dev(p.b, torch)
    (_, info), kt = _ran_fused(sns, lambda: sns.lstsq(A, b, "count", d, 1))
    assert "fused_sq" not in kt and "qr_panel" in kt
    assert info.status == 0


def test_fused_batch_bitwise_equals_solo_and_refines(gpu_lib):
    """Uneven problems (some fused, some on the blocked path) in one batch:
    x and info equal their solo calls bit for bit, refined to the stop rule."""
    import torch
    sns = gpu_lib
    shapes = [(4096, 16), (150001, 64), (9000, 8), (30000, 32), (5000, 128), (70000, 64)]
    probs = []
    for k, (m, n) in enumerate(shapes):
        p = dense_gaussian(m, n, seed=900 + k, dtype=np.float32)
        probs.append((p, _dev(p.A, torch), _dev(p.b, torch), 4 * n, 300 + k))
    solo = [sns.lstsq(A, b, "count", d, s, refine=True, max_iters=60, rtol=1e-6)
            for _, A, b, d, s in probs]
    xs, infos = sns.lstsq_batched([q[1] for q in probs], [q[2] for q in probs],
                                  [q[3] for q in probs], [q[4] for q in probs], refine=True,
                                  max_iters=60, rtol=1e-6, use_graph=False)
    for (xs_, is_), xb, ib in zip(solo, xs, infos):
        assert np.array_equal(xs_.cpu().numpy().view(np.uint64), xb.cpu().numpy().view(np.uint64))
        assert (is_.status, is_.iters, is_.sketch_resid) == (ib.status, ib.iters, ib.sketch_resid)
        assert ib.status == 0


def test_fused_statuses(gpu_lib):
    import torch
    sns = gpu_lib
    rng = np.random.default_rng(4)
    A = rng.standard_normal((5000, 20))
    A[:, 7] = A[:, 3]
    b = rng.standard_normal(5000)
    _, info = sns.lstsq(_dev(A, torch), _dev(b, torch), "count", 80, 3)
    assert info.status == 4  # SNS_ERR_RANK_DEFICIENT
    A = rng.standard_normal((5000, 20))
    b[17] = np.nan
    _, info = sns.lstsq(_dev(A, torch), _dev(b, torch), "count", 80, 3)
    assert info.status == 6  # SNS_ERR_NUMERICAL


def test_server_graph_replays_equal_solo(gpu_lib):
    """The server sets up its small requests by replaying a captured graph of
    the fused launch with each round's problem table.  Many rounds of small
    requests (two slots, so the two graphs alternate many times), submitted
    while the host keeps other device work and synchronisations going: every
    result equals its solo call bit for bit, plain and refined."""
    import time

    import torch
    sns = gpu_lib
    shapes = [(4096 + 997 * k, (8, 16, 32, 64)[k % 4]) for k in range(14)]
    reqs = []
    for k, (m, n) in enumerate(shapes):
        p = dense_gaussian(m, n, seed=700 + k, dtype=np.float32)
        reqs.append((_dev(p.A, torch), _dev(p.b, torch), 4 * n, 40 + k, k % 3 == 0))
    torch.cuda.synchronize()
    srv = sns.Server(1 << 29, max_slots=2, chunk_iters=2)
    try:
        tickets = []
        scratch = torch.zeros(1 << 20, device="cuda")
        for k, (A, b, d, seed, plain) in enumerate(reqs):
            if plain:
                tickets.append(srv.submit(A, b, d, seed, refine=False))
            else:
                tickets.append(srv.submit(A, b, d, seed, max_iters=60))
            scratch.add_(1.0)  # the caller's own eager work between submissions
            if k % 4 == 3:
                torch.cuda.synchronize()
                time.sleep(0.001)
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    assert st.rounds >= 7
    for (A, b, d, seed, plain), (x, info) in zip(reqs, got):
        if plain:
            xs, infs = sns.lstsq(A, b, "count", d, seed)
        else:
            xs, infs = sns.lstsq(A, b, "count", d, seed, refine=True, max_iters=60, rtol=1e-6)
        assert np.array_equal(x.cpu().numpy().view(np.uint64), xs.cpu().numpy().view(np.uint64))
        assert (info.status, info.iters, info.sketch_resid) == (infs.status, infs.iters,
                                                                infs.sketch_resid)
        assert info.status == 0
