"""GPU parity of the sparse sign embedding (the sparse sketch family of
Sec. 1.2.2 with zeta nonzeros per column of S) against the oracle.

The device sorts the zeta * m (row, hash) keys by bucket and reduces each
bucket with the CountSketch gather.  Bars: integer-valued inputs give
bit-exact SA and Sb; zeta = 1 is bit-identical to the CountSketch; random
inputs agree to a relative Frobenius error of 1e-5 (fp32) / 1e-12 (fp64) and
every entry lies within 128 u (sum_k |S_k|) |A| of the oracle; a solve with
the sparse sign embedding reaches RE <= 1e-6, and at d = 2n it needs no more
LSQR iterations than the CountSketch; a batch of one gives the solo answer
bit for bit.
"""
import numpy as np
import pytest

from oracle import metrics as OM
from oracle import sketch as OS
from workloads import dense_gaussian, dense_ill_conditioned

pytestmark = pytest.mark.gpu


def _dev(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


CASES = [
    # m, n, d, zeta, dtype
    (20000, 64, 256, 2, np.float32),
    (10007, 33, 130, 8, np.float64),
    (5000, 100, 400, 3, np.float32),
    (131072, 256, 1024, 4, np.float32),
    (3000, 300, 300, 16, np.float64),
    (777, 3, 5, 5, np.float32),
]


def _sketch(sns, torch, A, b, d, seed, zeta):
    SA, Sb = sns.sketch(_dev(A, torch), _dev(b, torch), "sparse", d, seed, zeta=zeta)
    torch.cuda.synchronize()
    return SA.cpu().numpy().astype(np.float64), Sb.cpu().numpy().astype(np.float64)


def _abs_bound(seed, d, m, zeta, M):
    out = np.zeros((d, M.shape[1]))
    for k in range(zeta):
        h, _ = OS.sparse_sign_hash(seed, d, 0, m, k)
        np.add.at(out, h.astype(np.int64), np.abs(M))
    return out


@pytest.mark.parametrize("m,n,d,zeta,dt", CASES)
def test_integer_inputs_bit_exact(gpu_lib, m, n, d, zeta, dt):
    import torch
    rng = np.random.default_rng(m + n + zeta)
    A = rng.integers(-8, 9, size=(m, n)).astype(dt)
    b = rng.integers(-8, 9, size=m).astype(dt)
    SA, Sb = _sketch(gpu_lib, torch, A, b, d, 42, zeta)
    SAr, Sbr = OS.sparse_sign_apply(A, b, 42, d, zeta)
    assert np.array_equal(SA, SAr)
    assert np.array_equal(Sb, Sbr)


@pytest.mark.parametrize("m,n,d,zeta,dt", CASES)
def test_random_inputs_within_tolerance(gpu_lib, m, n, d, zeta, dt):
    import torch
    rng = np.random.default_rng(7 * m + n + zeta)
    A = rng.standard_normal((m, n)).astype(dt)
    b = rng.standard_normal(m).astype(dt)
    SA, Sb = _sketch(gpu_lib, torch, A, b, d, 7, zeta)
    SAr, Sbr = OS.sparse_sign_apply(A, b, 7, d, zeta)
    full, ref = np.column_stack([SA, Sb]), np.column_stack([SAr, Sbr])
    tol = 1e-5 if dt == np.float32 else 1e-12
    assert np.linalg.norm(full - ref) <= tol * np.linalg.norm(ref)
    u = 2.0 ** -24 if dt == np.float32 else 2.0 ** -53
    bound = _abs_bound(7, d, m, zeta, np.column_stack([A, b]).astype(np.float64))
    assert np.all(np.abs(full - ref) <= 128 * u * bound + 1e-300)


def test_zeta_one_is_countsketch(gpu_lib):
    import torch
    rng = np.random.default_rng(3)
    A = rng.standard_normal((30000, 40)).astype(np.float32)
    b = rng.standard_normal(30000).astype(np.float32)
    Ad, bd = _dev(A, torch), _dev(b, torch)
    s1 = gpu_lib.sketch(Ad, bd, "sparse", 160, 11, zeta=1)
    s0 = gpu_lib.sketch(Ad, bd, "count", 160, 11)
    assert torch.equal(s1[0], s0[0]) and torch.equal(s1[1], s0[1])


def test_sparse_sign_solve_reaches_target_and_preconditions_better(gpu_lib):
    import torch
    p = dense_ill_conditioned(200000, 64, seed=41, cond=1e6)
    A, b = _dev(p.A, torch), _dev(p.b, torch)
    d = 128  # d = 2n: one nonzero per column embeds poorly
    xs = OM.lstsq_exact(p.A, p.b)
    x4, i4 = gpu_lib.lstsq(A, b, "sparse", d, 42, refine=True, max_iters=200, rtol=1e-6, zeta=4)
    x1, i1 = gpu_lib.lstsq(A, b, "count", d, 42, refine=True, max_iters=200, rtol=1e-6)
    assert i4.status == 0
    assert OM.metrics(p.A, p.b, x4.cpu().numpy(), xs)["RE"] <= 1e-6
    assert i4.iters <= i1.iters


def test_batch_of_one_equals_solo(gpu_lib):
    import torch
    sns = gpu_lib
    p = dense_gaussian(60000, 48, seed=43, dtype=np.float32)
    A, b = _dev(p.A, torch), _dev(p.b, torch)
    x, info = sns.lstsq(A, b, "sparse", 192, 5, refine=True, max_iters=50, rtol=1e-6, zeta=3)
    sk = sns.sketch_desc("sparse", 192, 5, 3)
    o = sns.opts(1, 50, 1e-6)
    xb = torch.empty(48, dtype=torch.float64, device="cuda")
    probs = [sns.problem(sk, sns.dense(A), b, xb, o)]
    nbytes = sns.sns_lstsq_batched_workspace_size(probs)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    infos = (sns.Info * 1)()
    sns.sns_lstsq_batched(probs, ws, infos, True)
    torch.cuda.synchronize()
    assert infos[0].iters == info.iters
    assert torch.equal(x, xb)
