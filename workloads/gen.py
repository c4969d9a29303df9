"""Generators for the five least-squares workloads and the paper's own
benchmark family.

Every generator takes an explicit seed and draws from numpy's default_rng, so
each input is reproducible.  Values are drawn in float64 and rounded once to
the stored dtype; the stored values *are* the problem (the oracle widens them
back to float64).

Workloads (sizes are the defaults; tests pass smaller ones):
  plain FP64 sketch-and-solve   dense_gaussian(20000, 50, float64), d = 200
  ill-conditioned FP32          dense_ill_conditioned(4194304, 256), d = 1024
  sparse CSR FP32               sparse_csr(2**24, 1000), d = 4000
  Gaussian sketch on MFMA       dense_scaled_columns(262144, 512), d = 2048
  serving mix                   serving_requests(10000, 2000.0) + dense_gaussian per request
  paper benchmark (Sec. 3.1)    paper_benchmark(m, 1000, cond 1e10, beta 1e-10)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

DATA_SEED_BASE = 1000
SKETCH_SEED = 42


@dataclass
class Dense:
    A: np.ndarray
    b: np.ndarray
    x_true: np.ndarray
    meta: dict = field(default_factory=dict)


@dataclass
class Sparse:
    A: sp.csr_matrix
    b: np.ndarray
    x_true: np.ndarray
    meta: dict = field(default_factory=dict)


def dense_gaussian(m: int, n: int, seed: int, noise: float = 1e-3, dtype=np.float64) -> Dense:
    """A_ij ~ N(0,1), x_true ~ N(0, I), b = A x_true + noise * N(0, I)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)).astype(dtype)
    x = rng.standard_normal(n)
    b = (A.astype(np.float64) @ x + noise * rng.standard_normal(m)).astype(dtype)
    return Dense(A, b, x, {"kind": "dense_gaussian", "m": m, "n": n, "seed": seed, "noise": noise})


def random_orthogonal(n: int, rng) -> np.ndarray:
    """Q factor of an n x n Gaussian matrix with the signs fixed so diag(R) > 0."""
    Q, R = np.linalg.qr(rng.standard_normal((n, n)))
    return Q * np.sign(np.diag(R))


def _block_rngs(seed: int, nblocks: int):
    """Independent generators for row blocks (numpy SeedSequence.spawn)."""
    return [np.random.default_rng(c) for c in np.random.SeedSequence(seed).spawn(nblocks)]


def _parallel(fn, items, workers: int = 0):
    import os
    from concurrent.futures import ThreadPoolExecutor
    workers = workers or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(fn, items))


def dense_ill_conditioned(m: int, n: int, seed: int, cond: float = 1e6, rel_noise: float = 1e-4,
                          dtype=np.float32, block: int = 1 << 16) -> Dense:
    """A = G diag(sigma) V^T with G Gaussian, sigma log-spaced 1 .. 1/cond, V orthogonal.

    b = A x_true + rel_noise * (||A x_true|| / ||z||) z with z ~ N(0, I_m).
    A is built in float64 row blocks (each block with its own spawned
    generator, so blocks can be drawn in parallel) and rounded to dtype; b is
    computed from the rounded A.
    """
    nblk = (m + block - 1) // block
    rngs = _block_rngs(seed, nblk + 1)
    head = rngs[nblk]
    sigma = np.logspace(0.0, -np.log10(cond), n)
    V = random_orthogonal(n, head)
    W = (sigma[:, None] * V.T)  # diag(sigma) V^T
    x = head.standard_normal(n)
    A = np.empty((m, n), dtype=dtype)
    b0 = np.empty(m)
    z = np.empty(m)

    def fill(k):
        r0, r1 = k * block, min(m, (k + 1) * block)
        G = rngs[k].standard_normal((r1 - r0, n))
        A[r0:r1] = (G @ W).astype(dtype)
        b0[r0:r1] = A[r0:r1].astype(np.float64) @ x
        z[r0:r1] = rngs[k].standard_normal(r1 - r0)

    _parallel(fill, range(nblk))
    b = (b0 + rel_noise * (np.linalg.norm(b0) / np.linalg.norm(z)) * z).astype(dtype)
    return Dense(A, b, x, {"kind": "dense_ill_conditioned", "m": m, "n": n, "seed": seed,
                           "cond": cond, "rel_noise": rel_noise})


def dense_scaled_columns(m: int, n: int, seed: int, decades: float = 3.0, noise: float = 1e-3,
                         dtype=np.float32) -> Dense:
    """A_ij ~ N(0,1) * 10^(-decades * j / (n-1)), b = A x_true + noise * N(0, I)."""
    rng = np.random.default_rng(seed)
    scale = 10.0 ** (-decades * np.arange(n) / max(n - 1, 1))
    A = np.empty((m, n), dtype=dtype)
    blk = 1 << 16
    for r0 in range(0, m, blk):
        r1 = min(m, r0 + blk)
        A[r0:r1] = (rng.standard_normal((r1 - r0, n)) * scale).astype(dtype)
    x = rng.standard_normal(n)
    b = (A.astype(np.float64) @ x + noise * rng.standard_normal(m)).astype(dtype)
    return Dense(A, b, x, {"kind": "dense_scaled_columns", "m": m, "n": n, "seed": seed})


def sparse_csr(m: int, n: int, seed: int, nnz_per_col: int = 1000, dense_block: int = 1000,
               noise: float = 1e-3, dtype=np.float32) -> Sparse:
    """Each column gets nnz_per_col distinct uniformly random rows with N(0,1)
    values; a dense N(0,1) block on rows/columns [0, dense_block) makes A full
    rank.  CSR with int32 indices sorted within rows; duplicates are summed."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    k = min(nnz_per_col, m)
    for j in range(n):
        r = rng.choice(m, size=k, replace=False)
        rows.append(r)
        cols.append(np.full(k, j))
        vals.append(rng.standard_normal(k))
    db = min(dense_block, m, n)
    if db > 0:
        rr, cc = np.meshgrid(np.arange(db), np.arange(db), indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(rng.standard_normal(db * db))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A = sp.csr_matrix((A.data.astype(dtype), A.indices.astype(np.int32), A.indptr.astype(np.int32)),
                      shape=(m, n))
    x = rng.standard_normal(n)
    b = (A.astype(np.float64) @ x + noise * rng.standard_normal(m)).astype(dtype)
    return Sparse(A, b, x, {"kind": "sparse_csr", "m": m, "n": n, "seed": seed, "nnz": int(A.nnz)})


def serving_requests(count: int, rate: float, seed: int, log2_m=(12.0, 20.0),
                     n_choices=(16, 32, 64, 128, 256), d_factor: int = 4,
                     pool_rows: int = 1 << 23):
    """Poisson arrivals at `rate` per second; m = floor(2^U[lo, hi]); n uniform
    over n_choices; d = d_factor * n.  Returns a list of dicts sorted by arrival.
    "offset" is the request's first row in the pool of its n: the requests of
    one n take consecutive windows through a pool of pool_rows rows (wrapping
    round), so requests that are in flight together never share rows."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    ms = np.floor(2.0 ** rng.uniform(log2_m[0], log2_m[1], size=count)).astype(np.int64)
    ns = rng.choice(np.asarray(n_choices), size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    nxt = {int(n): 0 for n in n_choices}
    out = []
    for i in range(count):
        n, m = int(ns[i]), int(ms[i])
        off = nxt[n] if nxt[n] + m <= pool_rows else 0
        nxt[n] = off + m
        out.append({"id": i, "t": float(t[i]), "m": m, "n": n, "d": int(d_factor * n),
                    "seed": int(seeds[i]), "offset": off})
    return out


def serving_pool(rows: int = 1 << 20, n_choices=(16, 32, 64, 128, 256), seed: int = 0,
                 noise: float = 1e-3, device="cuda", fp64: bool = False):
    """Device-resident data for the serving mix (the whole run does not fit in
    memory as separate matrices).  For each n: A_n (rows x n, N(0,1), fp32, or
    fp64 with fp64=True), x_n ~ N(0, I) and b_n = A_n x_n + noise N(0, I),
    drawn with torch's seeded generator on the device.  A request (m, n) uses
    the contiguous row window request_window() of A_n, b_n, which is itself
    a problem with i.i.d. N(0,1) entries and b = A x_n + noise."""
    import torch
    g = torch.Generator(device=device)
    out = {}
    for k, n in enumerate(n_choices):
        g.manual_seed(seed * 1000 + k)
        A = torch.randn(rows, n, generator=g, device=device, dtype=torch.float32)
        x = torch.randn(n, generator=g, device=device, dtype=torch.float64)
        e = torch.randn(rows, generator=g, device=device, dtype=torch.float64)
        Ad = A.double() if fp64 else None
        b64 = (Ad if fp64 else A.double()) @ x + noise * e
        out[n] = dict(A=Ad if fp64 else A, b=b64 if fp64 else b64.float(), x=x.cpu().numpy())
        del e
    return out


def request_window(req: dict, rows: int):
    """First row of the request's window in its pool (deterministic): the
    consecutive-window offset when the request carries one and it fits."""
    off = req.get("offset")
    if off is not None and off + int(req["m"]) <= rows:
        return int(off)
    return int(req["seed"]) % (rows - int(req["m"]) + 1)


def paper_benchmark(m: int, n: int, seed: int, cond: float = 1e10, beta: float = 1e-10) -> Dense:
    """Sec. 3.1 family: A = U diag(sigma) V^T with Haar U (m x n) and V (n x n),
    sigma log-spaced 1 .. 1/cond; b = A x + beta r_perp with r_perp a unit
    vector orthogonal to range(A), so the optimal residual norm is beta."""
    rng = np.random.default_rng(seed)
    U, R = np.linalg.qr(rng.standard_normal((m, n)))
    U = U * np.sign(np.diag(R))
    V = random_orthogonal(n, rng)
    sigma = np.logspace(0.0, -np.log10(cond), n)
    A = (U * sigma) @ V.T
    x = rng.standard_normal(n)
    x /= np.linalg.norm(x)
    z = rng.standard_normal(m)
    z -= U @ (U.T @ z)
    z /= np.linalg.norm(z)
    b = A @ x + beta * z
    return Dense(A, b, x, {"kind": "paper_benchmark", "m": m, "n": n, "seed": seed,
                           "cond": cond, "beta": beta})


def paper_benchmark_device(m: int, n: int, seed: int, cond: float = 1e10, beta: float = 1e-10,
                           device="cuda"):
    """The paper_benchmark family drawn on the device with torch's seeded
    generator (the paper's largest sizes do not fit a host-side draw in
    reasonable time).  U is the Q factor of an m x n Gaussian by two rounds of
    Cholesky QR (positive diagonal, so U is Haar distributed), V the same for
    an n x n Gaussian; A = U diag(sigma) V^T, ||x|| = 1, b = A x + beta r_perp.
    Returns (A, b, x) as float64 device tensors; x is the exact least-squares
    solution and beta the optimal residual norm."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def orth(M):
        eye = torch.eye(M.shape[1], device=M.device, dtype=M.dtype)
        for _ in range(2):
            L = torch.linalg.cholesky(M.T @ M)
            Linv = torch.linalg.solve_triangular(L, eye, upper=False)  # small n x n solve
            M = M @ Linv.T
        return M

    U = orth(torch.randn(m, n, generator=g, device=device, dtype=torch.float64))
    V = orth(torch.randn(n, n, generator=g, device=device, dtype=torch.float64))
    sigma = torch.logspace(0.0, -float(np.log10(cond)), n, device=device, dtype=torch.float64)
    A = (U * sigma) @ V.T
    x = torch.randn(n, generator=g, device=device, dtype=torch.float64)
    x /= torch.linalg.norm(x)
    z = torch.randn(m, generator=g, device=device, dtype=torch.float64)
    z -= U @ (U.T @ z)
    z /= torch.linalg.norm(z)
    b = A @ x + beta * z
    del U, z
    return A, b, x


# Named workload configurations (sizes, sketch, solver settings).
CONFIGS = {
    "plain_fp64_20000x50": dict(gen="dense_gaussian", m=20000, n=50, d=200, dtype="f64",
                                sketch="count", refine=0, seed=DATA_SEED_BASE + 0),
    "illcond_fp32_4194304x256": dict(gen="dense_ill_conditioned", m=4194304, n=256, d=1024,
                                     dtype="f32", sketch="count", refine=1, iters=3,
                                     seed=DATA_SEED_BASE + 1),
    "csr_fp32_16777216x1000": dict(gen="sparse_csr", m=1 << 24, n=1000, d=4000, dtype="f32",
                                   sketch="count", refine=0, seed=DATA_SEED_BASE + 2),
    "gauss_bf16_262144x512": dict(gen="dense_scaled_columns", m=262144, n=512, d=2048, dtype="f32",
                                  sketch="gaussian", refine=1, rtol=1e-6, seed=DATA_SEED_BASE + 3),
    "serve_mix_10000": dict(gen="serving_requests", count=10000, rate=2000.0,
                            seed=DATA_SEED_BASE + 4),
}
