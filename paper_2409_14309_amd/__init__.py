"""Sketch-and-solve least squares on MI355X (gfx950).

The compute lives in libsns.so (HIP); this package is its Python binding.
Names follow the C ABI of include/sns.h.  Convenience wrappers (`sketch`,
`lstsq`) allocate the workspace with torch and call the ABI.
"""
from __future__ import annotations

from ._binding import (SNS_CSR, SNS_DENSE_ROWMAJOR, SNS_F32, SNS_F64, SNS_SKETCH_COUNT,  # noqa: F401
                       ServeConfig, ServeStats, TuneEntry, sns_serve_create, sns_serve_destroy,
                       sns_tune_clear, sns_tune_load, sns_tune_pass, sns_tune_save, sns_tune_set,
                       sns_tune_workspace_size, TuneGatherEntry, TuneQrEntry, sns_tune_gather,
                       sns_tune_gather_set, sns_tune_gather_workspace_size, sns_tune_qr,
                       sns_tune_qr_set, sns_tune_qr_workspace_size,
                       sns_serve_poll, sns_serve_stats_get, sns_serve_submit, sns_serve_wait,
                       SNS_SKETCH_GAUSSIAN, Info, Matrix, Problem, Sketch, SnsError, SolveOpts,
                       csr, dense, exported_symbols, load, opts, problem, sketch_desc,
                       sns_gaussian_table, sns_hash, sns_lstsq, sns_lstsq_batched,
                       sns_lstsq_batched_workspace_size, sns_lstsq_workspace_size,
                       sns_qr_solve, sns_qr_solve_noalloc, sns_qr_solve_workspace_size, sns_sketch_apply,
                       sns_sketch_workspace_size, sns_status_string, sns_timing_enable,
                       sns_fused_enable, sns_fused_enabled,
                       sns_timing_reset, sns_timing_select, sns_timing_summary, sns_version)


class CsrMatrix:
    """A CSR matrix held in device tensors: row_ptr int32[m+1], col_idx
    int32[nnz] (distinct columns within a row), values float32/float64[nnz]."""

    def __init__(self, row_ptr, col_idx, values, shape):
        self.row_ptr, self.col_idx, self.values = row_ptr, col_idx, values
        self.shape = (int(shape[0]), int(shape[1]))
        self.dtype, self.device = values.dtype, values.device


def check_args(A, b=None, x=None, need_cuda: bool = True):
    """Reject tensors the kernels would misread, before anything is launched:
    every tensor on one device (a GPU unless need_cuda is False), A dense
    (2-D float32/float64 with unit column stride and row stride >= n) or a
    CsrMatrix (contiguous int32 row_ptr of m+1 and col_idx of nnz entries,
    contiguous float32/float64 values), b contiguous with m entries of A's
    dtype, x contiguous float64 with n entries.  Raises ValueError."""
    import torch
    tensors = []
    if isinstance(A, CsrMatrix):
        m, n = A.shape
        for name, t, dt in (("row_ptr", A.row_ptr, torch.int32), ("col_idx", A.col_idx, torch.int32)):
            if not isinstance(t, torch.Tensor) or t.dtype != dt or not t.is_contiguous():
                raise ValueError(f"CSR {name} must be a contiguous int32 tensor")
        if A.row_ptr.numel() != m + 1:
            raise ValueError(f"CSR row_ptr has {A.row_ptr.numel()} entries, expected m + 1 = {m + 1}")
        v = A.values
        if not isinstance(v, torch.Tensor) or v.dtype not in (torch.float32, torch.float64) \
                or not v.is_contiguous():
            raise ValueError("CSR values must be a contiguous float32 or float64 tensor")
        if A.col_idx.numel() != v.numel():
            raise ValueError("CSR col_idx and values must have the same number of entries")
        tensors += [A.row_ptr, A.col_idx, v]
        dtype = v.dtype
    else:
        if not isinstance(A, torch.Tensor) or A.dim() != 2:
            raise ValueError("A must be a 2-D tensor or a CsrMatrix")
        if A.dtype not in (torch.float32, torch.float64):
            raise ValueError(f"A must be float32 or float64, not {A.dtype}")
        m, n = A.shape
        if A.stride(1) != 1 or (m > 1 and A.stride(0) < n):
            raise ValueError("A must be row-major with unit column stride")
        tensors.append(A)
        dtype = A.dtype
    if b is not None:
        if not isinstance(b, torch.Tensor) or b.dtype != dtype:
            raise ValueError(f"b must be a tensor of A's dtype {dtype}")
        if not b.is_contiguous() or b.numel() != m:
            raise ValueError(f"b must be contiguous with m = {m} entries")
        tensors.append(b)
    if x is not None:
        if not isinstance(x, torch.Tensor) or x.dtype != torch.float64:
            raise ValueError("x must be a float64 tensor")
        if not x.is_contiguous() or x.numel() != n:
            raise ValueError(f"x must be contiguous with n = {n} entries")
        tensors.append(x)
    dev = tensors[0].device
    for t in tensors:
        if t.device != dev:
            raise ValueError("A, b and x must be on the same device")
    if need_cuda and dev.type != "cuda":
        raise ValueError(f"A, b and x must be in GPU memory, not on {dev}")
    return m, n


def _describe(A) -> Matrix:
    if isinstance(A, CsrMatrix):
        return csr(A.row_ptr, A.col_idx, A.values, A.shape[0], A.shape[1])
    return dense(A)


def _workspace(nbytes: int, device):
    import torch
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def sketch(A, b=None, kind: str = "count", d: int = None, seed: int = 42, accum_fp64: bool = False,
           stream=None, zeta: int = 1):
    """SA, Sb = S A, S b for a dense device tensor or a CsrMatrix A (and
    optional b)."""
    import torch
    check_args(A, b)
    sk = sketch_desc(kind, d, seed, zeta)
    M = _describe(A)
    ws = _workspace(sns_sketch_workspace_size(sk, M), A.device)
    SA = torch.empty((d, A.shape[1]), dtype=A.dtype, device=A.device)
    Sb = torch.empty(d, dtype=A.dtype, device=A.device) if b is not None else None
    sns_sketch_apply(sk, M, b, SA, Sb, ws, opts(accum_fp64=int(accum_fp64)), stream)
    return SA, Sb


REFINE = {False: 0, True: 1, 0: 0, 1: 1, 2: 2, "sas": 0, "sap": 1, "saa": 2}


def lstsq(A, b, kind: str = "count", d: int = None, seed: int = 42, refine=False,
          max_iters: int = 100, rtol: float = 1e-6, accum_fp64: bool = False, stream=None,
          zeta: int = 1):
    """x (float64 device tensor) and Info for min ||A x - b||.  refine: False /
    "sas" (plain sketch-and-solve), True / "sap" (SAP-SAS) or "saa" (SAA-SAS)."""
    import torch
    check_args(A, b)
    sk = sketch_desc(kind, d, seed, zeta)
    M = _describe(A)
    r = REFINE[refine]
    o = opts(r, max_iters if r else 0, rtol if r else 0.0, int(accum_fp64))
    ws = _workspace(sns_lstsq_workspace_size(sk, M, o), A.device)
    x = torch.empty(A.shape[1], dtype=torch.float64, device=A.device)
    info = Info()
    sns_lstsq(sk, M, b, x, o, ws, info, stream)
    (stream or torch.cuda.current_stream()).synchronize()
    return x, info


def lstsq_batched(As, bs, ds, seeds, refine: bool = True, max_iters: int = 100, rtol: float = 1e-6,
                  use_graph: bool = True, stream=None, zeta: int = 1):
    """Solve several dense problems in one batch (CountSketch, or the sparse
    sign embedding with zeta > 1); returns ([x], [Info])."""
    import torch
    probs, xs = [], []
    for A, b, d, seed in zip(As, bs, ds, seeds):
        check_args(A, b)
        x = torch.empty(A.shape[1], dtype=torch.float64, device=A.device)
        o = opts(int(refine), max_iters if refine else 0, rtol if refine else 0.0)
        sk = sketch_desc("sparse", d, seed, zeta) if zeta > 1 else sketch_desc("count", d, seed)
        probs.append(problem(sk, dense(A), b, x, o))
        xs.append(x)
    ws = _workspace(sns_lstsq_batched_workspace_size(probs), As[0].device)
    infos = (Info * len(probs))()
    sns_lstsq_batched(probs, ws, infos, use_graph, stream)
    (stream or torch.cuda.current_stream()).synchronize()
    return xs, list(infos)


class Server:
    """Continuous-batching solver service over a device memory pool.

    submit() queues a dense CountSketch (or, with zeta > 1, sparse sign
    embedding) problem (device tensors A, b; the
    answer goes to a new fp64 tensor) and returns a ticket; wait()/poll()
    return (x, Info) once it has completed.  submit() first waits for the
    caller's current stream, so work queued there on A, b or x is complete
    before the server's own streams touch them."""

    def __init__(self, pool_bytes: int, dtype=None, max_slots: int = 64,
                 queue_capacity: int = 65536, chunk_iters: int = 4, device=None):
        import torch
        self.pool = torch.empty(pool_bytes, dtype=torch.uint8, device=device or "cuda")
        code = SNS_F64 if dtype == torch.float64 else SNS_F32
        self.handle = sns_serve_create(self.pool, code, max_slots, queue_capacity, chunk_iters)
        self._live = {}

    def submit(self, A, b, d: int, seed: int, refine: bool = True, max_iters: int = 100,
               rtol: float = 1e-6, x=None, zeta: int = 1) -> int:
        import torch
        check_args(A, b, x)
        if x is None:
            x = torch.empty(A.shape[1], dtype=torch.float64, device=A.device)
        o = opts(int(refine), max_iters if refine else 0, rtol if refine else 0.0)
        sk = sketch_desc("sparse", d, seed, zeta) if zeta > 1 else sketch_desc("count", d, seed)
        # the server's streams do not wait on the caller's: whatever the
        # caller's stream still has queued on A, b or x must finish first
        torch.cuda.current_stream(A.device).synchronize()
        t = sns_serve_submit(self.handle, problem(sk, dense(A), b, x, o))
        self._live[t] = (A, b, x)  # keep the buffers alive while the request runs
        return t

    def poll(self, ticket: int):
        info = sns_serve_poll(self.handle, ticket)
        if info is None:
            return None
        return self._live.pop(ticket)[2], info

    def wait(self, ticket: int):
        info = sns_serve_wait(self.handle, ticket)
        return self._live.pop(ticket)[2], info

    def stats(self):
        return sns_serve_stats_get(self.handle)

    def close(self):
        if self.handle is not None:
            sns_serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
