"""ctypes binding of libsns (the C ABI declared in include/sns.h).

Argument marshalling only: every computation runs in the HIP library.  Device
buffers are torch tensors (their data_ptr() is passed); streams default to
torch's current stream.  A missing library raises instead of falling back.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsns.so")

SNS_OK = 0
STATUS_NAMES = ["SNS_OK", "SNS_ERR_INVALID_ARG", "SNS_ERR_SHAPE", "SNS_ERR_DTYPE",
                "SNS_ERR_RANK_DEFICIENT", "SNS_ERR_NOT_CONVERGED", "SNS_ERR_NUMERICAL",
                "SNS_ERR_OUT_OF_MEMORY", "SNS_ERR_QUEUE_FULL", "SNS_ERR_NOT_READY", "SNS_ERR_HIP"]
SNS_ERR_QUEUE_FULL, SNS_ERR_NOT_READY = 8, 9
SNS_F32, SNS_F64 = 0, 1
SNS_DENSE_ROWMAJOR, SNS_CSR = 0, 1
SNS_SKETCH_COUNT, SNS_SKETCH_GAUSSIAN, SNS_SKETCH_SPARSE_SIGN, SNS_SKETCH_HADAMARD = 0, 1, 2, 3


class SnsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{where}: {name}")


class Matrix(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("dtype", C.c_int), ("layout", C.c_int),
                ("values", C.c_void_p), ("ld", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("nnz", C.c_int64)]


class Sketch(C.Structure):
    _fields_ = [("kind", C.c_int), ("d", C.c_int64), ("seed", C.c_uint64), ("zeta", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("refine", C.c_int), ("max_iters", C.c_int), ("rtol", C.c_double),
                ("accum_fp64", C.c_int)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("rel_resid_est", C.c_double),
                ("sketch_resid", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("sketch", Sketch), ("A", Matrix), ("b", C.c_void_p), ("x", C.c_void_p),
                ("opts", SolveOpts)]


class ServeConfig(C.Structure):
    _fields_ = [("pool", C.c_void_p), ("pool_bytes", C.c_size_t), ("dtype", C.c_int),
                ("max_slots", C.c_int), ("queue_capacity", C.c_int), ("chunk_iters", C.c_int)]


class ServeStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("p50_ms", C.c_double),
                ("p99_ms", C.c_double), ("mean_ms", C.c_double), ("span_s", C.c_double),
                ("peak_pool_bytes", C.c_size_t), ("peak_slots", C.c_int), ("rounds", C.c_uint64)]


class TuneEntry(C.Structure):
    _fields_ = [("dtype", C.c_int), ("n", C.c_int), ("m_lo", C.c_int64), ("m_hi", C.c_int64),
                ("lpr", C.c_int), ("nch", C.c_int), ("grid", C.c_int), ("unroll", C.c_int),
                ("us", C.c_double), ("waves", C.c_int)]


class TuneGatherEntry(C.Structure):
    _fields_ = [("dtype", C.c_int), ("n", C.c_int), ("d", C.c_int), ("m_lo", C.c_int64),
                ("m_hi", C.c_int64), ("lpr", C.c_int), ("nseg", C.c_int), ("us", C.c_double)]


class TuneQrEntry(C.Structure):
    _fields_ = [("d_lo", C.c_int), ("d_hi", C.c_int), ("n_lo", C.c_int), ("n_hi", C.c_int),
                ("cfg", C.c_int), ("cb", C.c_int), ("us", C.c_double)]


TUNING_PATH = os.path.join(HERE, "tuning.txt")

_lib = None

_SIGS = {
    "sns_status_string": (C.c_char_p, [C.c_int]),
    "sns_version": (C.c_int, []),
    "sns_hash": (C.c_int, [C.c_uint64, C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                           C.c_void_p]),
    "sns_gaussian_table": (C.c_int, [C.c_void_p]),
    "sns_sketch_workspace_size": (C.c_int, [C.POINTER(Sketch), C.POINTER(Matrix),
                                            C.POINTER(C.c_size_t)]),
    "sns_sketch_apply": (C.c_int, [C.POINTER(Sketch), C.POINTER(Matrix), C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.POINTER(SolveOpts), C.c_void_p, C.c_size_t,
                                   C.c_void_p]),
    "sns_qr_solve_workspace_size": (C.c_int, [C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "sns_qr_solve": (C.c_int, [C.c_int64, C.c_int64, C.c_int, C.c_void_p, C.c_int64, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.POINTER(Info), C.c_void_p, C.c_size_t,
                               C.c_void_p]),
    "sns_qr_solve_noalloc": (C.c_int, [C.c_int64, C.c_int64, C.c_int, C.c_void_p, C.c_int64,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Info),
                                       C.c_void_p]),
    "sns_lstsq_workspace_size": (C.c_int, [C.POINTER(Sketch), C.POINTER(Matrix),
                                           C.POINTER(SolveOpts), C.POINTER(C.c_size_t)]),
    "sns_lstsq": (C.c_int, [C.POINTER(Sketch), C.POINTER(Matrix), C.c_void_p, C.c_void_p,
                            C.POINTER(SolveOpts), C.c_void_p, C.c_size_t, C.POINTER(Info),
                            C.c_void_p]),
    "sns_lstsq_batched_workspace_size": (C.c_int, [C.POINTER(Problem), C.c_int,
                                                   C.POINTER(C.c_size_t)]),
    "sns_lstsq_batched": (C.c_int, [C.POINTER(Problem), C.c_int, C.c_void_p, C.c_size_t,
                                    C.POINTER(Info), C.c_int, C.c_void_p]),
    "sns_serve_create": (C.c_int, [C.POINTER(ServeConfig), C.POINTER(C.c_void_p)]),
    "sns_serve_submit": (C.c_int, [C.c_void_p, C.POINTER(Problem), C.POINTER(C.c_uint64)]),
    "sns_serve_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(Info)]),
    "sns_serve_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(Info)]),
    "sns_serve_stats_get": (C.c_int, [C.c_void_p, C.POINTER(ServeStats)]),
    "sns_serve_destroy": (C.c_int, [C.c_void_p]),
    "sns_tune_workspace_size": (C.c_int, [C.POINTER(Matrix), C.POINTER(C.c_size_t)]),
    "sns_tune_pass": (C.c_int, [C.POINTER(Matrix), C.c_int, C.c_void_p, C.c_size_t,
                                C.POINTER(TuneEntry), C.c_void_p]),
    "sns_tune_set": (C.c_int, [C.POINTER(TuneEntry)]),
    "sns_tune_gather_workspace_size": (C.c_int, [C.POINTER(Matrix), C.c_int64,
                                                 C.POINTER(C.c_size_t)]),
    "sns_tune_gather": (C.c_int, [C.POINTER(Matrix), C.c_void_p, C.c_int64, C.c_uint64, C.c_int,
                                  C.c_void_p, C.c_size_t, C.POINTER(TuneGatherEntry),
                                  C.c_void_p]),
    "sns_tune_qr_workspace_size": (C.c_int, [C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "sns_tune_qr": (C.c_int, [C.c_int, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_int,
                              C.c_void_p, C.c_size_t, C.POINTER(TuneQrEntry), C.c_void_p]),
    "sns_tune_gather_set": (C.c_int, [C.POINTER(TuneGatherEntry)]),
    "sns_tune_qr_set": (C.c_int, [C.POINTER(TuneQrEntry)]),
    "sns_tune_clear": (C.c_int, []),
    "sns_tune_load": (C.c_int, [C.c_char_p]),
    "sns_tune_save": (C.c_int, [C.c_char_p]),
    "sns_timing_enable": (None, [C.c_int]),
    "sns_fused_enable": (None, [C.c_int]),
    "sns_fused_enabled": (C.c_int, []),
    "sns_timing_select": (None, [C.c_char_p]),
    "sns_timing_reset": (None, []),
    "sns_timing_summary": (C.c_int, [C.c_char_p, C.c_size_t]),
}


def load(path: str | None = None):
    """Load libsns.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    # torch brings its own HIP runtime: load it first so that libsns binds to
    # the same runtime as the device memory it is handed
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(p):
        raise RuntimeError(f"libsns.so not built ({p}); run `python -m paper_2409_14309_amd.build`")
    lib = C.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    # the tuning table written by the autotuner, when present
    if os.path.exists(TUNING_PATH):
        _check(lib.sns_tune_load(TUNING_PATH.encode()), "sns_tune_load")
    return lib


def exported_symbols():
    return list(_SIGS)


def _check(status: int, where: str):
    if status != SNS_OK:
        raise SnsError(status, where)


def _torch():
    import torch
    return torch


def _stream(stream):
    if stream is None:
        return C.c_void_p(_torch().cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float32:
        return SNS_F32
    if t.dtype == torch.float64:
        return SNS_F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def dense(A) -> Matrix:
    """Describe a 2-D device tensor (row-major, unit column stride) as sns_matrix."""
    if A.dim() != 2 or A.stride(1) != 1 or (A.shape[0] > 1 and A.stride(0) < A.shape[1]):
        raise ValueError("A must be 2-D and row-major with unit column stride")
    return Matrix(A.shape[0], A.shape[1], _dtype_code(A), SNS_DENSE_ROWMAJOR, A.data_ptr(),
                  A.stride(0), None, None, 0)


def csr(row_ptr, col_idx, values, m: int, n: int) -> Matrix:
    return Matrix(m, n, _dtype_code(values), SNS_CSR, values.data_ptr(), 0, row_ptr.data_ptr(),
                  col_idx.data_ptr(), values.numel())


SKETCH_KINDS = {"count": SNS_SKETCH_COUNT, "gaussian": SNS_SKETCH_GAUSSIAN,
                "sparse": SNS_SKETCH_SPARSE_SIGN, "hadamard": SNS_SKETCH_HADAMARD}


def sketch_desc(kind: str, d: int, seed: int, zeta: int = 1) -> Sketch:
    """kind: "count" (CountSketch), "gaussian", "sparse" (sparse sign
    embedding with zeta nonzeros per column) or "hadamard" (SRHT)."""
    return Sketch(SKETCH_KINDS[kind], d, seed, zeta)


def opts(refine: int = 0, max_iters: int = 0, rtol: float = 0.0, accum_fp64: int = 0) -> SolveOpts:
    return SolveOpts(refine, max_iters, rtol, accum_fp64)


# ---------------------------------------------------------------- calls ----

def sns_version() -> int:
    return load().sns_version()


def sns_status_string(status: int) -> str:
    return load().sns_status_string(status).decode()


def sns_hash(seed: int, d: int, i0: int, count: int, h=None, s=None, stream=None):
    _check(load().sns_hash(seed, d, i0, count, _ptr(h), _ptr(s), _stream(stream)), "sns_hash")


def sns_gaussian_table():
    import numpy as np
    out = np.zeros(256, dtype=np.uint16)
    _check(load().sns_gaussian_table(out.ctypes.data_as(C.c_void_p)), "sns_gaussian_table")
    return out


def sns_sketch_workspace_size(sk: Sketch, A: Matrix) -> int:
    n = C.c_size_t(0)
    _check(load().sns_sketch_workspace_size(C.byref(sk), C.byref(A), C.byref(n)),
           "sns_sketch_workspace_size")
    return n.value


def sns_sketch_apply(sk: Sketch, A: Matrix, b, SA, Sb, workspace, opt: SolveOpts | None = None,
                     stream=None):
    _check(load().sns_sketch_apply(C.byref(sk), C.byref(A), _ptr(b), _ptr(SA), _ptr(Sb),
                                   C.byref(opt) if opt is not None else None, _ptr(workspace),
                                   workspace.numel() * workspace.element_size(), _stream(stream)),
           "sns_sketch_apply")


def sns_qr_solve_workspace_size(d: int, n: int) -> int:
    b = C.c_size_t(0)
    _check(load().sns_qr_solve_workspace_size(d, n, C.byref(b)), "sns_qr_solve_workspace_size")
    return b.value


def sns_qr_solve(d: int, n: int, SA, Sb, x0, R, workspace, info: Info | None = None,
                 stream=None):
    _check(load().sns_qr_solve(d, n, _dtype_code(SA), _ptr(SA), SA.stride(0), _ptr(Sb), _ptr(x0),
                               _ptr(R), C.byref(info) if info is not None else None,
                               _ptr(workspace), workspace.numel() * workspace.element_size(),
                               _stream(stream)), "sns_qr_solve")


def sns_qr_solve_noalloc(d: int, n: int, SA, Sb, x0, R, info: Info | None = None, stream=None):
    """sns_qr_solve with the workspace in the library's static device array."""
    _check(load().sns_qr_solve_noalloc(d, n, _dtype_code(SA), _ptr(SA), SA.stride(0), _ptr(Sb),
                                       _ptr(x0), _ptr(R),
                                       C.byref(info) if info is not None else None,
                                       _stream(stream)), "sns_qr_solve_noalloc")


def sns_lstsq_workspace_size(sk: Sketch, A: Matrix, opt: SolveOpts) -> int:
    b = C.c_size_t(0)
    _check(load().sns_lstsq_workspace_size(C.byref(sk), C.byref(A), C.byref(opt), C.byref(b)),
           "sns_lstsq_workspace_size")
    return b.value


def sns_lstsq(sk: Sketch, A: Matrix, b, x, opt: SolveOpts, workspace, info: Info | None = None,
              stream=None):
    _check(load().sns_lstsq(C.byref(sk), C.byref(A), _ptr(b), _ptr(x), C.byref(opt),
                            _ptr(workspace), workspace.numel() * workspace.element_size(),
                            C.byref(info) if info is not None else None, _stream(stream)),
           "sns_lstsq")


def problem(sk: Sketch, A: Matrix, b, x, opt: SolveOpts) -> Problem:
    return Problem(sk, A, b.data_ptr(), x.data_ptr(), opt)


def sns_lstsq_batched_workspace_size(probs) -> int:
    arr = (Problem * len(probs))(*probs)
    n = C.c_size_t(0)
    _check(load().sns_lstsq_batched_workspace_size(arr, len(probs), C.byref(n)),
           "sns_lstsq_batched_workspace_size")
    return n.value


def sns_lstsq_batched(probs, workspace, infos=None, use_graph: bool = True, stream=None):
    """infos: a ctypes array of Info (len(probs)) or None."""
    arr = (Problem * len(probs))(*probs)
    _check(load().sns_lstsq_batched(arr, len(probs), _ptr(workspace),
                                    workspace.numel() * workspace.element_size(), infos,
                                    1 if use_graph else 0, _stream(stream)),
           "sns_lstsq_batched")


# ------------------------------------------------------------ serving ----

def sns_serve_create(pool, dtype: int, max_slots: int = 64, queue_capacity: int = 65536,
                     chunk_iters: int = 4):
    """Server handle over the device tensor `pool` (kept alive by the caller)."""
    cfg = ServeConfig(pool.data_ptr(), pool.numel() * pool.element_size(), dtype, max_slots,
                      queue_capacity, chunk_iters)
    h = C.c_void_p()
    _check(load().sns_serve_create(C.byref(cfg), C.byref(h)), "sns_serve_create")
    return h


def sns_serve_submit(srv, prob: Problem) -> int:
    t = C.c_uint64(0)
    _check(load().sns_serve_submit(srv, C.byref(prob), C.byref(t)), "sns_serve_submit")
    return t.value


def sns_serve_poll(srv, ticket: int):
    """Info once the request has completed, else None."""
    info = Info()
    st = load().sns_serve_poll(srv, ticket, C.byref(info))
    if st == SNS_ERR_NOT_READY:
        return None
    _check(st, "sns_serve_poll")
    return info


def sns_serve_wait(srv, ticket: int) -> Info:
    info = Info()
    _check(load().sns_serve_wait(srv, ticket, C.byref(info)), "sns_serve_wait")
    return info


def sns_serve_stats_get(srv) -> ServeStats:
    s = ServeStats()
    _check(load().sns_serve_stats_get(srv, C.byref(s)), "sns_serve_stats_get")
    return s


def sns_serve_destroy(srv):
    _check(load().sns_serve_destroy(srv), "sns_serve_destroy")


# ---------------------------------------------------------- autotuner ----

def sns_tune_workspace_size(A: Matrix) -> int:
    n = C.c_size_t(0)
    _check(load().sns_tune_workspace_size(C.byref(A), C.byref(n)), "sns_tune_workspace_size")
    return n.value


def sns_tune_pass(A: Matrix, reps: int, workspace, stream=None) -> TuneEntry:
    e = TuneEntry()
    _check(load().sns_tune_pass(C.byref(A), reps, _ptr(workspace),
                                workspace.numel() * workspace.element_size(), C.byref(e),
                                _stream(stream)), "sns_tune_pass")
    return e


def sns_tune_set(e: TuneEntry):
    _check(load().sns_tune_set(C.byref(e)), "sns_tune_set")


def sns_tune_gather_workspace_size(A: Matrix, d: int) -> int:
    n = C.c_size_t(0)
    _check(load().sns_tune_gather_workspace_size(C.byref(A), d, C.byref(n)),
           "sns_tune_gather_workspace_size")
    return n.value


def sns_tune_gather(A: Matrix, b, d: int, seed: int, reps: int, workspace,
                    stream=None) -> TuneGatherEntry:
    e = TuneGatherEntry()
    _check(load().sns_tune_gather(C.byref(A), _ptr(b), d, seed, reps, _ptr(workspace),
                                  workspace.numel() * workspace.element_size(), C.byref(e),
                                  _stream(stream)), "sns_tune_gather")
    return e


def sns_tune_qr_workspace_size(d: int, n: int) -> int:
    k = C.c_size_t(0)
    _check(load().sns_tune_qr_workspace_size(d, n, C.byref(k)), "sns_tune_qr_workspace_size")
    return k.value


def sns_tune_qr(SA, Sb, reps: int, workspace, stream=None) -> TuneQrEntry:
    """SA: (d, n) contiguous device tensor, Sb: (d,), both float32 or float64."""
    d, n = SA.shape
    e = TuneQrEntry()
    _check(load().sns_tune_qr(_dtype_code(SA), d, n, _ptr(SA), _ptr(Sb), reps, _ptr(workspace),
                              workspace.numel() * workspace.element_size(), C.byref(e),
                              _stream(stream)), "sns_tune_qr")
    return e


def sns_tune_gather_set(e: TuneGatherEntry):
    _check(load().sns_tune_gather_set(C.byref(e)), "sns_tune_gather_set")


def sns_tune_qr_set(e: TuneQrEntry):
    _check(load().sns_tune_qr_set(C.byref(e)), "sns_tune_qr_set")


def sns_tune_clear():
    _check(load().sns_tune_clear(), "sns_tune_clear")


def sns_tune_load(path: str):
    _check(load().sns_tune_load(path.encode()), "sns_tune_load")


def sns_tune_save(path: str):
    _check(load().sns_tune_save(path.encode()), "sns_tune_save")


# ----------------------------------------------------- fused set-up ----

def sns_fused_enable(on: bool = True):
    """Small problems (d <= 256, n <= 64, m (n + 1) <= 2^21) set up in the
    persistent fused launch, or (False, the default) on the blocked path like
    larger ones."""
    load().sns_fused_enable(1 if on else 0)


def sns_fused_enabled() -> bool:
    return bool(load().sns_fused_enabled())


# ------------------------------------------------------------- timing ----

def sns_timing_enable(on: bool = True):
    load().sns_timing_enable(1 if on else 0)


def sns_timing_select(names=None):
    """Time only the named kernels (an iterable of names, or None for all)."""
    load().sns_timing_select(None if names is None else ",".join(names).encode())


def sns_timing_reset():
    load().sns_timing_reset()


def sns_timing_summary() -> dict:
    """{kernel: (launches, total_ms, avg_us)} of the launches timed so far."""
    lib = load()
    need = lib.sns_timing_summary(None, 0)
    buf = C.create_string_buffer(need + 1)
    lib.sns_timing_summary(buf, need + 1)
    out = {}
    for line in buf.value.decode().splitlines():
        if not line or line.startswith("#"):
            continue
        name, cnt, tot, avg = line.split()
        out[name] = (int(cnt), float(tot), float(avg))
    return out
