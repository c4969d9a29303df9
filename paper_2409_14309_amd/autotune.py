"""Autotuner driver for the refinement pass's launch shape.

For each (dtype, n, m) of the sweep it fills a device matrix with N(0,1)
values, asks the library to time every candidate plan of the fused LSQR pass
(sns_tune_pass) and records the fastest as a tuning-table entry covering the
m range around the swept m (geometric midpoints between neighbours).  The
table is written where the Python binding loads it from.

    python -m paper_2409_14309_amd.autotune [--out PATH] [--quick]
    python -m paper_2409_14309_amd.autotune --merge --f64-n 1000   # add shapes to the table
"""
from __future__ import annotations

import argparse
import math
import sys
import time

F32_N = (16, 32, 64, 128, 256, 512, 1024, 2048)
F64_N = (16, 32, 50, 64, 128, 256, 512)
MS = (1 << 12, 1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22)
MAX_BYTES = 16 << 30


def sweep(dtype_code: int, ns, ms, reps: int, log):
    import torch

    import paper_2409_14309_amd as sns
    tdt = torch.float64 if dtype_code == sns.SNS_F64 else torch.float32
    es = 8 if dtype_code == sns.SNS_F64 else 4
    out = []
    for n in ns:
        ms_n = [m for m in ms if m * n * es <= MAX_BYTES]
        for k, m in enumerate(ms_n):
            A = torch.randn(m, n, dtype=tdt, device="cuda")
            M = sns.dense(A)
            ws = torch.empty(sns.sns_tune_workspace_size(M), dtype=torch.uint8, device="cuda")
            e = sns.sns_tune_pass(M, reps if m < (1 << 20) else max(3, reps // 2), ws)
            lo = 1 if k == 0 else int(math.sqrt(ms_n[k - 1] * m))
            hi = (1 << 31) - 1 if k == len(ms_n) - 1 else int(math.sqrt(m * ms_n[k + 1])) - 1
            e.m_lo, e.m_hi = lo, hi
            out.append(e)
            log(f"dtype {dtype_code} n {n:5d} m {m:8d}: lpr {e.lpr:2d} nch {e.nch} grid {e.grid:4d} "
                f"unroll {e.unroll}  {e.us:9.2f} us")
            del A, ws
    return out


def main(argv=None):
    import paper_2409_14309_amd as sns
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="table path (default: next to libsns.so)")
    ap.add_argument("--quick", action="store_true", help="few shapes (for tests)")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--merge", action="store_true",
                    help="keep the current table and add or replace only the swept shapes")
    ap.add_argument("--f32-n", type=int, nargs="*", default=None, help="fp32 widths to sweep")
    ap.add_argument("--f64-n", type=int, nargs="*", default=None, help="fp64 widths to sweep")
    args = ap.parse_args(argv)

    def log(msg):
        print(f"[autotune] {msg}", file=sys.stderr, flush=True)

    from paper_2409_14309_amd._binding import TUNING_PATH
    out = args.out or TUNING_PATH
    sns.load()
    if not args.merge:
        sns.sns_tune_clear()  # time against the built-in rule only
    t0 = time.time()
    f32_n, f64_n, ms = (F32_N, F64_N, MS) if not args.quick else ((64,), (50,), (1 << 14, 1 << 18))
    if args.f32_n is not None or args.f64_n is not None:
        f32_n, f64_n = tuple(args.f32_n or ()), tuple(args.f64_n or ())
    entries = sweep(sns.SNS_F32, f32_n, ms, args.reps, log) + sweep(sns.SNS_F64, f64_n, ms, args.reps, log)
    for e in entries:
        sns.sns_tune_set(e)
    sns.sns_tune_save(out)
    log(f"{len(entries)} entries in {time.time() - t0:.1f}s -> {out}")


if __name__ == "__main__":
    main()
