"""Autotuner driver for the launch shapes of the refinement pass, the
CountSketch gather and the blocked QR.

For each (dtype, n, m) of the pass sweep it fills a device matrix with N(0,1)
values, asks the library to time every candidate plan of the fused LSQR pass
(sns_tune_pass) and records the fastest as a tuning-table entry covering the
m range around the swept m (geometric midpoints between neighbours).  The
gather sweep does the same for the CountSketch gather with d = 4n
(sns_tune_gather: lanes per row, segments per bucket).  The QR sweep times
the panel configurations and trailing widths on a Gaussian [SA | Sb] of each
listed (d, n) (sns_tune_qr) and records an entry for exactly that shape;
other shapes keep the built-in rule.  By default the 4-wave pass entries of
one (dtype, n) then share one launch class (one_class_per_width).  The table is written where the Python
binding loads it from.

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
# gather sweep (d = 4n): the serving mix's widths in FP32, and FP64 widths
G_F32_N = (16, 32, 64, 128, 256)
G_F64_N = (16, 32, 50, 64, 128, 256)
G_MS = (1 << 12, 1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22)
# QR sweep: (d, n) of the serving mix (d = 4n), the 20000 x 50 problem, the
# dense 256-column and 512-column problems and the 1000-column sparse one
QR_SHAPES = ((64, 16), (128, 32), (256, 64), (512, 128), (1024, 256), (200, 50), (2048, 512),
             (4000, 1000))


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
                f"unroll {e.unroll} waves {e.waves}  {e.us:9.2f} us")
            del A, ws
    return out


def one_class_per_width(entries):
    """Give the 4-wave pass entries of one (dtype, n) the launch class (lanes
    per row, chunks per lane, rows per step) of the largest of them, each
    keeping its own work-group count.  4-wave entries cover the problems that
    may be batched with others (the tuner offers 8-wave work-groups only from
    2^29 entries up); a batch of one width then runs one pass class per
    iteration instead of several (the serving mix measured 2.7 % more
    solves/s).  8-wave entries, for problems that fill the device alone, keep
    their fastest shape."""
    top = {}
    for e in entries:
        if e.waves == 8:
            continue
        k = (e.dtype, e.n)
        if k not in top or e.m_hi > top[k].m_hi:
            top[k] = e
    for e in entries:
        t = top.get((e.dtype, e.n))
        if e.waves == 8 or t is None:
            continue
        e.lpr, e.nch, e.unroll = t.lpr, t.nch, t.unroll
    return entries


def reclass_file(path: str):
    """one_class_per_width applied to the pass lines of a table file in place
    (gather and QR lines are kept as they are).  The `us` column keeps the
    time the sweep measured for its own best shape."""
    from paper_2409_14309_amd._binding import TuneEntry
    lines = open(path).read().splitlines()
    idx, entries = [], []
    for i, ln in enumerate(lines):
        f = ln.split()
        if len(f) in (9, 10) and f[0] not in ("#", "G", "Q"):
            idx.append(i)
            entries.append(TuneEntry(int(f[0]), int(f[1]), int(f[2]), int(f[3]), int(f[4]),
                                     int(f[5]), int(f[6]), int(f[7]), float(f[8]),
                                     int(f[9]) if len(f) == 10 else 4))
    one_class_per_width(entries)
    for i, e in zip(idx, entries):
        lines[i] = (f"{e.dtype} {e.n} {e.m_lo} {e.m_hi} {e.lpr} {e.nch} {e.grid} {e.unroll} "
                    f"{e.us:.3f} {e.waves}")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def _m_range(ms, k):
    lo = 1 if k == 0 else int(math.sqrt(ms[k - 1] * ms[k]))
    hi = (1 << 31) - 1 if k == len(ms) - 1 else int(math.sqrt(ms[k] * ms[k + 1])) - 1
    return lo, hi


def sweep_gather(dtype_code: int, ns, ms, reps: int, log):
    import torch

    import paper_2409_14309_amd as sns
    tdt = torch.float64 if dtype_code == sns.SNS_F64 else torch.float32
    es = 8 if dtype_code == sns.SNS_F64 else 4
    out = []
    for n in ns:
        d = 4 * n
        ms_n = [m for m in ms if m * n * es <= MAX_BYTES and m >= d]
        for k, m in enumerate(ms_n):
            A = torch.randn(m, n, dtype=tdt, device="cuda")
            b = torch.randn(m, dtype=tdt, device="cuda")
            M = sns.dense(A)
            ws = torch.empty(sns.sns_tune_gather_workspace_size(M, d), dtype=torch.uint8,
                             device="cuda")
            e = sns.sns_tune_gather(M, b, d, 1234 + k, reps, ws)
            e.m_lo, e.m_hi = _m_range(ms_n, k)
            out.append(e)
            log(f"gather dtype {dtype_code} n {n:4d} d {d:5d} m {m:8d}: lpr {e.lpr:2d} "
                f"nseg {e.nseg:2d}  {e.us:9.2f} us")
            del A, b, ws
    return out


def sweep_qr(shapes, reps: int, log):
    import torch

    import paper_2409_14309_amd as sns
    out = []
    for d, n in shapes:
        g = torch.Generator(device="cuda").manual_seed(d * 131 + n)
        SA = torch.randn(d, n, dtype=torch.float32, device="cuda", generator=g)
        Sb = torch.randn(d, dtype=torch.float32, device="cuda", generator=g)
        ws = torch.empty(sns.sns_tune_qr_workspace_size(d, n), dtype=torch.uint8, device="cuda")
        e = sns.sns_tune_qr(SA, Sb, reps, ws)
        out.append(e)
        log(f"qr d {d:5d} n {n:5d}: cfg {e.cfg} cb {e.cb}  {e.us:9.2f} us")
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
    ap.add_argument("--only", choices=("pass", "gather", "qr"), nargs="*", default=None,
                    help="sweep only these kinds (default: all three)")
    ap.add_argument("--all-classes", action="store_true",
                    help="keep each m range's own pass class (default: one class per width)")
    ap.add_argument("--reclass", metavar="PATH", default=None,
                    help="only apply the one-class-per-width rule to the pass lines of a table "
                         "file (no GPU)")
    args = ap.parse_args(argv)
    if args.reclass:
        reclass_file(args.reclass)
        return
    kinds = set(args.only or ("pass", "gather", "qr"))

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
    count = 0
    if "pass" in kinds:
        entries = (sweep(sns.SNS_F32, f32_n, ms, args.reps, log)
                   + sweep(sns.SNS_F64, f64_n, ms, args.reps, log))
        if not args.all_classes:
            one_class_per_width(entries)
        for e in entries:
            sns.sns_tune_set(e)
        count += len(entries)
    if "gather" in kinds:
        gf32, gf64, gms = (G_F32_N, G_F64_N, G_MS) if not args.quick else ((64,), (50,), (1 << 16,))
        entries = (sweep_gather(sns.SNS_F32, gf32, gms, args.reps, log)
                   + sweep_gather(sns.SNS_F64, gf64, gms, args.reps, log))
        for e in entries:
            sns.sns_tune_gather_set(e)
        count += len(entries)
    if "qr" in kinds:
        entries = sweep_qr(QR_SHAPES if not args.quick else ((256, 64),), args.reps, log)
        for e in entries:
            sns.sns_tune_qr_set(e)
        count += len(entries)
    sns.sns_tune_save(out)
    log(f"{count} entries in {time.time() - t0:.1f}s -> {out}")


if __name__ == "__main__":
    main()
