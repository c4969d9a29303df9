#!/usr/bin/env python3
"""Benchmark of the sketch-and-solve least-squares hot path on one MI355X.

A step is one complete solve of min ||A x - b|| for the ill-conditioned FP32
workload (A 4,194,304 x 256, sigma log-spaced 1 .. 1e-6, relative noise 1e-4):
CountSketch of [A | b] with d = 1024 (bucket sort + segmented reduction), FP64
Householder QR of [SA | Sb], triangular solve, then R^{-1}-preconditioned LSQR
on the full A until the device stop rule certifies residual error <= 1e-6.
Inputs are resident in HBM before timing starts.  --workload
gauss_bf16_262144x512 times the same solve with the dense Gaussian sketch
(d = 2048, bf16 MFMA) of a 262,144 x 512 column-scaled matrix instead;
--workload paper_fp64_1000000x1000 times the benchmark family of Sec. 3.1
(FP64, kappa 1e10, beta 1e-10, n = 1000, d = 4000; --m picks the row count) and
reports its residual and forward errors against the exact solution built into
the data.  --solver saa replaces SAP-SAS by SAA-SAS (Y = A R^-1 formed once);
--zeta Z > 1 uses the sparse sign embedding instead of the CountSketch,
--sketch hadamard the subsampled randomized Hadamard transform, --d the
sketch size.  --workload serve_mix_10000 drives the continuous-batching server
with 10,000 requests (Poisson arrivals at 2000/s, m = floor(2^U[12,20]),
n in {16, ..., 256}, d = 4n): open-loop latency percentiles, saturated
throughput (value) and one-problem-at-a-time baselines.

Prints one JSON line: solves/s (value), p50/p99 step latency, the CountSketch
pass bandwidth, a roofline record for the dominant kernel (timed with HIP
events inside the library over the timed region) and the CPU oracle timed on a
bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CountSketch HBM GB/s (% peak); LS solves/s + p99 latency at rel-residual 1e-6"
HBM_PEAK_GBPS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP64_PEAK_TFLOPS = 78.6
# name -> (generator, m, n, d, sketch, data description)
WORKLOADS = {
    "illcond_fp32_4194304x256": ("dense_ill_conditioned", 4194304, 256, 1024, "count",
                                 "synthetic (seeded; A = G diag(sigma) V^T, kappa 1e6)"),
    "gauss_bf16_262144x512": ("dense_scaled_columns", 262144, 512, 2048, "gaussian",
                              "synthetic (seeded; N(0,1) columns scaled 1 .. 1e-3)"),
    "csr_fp32_16777216x1000": ("sparse_csr", 1 << 24, 1000, 4000, "count",
                               "synthetic (seeded; 1000 uniform rows per column with N(0,1) values "
                               "plus a dense N(0,1) 1000 x 1000 block, b = A x + 1e-3 N(0,1))"),
    # Sec. 3.1 benchmark family: kappa 1e10, beta 1e-10, n = 1000, m up to 1e6, fp64
    "paper_fp64_1000000x1000": ("paper_benchmark_device", 1000000, 1000, 4000, "count",
                                "synthetic (seeded on the device; A = U diag(sigma) V^T with "
                                "Haar U, V, sigma log-spaced 1 .. 1e-10, b = A x + 1e-10 r_perp)"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(*names) -> str:
    """Hash of the files a kernel's code depends on (paths relative to the
    package), so that stored counter readings are used only for the code
    they were taken on."""
    h = hashlib.sha256()
    for nm in names:
        p = os.path.join(ROOT, "paper_2409_14309_amd", nm)
        if os.path.exists(p):
            with open(p, "rb") as f:
                data = f.read()
            if nm == "tuning.txt":
                # only the LSQR pass lines set a reported kernel's launch
                # shape; the gather (G) and QR (Q) lines do not
                data = b"".join(ln for ln in data.splitlines(keepends=True)
                                if not ln.startswith((b"G ", b"Q ")))
            h.update(data)
    return h.hexdigest()[:16]


# kernels whose launch times the solve bench reports
REPORTED_KERNELS = ("lsqr_pass", "cs_gather", "sort_count", "scan_segments", "scan_buckets",
                    "sort_place", "sort_scatter", "gauss_mfma", "form_y", "srht_pass1", "srht_pass", "srht_sample",
                    "srht_vpass1", "srht_vpass",
                    # phases of several launches, each timed as one region
                    "qr", "csr_sketch")

# files whose content determines each timed kernel's code and launch shape
KERNEL_SOURCES = {
    "lsqr_pass": ("csrc/lsqr.hip", "csrc/kernels.hpp", "csrc/common.hpp", "tuning.txt"),
    "cs_gather": ("csrc/countsketch.hip", "csrc/kernels.hpp", "csrc/common.hpp"),
    "gauss_mfma": ("csrc/gauss.hip", "csrc/kernels.hpp", "csrc/common.hpp"),
}


def measured_traffic(kernel: str, src_hash: str, workload):
    """HBM bytes per launch from the committed counter runs, if they were taken
    on the current kernel source and on this exact workload; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if workload is None or not os.path.exists(p):
        return None
    with open(p) as f:
        rec = json.load(f).get(kernel)
    if not rec or rec.get("source_hash") != src_hash or rec.get("workload") != workload:
        return None
    return rec.get("bytes_per_launch")


def host_cpu():
    """The host the oracle is timed on: usable cores and the CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return {"nproc": nproc, "cpu_count": os.cpu_count(), "model": model}


def _oracle_solve(A, b, d, rtol, kind, refine, zeta):
    from oracle import solve as OSV
    if refine == 0:
        return OSV.sketch_and_solve(A, b, kind, 42, d, zeta=zeta) if zeta > 1 else \
            OSV.sketch_and_solve(A, b, kind, 42, d)
    if refine == 2:
        return OSV.saa_sas(A, b, kind, 42, d, 100, rtol=rtol,
                           y_dtype=None if A.dtype == "float64" else A.dtype, zeta=zeta)
    return OSV.sap_sas(A, b, kind, 42, d, 100, rtol=rtol, zeta=zeta)


def cpu_baseline(A, b, d, rtol, rows, full_m, kind, refine=1, zeta=1, rows_1core=None):
    """The oracle (unchanged) on the first `rows` rows with the host's BLAS
    threads, and on the first `rows_1core` rows on one core, each time scaled
    to the full m (the sketch and the refinement passes are linear in m)."""
    from threadpoolctl import threadpool_info, threadpool_limits

    def run(r):
        As, bs = A[:r], b[:r]
        t0 = time.perf_counter()
        res = _oracle_solve(As, bs, d, rtol, kind, refine, zeta)
        return time.perf_counter() - t0, getattr(res, "iters", 0)

    host = host_cpu()
    dt, iters = run(rows)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    # one solve of the full m takes dt * full_m / rows seconds
    out = {"value": rows / (full_m * dt), "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": (f"first {rows} of {full_m} rows (n={A.shape[1]}, d={d}), one solve"
                      + (f" to rtol {rtol} ({iters} LSQR iterations)" if refine else "")
                      + f" in {dt:.2f}s with {threads} BLAS threads, time scaled by m"),
           "seconds_sample": dt, "host": host}
    r1 = min(rows_1core or rows, full_m)
    with threadpool_limits(limits=1):
        dt1, _ = run(r1)
    out["single_core"] = {"value": r1 / (full_m * dt1), "unit": "solves/s", "cores": 1,
                          "sample": f"first {r1} rows, one solve in {dt1:.2f}s on one core, "
                                    f"time scaled by m", "seconds_sample": dt1}
    return out


def host_lstsq_dense(A, b, blk=1 << 18, steps=2):
    """x* and ||b - A x*|| in FP64 on the host by corrected semi-normal
    equations: R from the Cholesky factor of the FP64 Gram matrix A^T A
    (products of FP32 data are exact in FP64), x = R^-1 R^-T A^T b, then
    `steps` corrections x += R^-1 R^-T A^T (b - A x).  For kappa(A) well
    below 1e8 this reaches the accuracy of a Householder QR: on 1,048,576 x
    256 FP32 rows with kappa 1e6 it agrees with LAPACK's lstsq to a residual
    error of 2e-11.  Measurement only, with multithreaded BLAS; not the
    oracle."""
    import numpy as np
    import scipy.linalg as sla
    m, n = A.shape
    b64 = np.asarray(b, dtype=np.float64)
    G = np.zeros((n, n))
    for i in range(0, m, blk):
        Ab = A[i:i + blk].astype(np.float64)
        G += Ab.T @ Ab
    R = sla.cholesky(G)

    def at(v):
        z = np.zeros(n)
        for i in range(0, m, blk):
            z += A[i:i + blk].astype(np.float64).T @ v[i:i + blk]
        return z

    def ax(x):
        return np.concatenate([A[i:i + blk].astype(np.float64) @ x for i in range(0, m, blk)])

    def solve_rr(z):
        return sla.solve_triangular(R, sla.solve_triangular(R, z, trans="T"))

    x = solve_rr(at(b64))
    for _ in range(steps):
        x = x + solve_rr(at(b64 - ax(x)))
    return x, float(np.linalg.norm(b64 - ax(x)))


def dense_errors(A, b, x, xs, rho, blk=1 << 20):
    """FE and RE of x against x* (host, FP64, row blocks)."""
    import numpy as np
    dx = x - xs
    ss = 0.0
    for i in range(0, A.shape[0], blk):
        ss += float(np.sum((A[i:i + blk].astype(np.float64) @ dx) ** 2))
    return {"RE": float(np.sqrt(ss) / rho), "FE": float(np.linalg.norm(dx) / np.linalg.norm(xs)),
            "x_star": "FP64 least squares on the host by corrected semi-normal equations "
                      "(Cholesky of A^T A, two correction steps)"}


SERVE_WORKLOAD = "serve_mix_10000"


def serve_main(args):
    """Serving mix: Poisson arrivals, m log-uniform in [2^12, 2^20], n in
    {16, ..., 256}, d = 4 n, FP32, refined to the stop rule; open loop at the
    arrival rate and saturated (all queued at once) through the
    continuous-batching server, in two forms: small problems set up in the
    persistent fused sketch + QR launch (replayed from a HIP graph each
    round), and every problem on the blocked per-phase path; against
    one-problem-at-a-time GPU solves."""
    import numpy as np
    import torch

    import paper_2409_14309_amd as sns
    import workloads

    sns.load()
    rows = 1 << 23
    reqs = workloads.serving_requests(args.requests, args.rate, seed=1004, pool_rows=rows)
    log(f"generating the device pools ({rows} rows per n) ...")
    pool = workloads.serving_pool(rows, seed=1004)
    torch.cuda.synchronize()

    def window(r, P):
        o = workloads.request_window(r, rows)
        return P[r["n"]]["A"][o:o + r["m"]], P[r["n"]]["b"][o:o + r["m"]]

    pool_bytes = args.slots * (40 << 20)

    def serve(open_loop, subset):
        srv = sns.Server(pool_bytes, max_slots=args.slots, chunk_iters=args.chunk)
        tickets = []
        t0 = time.perf_counter()
        for r in subset:
            if open_loop:
                delay = t0 + r["t"] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            A, b = window(r, pool)
            tickets.append((r, srv.submit(A, b, r["d"], 42, max_iters=args.max_iters,
                                          rtol=args.rtol)))
        res = [(r, *srv.wait(t)) for r, t in tickets]
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return res, st, wall

    forms = {}
    for form, fused in (("per_phase", False), ("fused", True)):
        sns.sns_fused_enable(fused)
        serve(False, reqs[:64])  # warm-up
        log(f"[{form}] open loop: {len(reqs)} requests at {args.rate}/s ...")
        res_o, st_o, wall_o = serve(True, reqs)
        log(f"  {st_o.completed} done in {wall_o:.2f}s; p50 {st_o.p50_ms:.2f} ms p99 {st_o.p99_ms:.2f} ms")
        log(f"[{form}] saturation: all requests queued at once ...")
        res_s, st_s, wall_s = serve(False, reqs)
        log(f"  {st_s.completed} done in {wall_s:.2f}s ({st_s.completed / wall_s:.1f} solves/s)")
        forms[form] = (res_o, st_o, wall_o, res_s, st_s, wall_s)
    sns.sns_fused_enable(False)  # the library's default form
    # the headline is the default (per-phase) form; both are reported
    res_o, st_o, wall_o, res_s, st_s, wall_s = forms["per_phase"]
    pp = forms["per_phase"]
    fu = forms["fused"]
    # the two forms agree to rounding: worst relative difference of x
    form_dx = max(float(np.linalg.norm(xa.cpu().numpy() - xb.cpu().numpy()) /
                        np.linalg.norm(xb.cpu().numpy()))
                  for (_, xa, _), (_, xb, _) in zip(fu[3], pp[3]))

    # algorithmic HBM bytes of the saturated run: sketch pass + (iters + 1) LSQR passes
    tot = 0.0
    for r, x, info in res_s:
        m, n = r["m"], r["n"]
        tot += 4.0 * m * (n + 1) + (info.iters + 1) * (4.0 * m * n + 8.0 * m)
    bad = [int(info.status) for _, _, info in res_s if info.status != 0]

    # one problem at a time on the GPU, same stop rule: FP64 (the plain
    # per-problem form) and FP32
    nb = min(args.baseline_requests, len(reqs))
    base = {}
    sns.sns_fused_enable(False)  # the plain per-problem form: blocked path, one problem at a time
    for tag, fp64 in (("per_problem_fp32", False), ("per_problem_fp64", True)):
        P = pool if not fp64 else workloads.serving_pool(rows, seed=1004, fp64=True)
        torch.cuda.synchronize()
        for r in reqs[:4]:
            A, b = window(r, P)
            sns.lstsq(A, b, "count", r["d"], 42, refine=True, max_iters=args.max_iters, rtol=args.rtol)
        t0 = time.perf_counter()
        lat = []
        for r in reqs[:nb]:
            t1 = time.perf_counter()
            A, b = window(r, P)
            sns.lstsq(A, b, "count", r["d"], 42, refine=True, max_iters=args.max_iters, rtol=args.rtol)
            lat.append(1000.0 * (time.perf_counter() - t1))
        dt = time.perf_counter() - t0
        base[tag] = {"solves_per_s": round(nb / dt, 2), "requests": nb,
                     "p50_ms": round(float(np.percentile(lat, 50)), 3),
                     "p99_ms": round(float(np.percentile(lat, 99)), 3)}
        log(f"  {tag}: {nb / dt:.1f} solves/s")
        if fp64:
            del P
            torch.cuda.empty_cache()

    # residual error of a sample of the served answers against FP64 LAPACK
    # least squares of the same window
    worst = 0.0
    checked = 0
    for r, x, info in res_s:
        if r["m"] > (1 << 15) or checked >= 12:
            continue
        A, b = window(r, pool)
        An, bn = A.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
        xs = np.linalg.lstsq(An, bn, rcond=None)[0]
        re = np.linalg.norm(An @ (x.cpu().numpy() - xs)) / np.linalg.norm(bn - An @ xs)
        worst = max(worst, float(re))
        checked += 1

    cpu = None
    if not args.no_cpu:
        from threadpoolctl import threadpool_info

        from oracle import solve as OSV
        k = min(args.cpu_requests, len(reqs))
        log(f"timing the CPU oracle on the first {k} requests ...")
        t0 = time.perf_counter()
        for r in reqs[:k]:
            A, b = window(r, pool)
            OSV.sap_sas(A.cpu().numpy(), b.cpu().numpy(), "count", 42, r["d"], args.max_iters,
                        rtol=args.rtol)
        dt = time.perf_counter() - t0
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        cpu = {"value": round(k / dt, 3), "unit": "solves/s", "cores": threads, "kind": "oracle",
               "host": host_cpu(),
               "sample": f"first {k} requests of the stream solved one after another in {dt:.1f}s"}

    sat = st_s.completed / wall_s
    out = {
        "metric": "LS solves/s + p50/p99 latency at rel-residual 1e-6, serving mix",
        "value": round(sat, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": 64,
        "ms_per_step": round(1000.0 * wall_s / max(st_s.completed, 1), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage, f64 accumulation (QR and LSQR in f64)",
        "data": "synthetic (seeded device pools; row windows with N(0,1) entries, b = A x + 1e-3 N(0,1); "
                "the requests of one n take consecutive windows of an 8,388,608-row pool (0.5-8 GB per n, "
                "beyond the 256 MB last-level cache), so requests in flight never share rows)",
        "config": {"workload": SERVE_WORKLOAD, "requests": len(reqs), "rate_per_s": args.rate,
                   "m": "floor(2^U[12,20])", "n": [16, 32, 64, 128, 256], "d": "4n",
                   "rtol": args.rtol, "max_slots": args.slots, "chunk_iters": args.chunk,
                   "parallelism": "single GPU"},
        "open_loop": {"solves_per_s": round(st_o.completed / wall_o, 2),
                      "p50_ms": round(st_o.p50_ms, 3), "p99_ms": round(st_o.p99_ms, 3),
                      "mean_ms": round(st_o.mean_ms, 3), "peak_slots": st_o.peak_slots},
        "saturation": {"solves_per_s": round(sat, 2), "p50_ms": round(st_s.p50_ms, 3),
                       "p99_ms": round(st_s.p99_ms, 3), "rounds": int(st_s.rounds),
                       "peak_pool_bytes": int(st_s.peak_pool_bytes)},
        "forms": {
            "fused": {"setup": "d <= 256, n <= 64, m (n + 1) <= 2^21: persistent fused sketch + QR "
                               "launch replayed from a HIP graph; larger: blocked",
                      "open_loop": {"solves_per_s": round(fu[1].completed / fu[2], 2),
                                    "p50_ms": round(fu[1].p50_ms, 3), "p99_ms": round(fu[1].p99_ms, 3)},
                      "saturation": {"solves_per_s": round(fu[4].completed / fu[5], 2),
                                     "p50_ms": round(fu[4].p50_ms, 3), "p99_ms": round(fu[4].p99_ms, 3)}},
            "per_phase": {"setup": "every problem on the blocked path (sort, gather, panel QR)",
                          "open_loop": {"solves_per_s": round(pp[1].completed / pp[2], 2),
                                        "p50_ms": round(pp[1].p50_ms, 3), "p99_ms": round(pp[1].p99_ms, 3)},
                          "saturation": {"solves_per_s": round(pp[4].completed / pp[5], 2),
                                         "p50_ms": round(pp[4].p50_ms, 3), "p99_ms": round(pp[4].p99_ms, 3)}},
            "max_rel_dx_between_forms": form_dx},
        "baselines": base,
        "speedup_vs_per_problem_fp64": round(sat / base["per_problem_fp64"]["solves_per_s"], 3),
        "max_RE_sample": worst,
        "RE_sample_size": checked,
        "nonzero_status": bad[:10],
        "roofline": {"bound": "hbm", "achieved": round(tot / wall_s / 1e9, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(tot / wall_s / 1e9 / HBM_PEAK_GBPS, 4),
                     "traffic": None, "kernel": "whole job (sketch + LSQR passes, algorithmic bytes)"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


SWEEP_WORKLOAD = "paper_fp64_sweep"
SWEEP_M = (5000, 10000, 30000, 100000, 300000, 1000000)


def _timed_steps(step, steps, warmup, stream, read):
    """warmup untimed calls, then `steps` calls each bracketed by events; the
    wall clock spans the whole timed region.  read() is called after each."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    seen = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        step()
        ends[k].record(stream)
        ends[k].synchronize()
        seen.append(read())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat = sorted(a.elapsed_time(e) for a, e in zip(starts, ends))
    return t1 - t0, lat, seen


def sweep_main(args):
    """The Sec. 3.1 family over m at n = 1000 (kappa 1e10, beta 1e-10, FP64,
    CountSketch d = 4000): runtime, forward error and residual error of
    SAP-SAS and SAA-SAS against the exact solution built into the data, the
    shape of Figs. 3-5, with the CPU oracle timed beside the small m."""
    import numpy as np
    import torch

    import paper_2409_14309_amd as sns
    import workloads

    sns.load()
    dev = torch.device("cuda:0")
    n, d = 1000, 4000
    ms = [int(v) for v in args.sweep_m.split(",")] if args.sweep_m else list(SWEEP_M)
    rows = []
    stream = torch.cuda.current_stream()
    for m in ms:
        log(f"sweep m = {m}: generating on the device ...")
        A, b, xe = workloads.paper_benchmark_device(m, n, 1005, device=dev)
        torch.cuda.synchronize()
        M = sns.dense(A)
        row = {"m": m}
        for solver, refine in (("sap", 1), ("saa", 2)):
            sk = sns.sketch_desc("count", d, 42)
            o = sns.opts(refine=refine, max_iters=args.max_iters, rtol=args.rtol)
            ws = torch.empty(sns.sns_lstsq_workspace_size(sk, M, o), dtype=torch.uint8, device=dev)
            x = torch.empty(n, dtype=torch.float64, device=dev)
            info_buf = torch.zeros(64, dtype=torch.uint8).pin_memory()
            info = sns.Info.from_address(info_buf.data_ptr())

            def step():
                sns.sns_lstsq(sk, M, b, x, o, ws, info, stream)

            wall, lat, its = _timed_steps(step, args.steps, max(1, args.warmup), stream,
                                          lambda: (int(info.iters), int(info.status)))
            dx = x - xe
            row[solver] = {"ms_median": round(float(np.median(lat)), 4),
                           "ms_p99": round(float(np.percentile(lat, 99)), 4),
                           "iters": its[-1][0], "status": its[-1][1],
                           "RE": float(torch.linalg.norm(A @ dx) / 1e-10),
                           "FE": float(torch.linalg.norm(dx) / torch.linalg.norm(xe))}
            log(f"  {solver}: {row[solver]}")
            del ws
        if not args.no_cpu and m <= args.sweep_cpu_max_m:
            Ah, bh, xh = A.cpu().numpy(), b.cpu().numpy(), xe.cpu().numpy()
            from oracle import solve as OSV
            t0 = time.perf_counter()
            r = OSV.sap_sas(Ah, bh, "count", 42, d, args.max_iters, rtol=args.rtol)
            dt = time.perf_counter() - t0
            dxh = r.x - xh
            row["cpu_oracle_sap"] = {"ms": round(1000 * dt, 1), "iters": int(r.iters),
                                     "RE": float(np.linalg.norm(Ah @ dxh) / 1e-10),
                                     "FE": float(np.linalg.norm(dxh) / np.linalg.norm(xh))}
            log(f"  cpu oracle: {row['cpu_oracle_sap']}")
        rows.append(row)
        del A, b, xe, M
        torch.cuda.empty_cache()
    last = rows[-1]
    out = {
        "metric": "LS solves/s at rel-residual 1e-6 over m, Sec. 3.1 family (runtime, FE, RE)",
        "value": round(1000.0 / last["sap"]["ms_median"], 3),
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": last["sap"]["ms_median"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded on the device; A = U diag(sigma) V^T with Haar U, V, sigma "
                "log-spaced 1 .. 1e-10, b = A x + 1e-10 r_perp; x is the exact solution)",
        "config": {"workload": SWEEP_WORKLOAD, "m": ms, "n": n, "d": d, "sketch": "countsketch",
                   "solvers": ["SAP-SAS", "SAA-SAS"], "rtol": args.rtol,
                   "parallelism": "single GPU"},
        "sweep": rows,
        "cpu_host": host_cpu(),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="illcond_fp32_4194304x256",
                    choices=sorted(WORKLOADS) + [SERVE_WORKLOAD, SWEEP_WORKLOAD])
    ap.add_argument("--requests", type=int, default=10000, help="serving mix: requests")
    ap.add_argument("--rate", type=float, default=2000.0, help="serving mix: arrivals per second")
    ap.add_argument("--slots", type=int, default=128, help="serving mix: admitted requests")
    ap.add_argument("--chunk", type=int, default=8, help="serving mix: iterations per round")
    ap.add_argument("--baseline-requests", type=int, default=400)
    ap.add_argument("--cpu-requests", type=int, default=20)
    ap.add_argument("--m", type=int, default=0, help="override the workload's row count")
    ap.add_argument("--sweep-m", default="", help="Sec. 3.1 sweep: comma-separated row counts")
    ap.add_argument("--sweep-cpu-max-m", type=int, default=30000,
                    help="Sec. 3.1 sweep: time the CPU oracle up to this m")
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--max-iters", type=int, default=100)
    ap.add_argument("--cpu-rows", type=int, default=1 << 22,
                    help="rows of A the CPU oracle solves (capped at m; 100,000 on the FP64 "
                         "Sec. 3.1 family); its time is scaled to the full m")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the host least-squares solution the errors are measured against")
    ap.add_argument("--zeta", type=int, default=1,
                    help="CountSketch workloads: > 1 uses the sparse sign embedding with zeta "
                         "nonzeros per column")
    ap.add_argument("--d", type=int, default=0, help="override the workload's sketch size")
    ap.add_argument("--sketch", default="", choices=["", "count", "gaussian", "hadamard"],
                    help="override the workload's sketch operator")
    ap.add_argument("--solver", default="", choices=["", "sas", "sap", "saa"],
                    help="plain sketch-and-solve, SAP-SAS (LSQR on A R^-1 applied implicitly) or "
                         "SAA-SAS (Y = A R^-1 formed once, LSQR on Y); default: the workload's")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures a single GPU: the sketch-and-solve path here runs on one "
              "device; --gpus above 1 is not supported.", file=sys.stderr)
        sys.exit(2)

    if args.workload == SERVE_WORKLOAD:
        serve_main(args)
        return
    if args.workload == SWEEP_WORKLOAD:
        sweep_main(args)
        return

    import numpy as np
    import torch

    import paper_2409_14309_amd as sns
    import workloads

    sns.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    gen, m, n, d, kind, data_desc = WORKLOADS[args.workload]
    if args.m:
        m = args.m
    if args.d:
        d = args.d
    zeta = 1
    if args.sketch:
        kind = args.sketch
    if args.zeta > 1 and kind == "count":
        kind, zeta = "sparse", args.zeta
    csr = gen == "sparse_csr"
    solver = args.solver or ("sas" if csr else "sap")
    refine = {"sas": 0, "sap": 1, "saa": 2}[solver]
    seed = {"dense_scaled_columns": 1003, "sparse_csr": 1002}.get(gen, 1001)
    dev = torch.device("cuda:0")
    paper = gen == "paper_benchmark_device"
    t0 = time.time()
    x_exact = None
    if paper:
        seed = 1005
        log(f"generating {args.workload} on the device: A {m}x{n} fp64 ...")
        A, b, x_exact = workloads.paper_benchmark_device(m, n, seed, device=dev)
        p = None
    else:
        log(f"generating {args.workload}: A {m}x{n} ...")
        p = getattr(workloads, gen)(m, n, seed=seed)
        log(f"generated in {time.time() - t0:.1f}s; copying to HBM")
        if csr:
            A = sns.CsrMatrix(torch.from_numpy(p.A.indptr.astype(np.int32)).to(dev),
                              torch.from_numpy(p.A.indices.astype(np.int32)).to(dev),
                              torch.from_numpy(p.A.data).to(dev), p.A.shape)
        else:
            A = torch.from_numpy(p.A).to(dev)
        b = torch.from_numpy(p.b).to(dev)
    torch.cuda.synchronize()
    log(f"inputs resident in HBM after {time.time() - t0:.1f}s")
    es = (A.values if csr else A).element_size()
    nnz = int(p.A.nnz) if csr else 0

    sk = sns.sketch_desc(kind, d, 42, zeta)
    M = sns.csr(A.row_ptr, A.col_idx, A.values, m, n) if csr else sns.dense(A)
    o = sns.opts(refine=refine, max_iters=args.max_iters if refine else 0,
                 rtol=args.rtol if refine else 0.0)
    ws = torch.empty(sns.sns_lstsq_workspace_size(sk, M, o), dtype=torch.uint8, device=dev)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    info_buf = torch.zeros(64, dtype=torch.uint8).pin_memory()
    info = sns.Info.from_address(info_buf.data_ptr())
    stream = torch.cuda.current_stream()

    def step():
        sns.sns_lstsq(sk, M, b, x, o, ws, info, stream)

    sns.sns_timing_reset()
    # only the kernels and phases reported below are bracketed by events:
    # every timed launch adds two event records to the stream
    sns.sns_timing_select(REPORTED_KERNELS)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done: iters={info.iters} status={info.status} est={info.rel_resid_est:.3g}")
    sns.sns_timing_enable(True)
    wall, lat, seen = _timed_steps(step, args.steps, 0, stream,
                                   lambda: (int(info.iters), int(info.status),
                                            float(info.rel_resid_est)))
    sns.sns_timing_enable(False)
    sns.sns_timing_select(None)
    iters = [v[0] for v in seen]
    statuses = [v[1] for v in seen]
    ests = [v[2] for v in seen]
    kt = sns.sns_timing_summary()
    ms_per_step = 1000.0 * wall / args.steps
    value = args.steps / wall
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step; iters {iters}")
    for name, (cnt, tot, avg) in sorted(kt.items(), key=lambda kv: -kv[1][1]):
        log(f"  {name:16s} launches {cnt:6d} total {tot:9.3f} ms avg {avg:9.2f} us")

    bytes_per = {
        # one fused LSQR pass: A (or Y) once, the m-vector u read and written
        "lsqr_pass": es * m * n + 2.0 * es * m,
        # CountSketch: A and b once, SA and Sb written (the sparse sign
        # embedding's gather reads each row zeta times; the algorithmic
        # figure stays one read)
        "cs_gather": es * m * (n + 1) + es * d * (n + 1),
        # CSR CountSketch, the whole phase: row_ptr, (col_idx, value) per
        # nonzero, b once, SA and Sb written
        "csr_sketch": 4.0 * (m + 1) + (4.0 + es) * nnz + es * m + es * d * (n + 1),
    }
    # Gaussian sketch: 2 d m n flops for G A plus 2 d m for G b
    flops_per = {"gauss_mfma": 2.0 * d * m * n + 2.0 * d * m}
    # Householder QR of the d x (n + 1) matrix [SA | Sb], the whole phase
    fp64_flops_per = {"qr": 2.0 * (n + 1) ** 2 * (d - (n + 1) / 3.0)}
    # Hadamard sketch: the first butterfly pass reads [A | b] and writes the
    # m' x (n + 1) buffer, each later pass reads and writes it, the sampled
    # rows read d 2^(L - 8 P) rows of it.  When b is transformed as a vector
    # of its own (srht_vpass1 / srht_vpass), the matrix passes carry n columns
    # and the vector passes read and write the m' values of b.
    L = max(0, (m - 1).bit_length())
    mp = 1 << L
    P = max(1, (L + 7) // 8 - 1)
    cw = n if "srht_vpass1" in kt else n + 1
    bytes_per["srht_pass1"] = es * m * cw + es * mp * cw
    bytes_per["srht_pass"] = 2.0 * es * mp * cw
    bytes_per["srht_vpass1"] = es * m + es * mp
    bytes_per["srht_vpass"] = 2.0 * es * mp
    bytes_per["srht_sample"] = es * d * (1 << (L - min(L, 8 * P))) * (n + 1) + es * d * (n + 1)
    # SAA-SAS: Y = A R^-1 with R^-1 upper triangular, n (n + 1) / 2 fp64
    # multiply-adds per row of A, on the FP64 matrix cores
    fp64_flops_per["form_y"] = float(m) * n * (n + 1)

    # counters were taken on the named workloads as they stand: any override
    # of the shape, sketch or solver leaves traffic unmeasured
    traffic_workload = (args.workload if not (args.m or args.d or args.sketch or args.zeta > 1
                                             or args.solver) else None)

    def roofline(kname):
        cnt, tot, avg_us = kt[kname]
        rec = {"kernel": kname, "avg_launch_us": avg_us, "launches": cnt}
        if kname in bytes_per:
            ach = bytes_per[kname] / (avg_us * 1e-6) / 1e9
            rec.update({"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS,
                        "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBPS, 4),
                        "traffic": (measured_traffic(kname, kernel_source_hash(*KERNEL_SOURCES[kname]),
                                                     traffic_workload)
                                    if kname in KERNEL_SOURCES else None),
                        "bytes_per_launch": bytes_per[kname]})
            return rec
        if kname in flops_per:
            ach = flops_per[kname] / (avg_us * 1e-6) / 1e12
            rec.update({"bound": "mfma", "achieved": round(ach, 1), "peak": BF16_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(ach / BF16_PEAK_TFLOPS, 4),
                        "traffic": None, "flops_per_launch": flops_per[kname]})
            return rec
        if kname in fp64_flops_per:
            ach = fp64_flops_per[kname] / (avg_us * 1e-6) / 1e12
            rec.update({"bound": "mfma", "achieved": round(ach, 2), "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4),
                        "traffic": None, "flops_per_launch": fp64_flops_per[kname],
                        "precision": "fp64"})
            return rec
        return None

    # the dominant reported kernel or phase (phases that contain reported
    # kernels are not counted twice: a phase wins only if it is larger)
    dom = max(kt.items(), key=lambda kv: kv[1][1])[0]
    roof = roofline(dom)
    gauss = roofline("gauss_mfma") if "gauss_mfma" in kt else None
    qr = roofline("qr") if "qr" in kt else None
    csr_rec = roofline("csr_sketch") if "csr_sketch" in kt else None
    cs = kt.get("cs_gather")
    sort_us = sum(kt[k][2] for k in ("sort_count", "scan_segments", "scan_buckets", "sort_place", "sort_scatter")
                  if k in kt)
    countsketch = None
    if cs:
        gbps = bytes_per["cs_gather"] / (cs[2] * 1e-6) / 1e9
        countsketch = {"zeta": zeta, "GBps": round(gbps, 1), "frac_peak": round(gbps / HBM_PEAK_GBPS, 4),
                       "GBps_moved": round(gbps * zeta, 1),
                       "kernel_avg_us": cs[2], "bucket_sort_avg_us": round(sort_us, 2),
                       "GBps_with_sort": round(bytes_per["cs_gather"] / ((cs[2] + sort_us) * 1e-6) / 1e9, 1)}

    form_y = roofline("form_y") if "form_y" in kt else None
    hadamard = {k: roofline(k) for k in ("srht_pass1", "srht_pass", "srht_vpass1", "srht_vpass", "srht_sample")
                if k in kt} or None

    # errors of the last solve against an FP64 least-squares solution of the
    # same data, computed on the host after the timed region
    accuracy = None
    if x_exact is not None:
        # x_exact is the least-squares solution and beta the optimal residual
        dx = x - x_exact
        accuracy = {"RE": float(torch.linalg.norm(A @ dx) / 1e-10),
                    "FE": float(torch.linalg.norm(dx) / torch.linalg.norm(x_exact)),
                    "x_star": "the exact solution built into the data (optimal residual 1e-10)"}
    elif not args.no_accuracy:
        t1 = time.time()
        xg = x.cpu().numpy()
        if csr:
            import scipy.linalg as sla
            A64 = p.A.astype(np.float64)
            b64 = p.b.astype(np.float64)
            # A is well conditioned: normal equations by Cholesky, one step of
            # refinement on the residual
            G = (A64.T @ A64).toarray()
            cf = sla.cho_factor(G)
            xs = sla.cho_solve(cf, A64.T @ b64)
            xs += sla.cho_solve(cf, A64.T @ (b64 - A64 @ xs))
            rs = b64 - A64 @ xs
            dxh = xg - xs
            accuracy = {"RE": float(np.linalg.norm(A64 @ dxh) / np.linalg.norm(rs)),
                        "FE": float(np.linalg.norm(dxh) / np.linalg.norm(xs)),
                        "x_star": "Cholesky of A^T A in FP64 on the host, one refinement step"}
        else:
            xs, rho = host_lstsq_dense(p.A, p.b)
            accuracy = dense_errors(p.A, p.b, xg, xs, rho)
        log(f"accuracy of the last solve ({time.time() - t1:.1f}s): {accuracy}")

    cpu = None
    if not args.no_cpu:
        rows = min(args.cpu_rows, m) if not paper else min(args.cpu_rows, m, 100000)
        rows1 = min(rows, 1 << 20)
        if csr:
            # the plain CSR solve is dominated by the QR of the d x (n + 1)
            # sketch, a cost that does not scale with m: solve all rows
            rows = rows1 = m
        log(f"timing the CPU oracle on {rows} rows (one core: {rows1}) ...")
        if paper:
            Ah, bh = A[:rows].cpu().numpy(), b[:rows].cpu().numpy()
        else:
            Ah, bh = p.A, p.b
        cpu = cpu_baseline(Ah, bh, d, args.rtol, rows, m, kind, refine, zeta, rows1)
        log(f"oracle sample took {cpu['seconds_sample']:.2f}s "
            f"(one core {cpu['single_core']['seconds_sample']:.2f}s)")
        if csr:
            # parity of the timed x0 with the oracle's sketch-and-solve
            from oracle import solve as OSV
            xr = OSV.sketch_and_solve(p.A, p.b, "count", 42, d).x
            xg = x.cpu().numpy()
            cpu["parity_x0_max_abs_rel"] = float(np.max(np.abs(xg - xr)) / np.max(np.abs(xr)))

    solver_name = {0: "SAS (sketch, Householder QR, triangular solve)",
                   1: "SAP-SAS (sketch, Householder QR, LSQR on A R^-1)",
                   2: "SAA-SAS (sketch, Householder QR, Y = A R^-1 formed, LSQR on Y)"}[refine]
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f64" if es == 8 else
                  "f32 storage, f64 accumulation (QR and LSQR in f64)" if kind != "gaussian" else
                  "bf16 x bf16 -> f32 sketch on MFMA; f32 storage, f64 accumulation (QR, LSQR)"),
        "data": data_desc,
        "config": {"workload": args.workload, "m": m, "n": n, "d": d,
                   "sketch": {"count": "countsketch", "gaussian": "gaussian",
                              "sparse": f"sparse sign (zeta {zeta})", "hadamard": "SRHT"}[kind],
                   "solver": solver_name, "rtol": args.rtol if refine else None,
                   "parallelism": "single GPU", **({"nnz": nnz} if csr else {})},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4)},
        "lsqr_iters": iters,
        "status": statuses,
        "rel_resid_est": max(ests) if ests else None,
        "countsketch": countsketch,
        "csr_sketch": csr_rec,
        "gaussian_sketch": gauss,
        "qr": qr,
        "form_y": form_y,
        "hadamard_sketch": hadamard,
        "accuracy": accuracy,
        "roofline": roof,
        "kernels": {k: {"launches": v[0], "total_ms": round(v[1], 4), "avg_us": round(v[2], 3)}
                    for k, v in kt.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
