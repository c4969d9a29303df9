// Shared host logic of the solve entry points and the server: argument
// checks, workspace layout of one problem, and the launch sequences built
// from it.
#include <math.h>
#include <string.h>

#include "common.hpp"
#include "kernels.hpp"
#include "solve.hpp"

namespace sns {

sns_status check_matrix(const sns_matrix* A) {
  if (!A) return SNS_ERR_INVALID_ARG;
  // a CSR matrix without nonzeros may leave values and col_idx NULL
  const bool empty_csr = A->layout == SNS_CSR && A->nnz == 0;
  if (!A->values && !empty_csr) return SNS_ERR_INVALID_ARG;
  if (A->dtype != SNS_F32 && A->dtype != SNS_F64) return SNS_ERR_DTYPE;
  if (A->layout != SNS_DENSE_ROWMAJOR && A->layout != SNS_CSR) return SNS_ERR_DTYPE;
  if (A->m < 1 || A->n < 1 || A->m > kMaxRows) return SNS_ERR_SHAPE;
  if (A->layout == SNS_DENSE_ROWMAJOR && A->ld < A->n) return SNS_ERR_SHAPE;
  if (A->layout == SNS_CSR) {
    if (!A->row_ptr || (!A->col_idx && !empty_csr)) return SNS_ERR_INVALID_ARG;
    if (A->nnz < 0 || A->nnz > kMaxRows - 128) return SNS_ERR_SHAPE;
  }
  return SNS_OK;
}

sns_status check_sketch(const sns_sketch* sk, const sns_matrix* A) {
  if (!sk) return SNS_ERR_INVALID_ARG;
  if (sk->kind != SNS_SKETCH_COUNT && sk->kind != SNS_SKETCH_GAUSSIAN &&
      sk->kind != SNS_SKETCH_SPARSE_SIGN && sk->kind != SNS_SKETCH_HADAMARD)
    return SNS_ERR_INVALID_ARG;
  if (sk->d < 1 || sk->d > kMaxD) return SNS_ERR_SHAPE;
  if (sk->kind == SNS_SKETCH_SPARSE_SIGN && (sk->zeta < 1 || sk->zeta > 64))
    return SNS_ERR_INVALID_ARG;
  if (A) {
    if (sk->kind == SNS_SKETCH_SPARSE_SIGN && A->layout != SNS_DENSE_ROWMAJOR) return SNS_ERR_DTYPE;
    if (sk->kind == SNS_SKETCH_HADAMARD && A->layout != SNS_DENSE_ROWMAJOR) return SNS_ERR_DTYPE;
    if (sk->kind == SNS_SKETCH_HADAMARD && A->m > kMaxHadRows) return SNS_ERR_SHAPE;
    if (sk->kind == SNS_SKETCH_SPARSE_SIGN && (int64_t)sk->zeta * A->m > kMaxRows)
      return SNS_ERR_SHAPE;
    if (sk->d < A->n || sk->d > A->m) return SNS_ERR_SHAPE;
    if (sk->kind == SNS_SKETCH_GAUSSIAN && A->dtype != SNS_F32) return SNS_ERR_DTYPE;
    if (sk->kind == SNS_SKETCH_GAUSSIAN && A->layout != SNS_DENSE_ROWMAJOR) return SNS_ERR_DTYPE;
    if (sk->kind == SNS_SKETCH_COUNT && A->layout == SNS_CSR && A->n > kMaxCsrN) return SNS_ERR_SHAPE;
  }
  return SNS_OK;
}

void carve_sketch(Carve& c, const sns_sketch& sk, const sns_matrix& A, bool with_b, bool acc64,
                  SketchWs& w) {
  const uint32_t zeta = sketch_zeta(sk);
  w.sp = make_sort_plan(A.m * zeta, (uint32_t)sk.d, zeta);
  w.gp = make_gather_plan(A, (uint32_t)sk.d, acc64, A.m * zeta);
  carve_sort(c, w.sp, with_b ? elem(A) : 0, w.sb);
  const size_t pb = gather_partial_bytes(w.gp, A, (uint32_t)sk.d);
  w.part = pb ? (void*)c.take<char>(pb) : nullptr;
}

void add_sketch_jobs(ArgTable& t, Jobs& J, const sns_sketch& sk, const sns_matrix& A,
                     const void* b, void* SA, void* Sb, const SketchWs& w) {
  const std::vector<SortArgs> sa{sort_args(w.sp, sk.seed, b, w.sb)};
  J.sort = build_sort_job(t, sa, A.dtype == SNS_F64);
  GatherProb g;
  g.plan = w.gp;
  g.args = gather_args(w.gp, A, (uint32_t)sk.d, w.sb, b != nullptr, SA, Sb, w.part);
  g.dtype = A.dtype;
  J.gather = build_gather_job(t, std::vector<GatherProb>{g});
}

sns_status run_sketch_jobs(const Jobs& J, hipStream_t st) {
  sns_status s = launch_sort_job(J.sort, st);
  if (s != SNS_OK) return s;
  return launch_gather_job(J.gather, st);
}

void carve_lstsq_bufs(Carve& c, const sns_sketch& sk, const sns_matrix& A,
                      const sns_solve_opts& o, LstsqWs& w) {
  if (sk.kind == SNS_SKETCH_HADAMARD) {
    w.gauss = c.take<char>(hadamard_workspace_bytes(A, (uint32_t)sk.d));
  } else if (sk.kind == SNS_SKETCH_GAUSSIAN) {
    w.gauss = c.take<char>(gauss_workspace_bytes(A, (uint32_t)sk.d));
  } else if (A.layout == SNS_CSR) {
    w.csr_bytes = csr_workspace_bytes(A, (uint32_t)sk.d, o.accum_fp64 != 0);
    w.csr = c.take<char>(w.csr_bytes);
  } else if (fused_eligible(sk, A)) {
    w.fused = true;
    w.fp = make_fused_plan(sk, A);
    carve_fused(c, w.fp, w.fb);
  } else {
    carve_sketch(c, sk, A, true, o.accum_fp64 != 0, w.sw);
  }
  w.SA = c.take<char>((size_t)sk.d * A.n * elem(A));
  w.Sb = c.take<char>((size_t)sk.d * elem(A));
  carve_qr(c, sk.d, A.n, w.q);
  if (o.refine) {
    w.lp = make_lsqr_plan(A);
    carve_lsqr(c, A, w.lp, w.l);
  }
  if (o.refine == 2) {
    w.ldy = saa_ldy(A);
    w.Y = c.take<char>((size_t)A.m * w.ldy * elem(A));
  }
  w.info = c.take<sns_info>(1);
}

void build_lstsq_jobs(ArgTable& t, Jobs& J, const sns_sketch& sk, const sns_matrix& A,
                      const void* b, double* x, const sns_solve_opts& o, const LstsqWs& w) {
  if (w.fused) {
    J.fused = build_fused_job(
        t, std::vector<FusedArgs>{fused_args(w.fp, sk, A, b, w.fb, w.q, w.q.xw, w.info)},
        A.dtype == SNS_F64);
  } else {
    if ((sk.kind == SNS_SKETCH_COUNT || sk.kind == SNS_SKETCH_SPARSE_SIGN) &&
        A.layout == SNS_DENSE_ROWMAJOR)
      add_sketch_jobs(t, J, sk, A, b, w.SA, w.Sb, w.sw);
    const std::vector<QrArgs> qa{
        qr_args(sk.d, A.n, w.SA, A.n, w.Sb, w.q, w.q.xw, nullptr, w.info)};
    J.qr = build_qr_job(t, qa, A.dtype == SNS_F64);
  }
  if (o.refine) {
    LsqrProb lp;
    lp.plan = w.lp;
    lp.args = lsqr_args(A, b, w.lp, w.l, w.q, (int)sk.d, o.max_iters, o.rtol, x, w.info,
                        o.refine == 2 ? w.Y : nullptr, w.ldy);
    J.lsqr = build_lsqr_job(t, std::vector<LsqrProb>{lp}, A.dtype == SNS_F64);
    if (o.refine == 2) {
      SaaJob& y = J.lsqr.saa;
      y.A = A.values;
      y.ld = A.ld;
      y.m = A.m;
      y.n = (int)A.n;
      y.X = w.l.Xr;
      y.Y = w.Y;
      y.ldy = w.ldy;
      y.f64 = A.dtype == SNS_F64;
    }
  }
}

// Full workspace layout of sns_lstsq: buffers, then the argument table.
void carve_lstsq(Carve& c, const sns_sketch& sk, const sns_matrix& A, const sns_solve_opts& o,
                 LstsqWs& w) {
  carve_lstsq_bufs(c, sk, A, o, w);
  const LstsqWs wz = w;
  const size_t tb = table_bytes([&](ArgTable& t, Jobs& J) {
    build_lstsq_jobs(t, J, sk, A, nullptr, nullptr, o, wz);
  });
  w.args = c.take<char>(tb);
}

sns_solve_opts default_opts() {
  sns_solve_opts o;
  o.refine = 0;
  o.max_iters = 0;
  o.rtol = 0.0;
  o.accum_fp64 = 0;
  return o;
}

// Checks of sns_lstsq beyond those of the sketch.
sns_status check_solve(const sns_sketch& sk, const sns_matrix& A, const sns_solve_opts& o) {
  if (o.refine < 0 || o.refine > 2) return SNS_ERR_INVALID_ARG;
  if (o.refine && (o.max_iters < 0 || !(o.rtol >= 0.0))) return SNS_ERR_INVALID_ARG;
  if (A.n > 4096 || sk.d > kMaxQrD) return SNS_ERR_SHAPE;
  if (o.refine && A.n > 2048) return SNS_ERR_SHAPE;
  if (o.refine && A.layout == SNS_CSR) return SNS_ERR_DTYPE;  // refinement streams dense rows
  if (o.refine && (((uintptr_t)A.values % 16) != 0 || (A.ld * elem(A)) % 16 != 0))
    return SNS_ERR_SHAPE;
  return SNS_OK;
}

void build_batch_jobs(ArgTable& t, Jobs& J, const sns_problem* P, int count, const BatchWs& B,
                      bool real) {
  std::vector<SortArgs> sa;
  std::vector<GatherProb> ga;
  std::vector<QrArgs> qa;
  std::vector<FusedArgs> fa;
  std::vector<LsqrProb> la;
  for (int i = 0; i < count; ++i) {
    const sns_problem& q = P[i];
    const LstsqWs& w = B.w[i];
    const void* b = real ? q.b : nullptr;
    if (w.fused) {
      fa.push_back(fused_args(w.fp, q.sketch, q.A, b, w.fb, w.q, w.q.xw, B.infos + i));
    } else {
      sa.push_back(sort_args(w.sw.sp, q.sketch.seed, b, w.sw.sb));
      GatherProb g;
      g.plan = w.sw.gp;
      g.args =
          gather_args(w.sw.gp, q.A, (uint32_t)q.sketch.d, w.sw.sb, true, w.SA, w.Sb, w.sw.part);
      g.dtype = q.A.dtype;
      ga.push_back(g);
      qa.push_back(qr_args(q.sketch.d, q.A.n, w.SA, q.A.n, w.Sb, w.q, w.q.xw, nullptr, B.infos + i));
    }
    if (q.opts.refine) {
      LsqrProb lp;
      lp.plan = w.lp;
      lp.args = lsqr_args(q.A, b, w.lp, w.l, w.q, (int)q.sketch.d, q.opts.max_iters, q.opts.rtol,
                          real ? q.x : nullptr, B.infos + i);
      la.push_back(lp);
    }
  }
  const bool f64 = P[0].A.dtype == SNS_F64;
  J.sort = build_sort_job(t, sa, f64);
  J.gather = build_gather_job(t, ga);
  J.qr = build_qr_job(t, qa, f64);
  J.fused = build_fused_job(t, fa, f64);
  J.lsqr = build_lsqr_job(t, la, f64);
}

void carve_batch(Carve& c, const sns_problem* P, int count, BatchWs& B) {
  B.w.assign(count, LstsqWs{});
  B.infos = c.take<sns_info>((size_t)count);
  B.active = c.take<int>(1);
  for (int i = 0; i < count; ++i) carve_lstsq_bufs(c, P[i].sketch, P[i].A, P[i].opts, B.w[i]);
  ArgTable t0(nullptr);
  Jobs J0;
  build_batch_jobs(t0, J0, P, count, B, false);
  B.args = c.take<char>(t0.bytes());
}

sns_status check_batch(const sns_problem* P, int count) {
  if (!P || count < 1) return SNS_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i) {
    const sns_problem& q = P[i];
    sns_status s = check_matrix(&q.A);
    if (s != SNS_OK) return s;
    if ((s = check_sketch(&q.sketch, &q.A)) != SNS_OK) return s;
    if ((q.sketch.kind != SNS_SKETCH_COUNT && q.sketch.kind != SNS_SKETCH_SPARSE_SIGN) ||
        q.A.layout != SNS_DENSE_ROWMAJOR)
      return SNS_ERR_DTYPE;
    if (q.A.dtype != P[0].A.dtype) return SNS_ERR_DTYPE;
    if (q.opts.refine == 2) return SNS_ERR_INVALID_ARG;  // SAA-SAS: single-problem calls only
    if ((s = check_solve(q.sketch, q.A, q.opts)) != SNS_OK) return s;
  }
  return SNS_OK;
}

namespace {

// A private stream for capturing graphs (capture is not possible on the
// legacy default stream a caller may pass).
hipStream_t capture_stream() {
  thread_local hipStream_t s = nullptr;
  if (!s && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
  return s;
}

struct PinnedInt {
  int* p = nullptr;
  hipEvent_t ev = nullptr;
  PinnedInt() {
    if (hipHostMalloc((void**)&p, sizeof(int), hipHostMallocDefault) != hipSuccess) p = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
  }
};

PinnedInt& pinned_int() {
  thread_local PinnedInt r;
  return r;
}

constexpr int kChunkIters = 4;  // refinement iterations per chunk

}  // namespace

// Refinement of a batch: setup, chunks of iterations until no problem is
// left running (read back between chunks), final update and report.
sns_status run_batch_lsqr(const LsqrJob& j, int max_iters, int* active_dev, bool use_graph,
                          hipStream_t st) {
  if (j.count == 0) return SNS_OK;
  sns_status s = launch_lsqr_setup(j, st);
  if (s != SNS_OK) return s;
  PinnedInt& pi = pinned_int();
  if (!pi.p || !pi.ev) return SNS_ERR_HIP;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  if (use_graph) {
    hipStream_t cs = capture_stream();
    if (!cs) return SNS_ERR_HIP;
    SNS_HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < kChunkIters && s == SNS_OK; ++k) s = launch_lsqr_iteration(j, cs);
    if (s == SNS_OK) s = launch_lsqr_active(j, active_dev, cs);
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    if (s != SNS_OK) return s;
    SNS_HIP_TRY(e);
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return SNS_ERR_HIP;
    }
  }
  // iteration 0 is the residual pass; iterations past a problem's own
  // max_iters or stop rule return at once
  for (int done = 0; done <= max_iters; done += kChunkIters) {
    if (use_graph) {
      if (hipGraphLaunch(exec, st) != hipSuccess) { s = SNS_ERR_HIP; break; }
    } else {
      for (int k = 0; k < kChunkIters && s == SNS_OK; ++k) s = launch_lsqr_iteration(j, st);
      if (s == SNS_OK) s = launch_lsqr_active(j, active_dev, st);
      if (s != SNS_OK) break;
    }
    if (hipMemcpyAsync(pi.p, active_dev, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipEventRecord(pi.ev, st) != hipSuccess || hipEventSynchronize(pi.ev) != hipSuccess) {
      s = SNS_ERR_HIP;
      break;
    }
    if (*pi.p == 0) break;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (s != SNS_OK) return s;
  return launch_lsqr_finish(j, st);
}

}  // namespace sns
