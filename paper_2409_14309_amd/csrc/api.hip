// C ABI of libsns: argument checks, workspace layout and dispatch.  Every
// entry point validates on the host before enqueuing anything.
#include <math.h>
#include <string.h>

#include "common.hpp"
#include "kernels.hpp"
#include "solve.hpp"

using namespace sns;


extern "C" {

const char* sns_status_string(int status) {
  switch (status) {
    case SNS_OK: return "SNS_OK";
    case SNS_ERR_INVALID_ARG: return "SNS_ERR_INVALID_ARG";
    case SNS_ERR_SHAPE: return "SNS_ERR_SHAPE";
    case SNS_ERR_DTYPE: return "SNS_ERR_DTYPE";
    case SNS_ERR_RANK_DEFICIENT: return "SNS_ERR_RANK_DEFICIENT";
    case SNS_ERR_NOT_CONVERGED: return "SNS_ERR_NOT_CONVERGED";
    case SNS_ERR_NUMERICAL: return "SNS_ERR_NUMERICAL";
    case SNS_ERR_OUT_OF_MEMORY: return "SNS_ERR_OUT_OF_MEMORY";
    case SNS_ERR_QUEUE_FULL: return "SNS_ERR_QUEUE_FULL";
    case SNS_ERR_NOT_READY: return "SNS_ERR_NOT_READY";
    case SNS_ERR_HIP: return "SNS_ERR_HIP";
    default: return "SNS_ERR_UNKNOWN";
  }
}

int sns_version(void) { return 100; }

sns_status sns_hash(uint64_t seed, int64_t d, int64_t i0, int64_t count, uint32_t* h, int8_t* s,
                    void* stream) {
  if (d < 1 || d > 0xFFFFFFFFll || count < 0 || i0 < 0) return SNS_ERR_SHAPE;
  if (count > 0 && !h && !s) return SNS_ERR_INVALID_ARG;
  return launch_hash(seed, (uint32_t)d, i0, count, h, s, (hipStream_t)stream);
}

sns_status sns_sketch_workspace_size(const sns_sketch* sk, const sns_matrix* A, size_t* bytes) {
  sns_status s = check_matrix(A);
  if (s != SNS_OK) return s;
  if ((s = check_sketch(sk, A)) != SNS_OK) return s;
  if (!bytes) return SNS_ERR_INVALID_ARG;
  if (sk->kind == SNS_SKETCH_GAUSSIAN) {
    *bytes = gauss_workspace_bytes(*A, (uint32_t)sk->d);
    return SNS_OK;
  }
  if (sk->kind == SNS_SKETCH_HADAMARD) {
    *bytes = hadamard_workspace_bytes(*A, (uint32_t)sk->d);
    return SNS_OK;
  }
  if (A->layout == SNS_CSR) {  // enough for either accumulator width
    *bytes = csr_workspace_bytes(*A, (uint32_t)sk->d, true);
    return SNS_OK;
  }
  Carve c(nullptr, 0);
  SketchWs w;
  carve_sketch(c, *sk, *A, true, true, w);
  const sns_sketch skv = *sk;
  const sns_matrix Av = *A;
  const size_t tb = table_bytes([&](ArgTable& t, Jobs& J) {
    add_sketch_jobs(t, J, skv, Av, (const void*)1, nullptr, nullptr, w);
  });
  c.take<char>(tb);
  *bytes = c.off;
  return SNS_OK;
}

sns_status sns_sketch_apply(const sns_sketch* sk, const sns_matrix* A, const void* b, void* SA,
                            void* Sb, const sns_solve_opts* opts, void* workspace, size_t ws_bytes,
                            void* stream) {
  sns_status s = check_matrix(A);
  if (s != SNS_OK) return s;
  if ((s = check_sketch(sk, A)) != SNS_OK) return s;
  if (!SA || !workspace) return SNS_ERR_INVALID_ARG;
  if ((b == nullptr) != (Sb == nullptr)) return SNS_ERR_INVALID_ARG;
  const bool acc64 = opts && opts->accum_fp64;
  hipStream_t st = (hipStream_t)stream;
  if (sk->kind == SNS_SKETCH_GAUSSIAN) {
    if (ws_bytes < gauss_workspace_bytes(*A, (uint32_t)sk->d)) return SNS_ERR_OUT_OF_MEMORY;
    return launch_gauss_sketch(*A, (uint32_t)sk->d, sk->seed, b, SA, Sb, workspace, st);
  }
  if (sk->kind == SNS_SKETCH_HADAMARD) {
    if (ws_bytes < hadamard_workspace_bytes(*A, (uint32_t)sk->d)) return SNS_ERR_OUT_OF_MEMORY;
    return launch_hadamard_sketch(*A, (uint32_t)sk->d, sk->seed, b, SA, Sb, workspace, st);
  }
  if (A->layout == SNS_CSR)
    return launch_csr_sketch(*A, (uint32_t)sk->d, sk->seed, b, SA, Sb, acc64, workspace, ws_bytes, st);
  Carve c(workspace, ws_bytes);
  SketchWs w;
  carve_sketch(c, *sk, *A, b != nullptr, acc64, w);
  const sns_sketch skv = *sk;
  const sns_matrix Av = *A;
  const size_t tb = table_bytes([&](ArgTable& t, Jobs& J) {
    add_sketch_jobs(t, J, skv, Av, b, nullptr, nullptr, w);
  });
  char* args = c.take<char>(tb);
  if (!c.ok()) return SNS_ERR_OUT_OF_MEMORY;
  ArgTable t(args);
  Jobs J;
  add_sketch_jobs(t, J, skv, Av, b, SA, Sb, w);
  sns_status s2 = t.upload(st);
  if (s2 != SNS_OK) return s2;
  return run_sketch_jobs(J, st);
}

sns_status sns_qr_solve_workspace_size(int64_t d, int64_t n, size_t* bytes) {
  if (!bytes) return SNS_ERR_INVALID_ARG;
  if (n < 1 || d < n || d > kMaxQrD || n > 4096) return SNS_ERR_SHAPE;
  Carve c(nullptr, 0);
  QrBufs q;
  carve_qr(c, d, n, q);
  c.take<sns_info>(1);
  ArgTable t(nullptr);
  build_qr_job(t, std::vector<QrArgs>{qr_args(d, n, nullptr, n, nullptr, q, nullptr, nullptr,
                                               nullptr)},
               false);
  c.take<char>(t.bytes());
  *bytes = c.off;
  return SNS_OK;
}

sns_status sns_qr_solve(int64_t d, int64_t n, sns_dtype dtype, const void* SA, int64_t ld_sa,
                        const void* Sb, double* x0, double* R, sns_info* info, void* workspace,
                        size_t ws_bytes, void* stream) {
  if (!SA || !Sb || !x0 || !workspace) return SNS_ERR_INVALID_ARG;
  if (dtype != SNS_F32 && dtype != SNS_F64) return SNS_ERR_DTYPE;
  if (n < 1 || d < n || d > kMaxQrD || n > 4096 || ld_sa < n) return SNS_ERR_SHAPE;
  Carve c(workspace, ws_bytes);
  QrBufs q;
  carve_qr(c, d, n, q);
  sns_info* idev = c.take<sns_info>(1);
  const std::vector<QrArgs> qa{qr_args(d, n, SA, ld_sa, Sb, q, x0, R, idev)};
  ArgTable t0(nullptr);
  build_qr_job(t0, qa, dtype == SNS_F64);
  char* args = c.take<char>(t0.bytes());
  if (!c.ok()) return SNS_ERR_OUT_OF_MEMORY;
  hipStream_t st = (hipStream_t)stream;
  ArgTable t(args);
  const QrJob job = build_qr_job(t, qa, dtype == SNS_F64);
  sns_status s = t.upload(st);
  if (s != SNS_OK) return s;
  if ((s = launch_qr_job(job, st)) != SNS_OK) return s;
  if (info) SNS_HIP_TRY(hipMemcpyAsync(info, idev, sizeof(sns_info), hipMemcpyDeviceToHost, st));
  return SNS_OK;
}

sns_status sns_lstsq_workspace_size(const sns_sketch* sk, const sns_matrix* A,
                                    const sns_solve_opts* opts, size_t* bytes) {
  sns_status s = check_matrix(A);
  if (s != SNS_OK) return s;
  if ((s = check_sketch(sk, A)) != SNS_OK) return s;
  if (!bytes) return SNS_ERR_INVALID_ARG;
  const sns_solve_opts o = opts ? *opts : default_opts();
  if ((s = check_solve(*sk, *A, o)) != SNS_OK) return s;
  Carve c(nullptr, 0);
  LstsqWs w;
  carve_lstsq(c, *sk, *A, o, w);
  *bytes = c.off;
  return SNS_OK;
}

sns_status sns_lstsq(const sns_sketch* sk, const sns_matrix* A, const void* b, double* x,
                     const sns_solve_opts* opts, void* workspace, size_t ws_bytes, sns_info* info,
                     void* stream) {
  sns_status s = check_matrix(A);
  if (s != SNS_OK) return s;
  if ((s = check_sketch(sk, A)) != SNS_OK) return s;
  if (!b || !x || !workspace) return SNS_ERR_INVALID_ARG;
  const sns_solve_opts o = opts ? *opts : default_opts();
  if ((s = check_solve(*sk, *A, o)) != SNS_OK) return s;
  Carve c(workspace, ws_bytes);
  LstsqWs w;
  carve_lstsq(c, *sk, *A, o, w);
  if (!c.ok()) return SNS_ERR_OUT_OF_MEMORY;
  hipStream_t st = (hipStream_t)stream;
  ArgTable t(w.args);
  Jobs J;
  build_lstsq_jobs(t, J, *sk, *A, b, x, o, w);
  if ((s = t.upload(st)) != SNS_OK) return s;
  if (w.fused)
    s = launch_fused_job(J.fused, st);
  else if (sk->kind == SNS_SKETCH_GAUSSIAN)
    s = launch_gauss_sketch(*A, (uint32_t)sk->d, sk->seed, b, w.SA, w.Sb, w.gauss, st);
  else if (sk->kind == SNS_SKETCH_HADAMARD)
    s = launch_hadamard_sketch(*A, (uint32_t)sk->d, sk->seed, b, w.SA, w.Sb, w.gauss, st);
  else if (A->layout == SNS_CSR)
    s = launch_csr_sketch(*A, (uint32_t)sk->d, sk->seed, b, w.SA, w.Sb, o.accum_fp64 != 0, w.csr,
                          w.csr_bytes, st);
  else
    s = run_sketch_jobs(J, st);
  if (s != SNS_OK) return s;
  if (!w.fused && (s = launch_qr_job(J.qr, st)) != SNS_OK) return s;
  if (o.refine) {
    if ((s = run_lsqr_single(J.lsqr, o.max_iters, true, st)) != SNS_OK) return s;
  } else {
    SNS_HIP_TRY(hipMemcpyAsync(x, w.q.xw, sizeof(double) * A->n, hipMemcpyDeviceToDevice, st));
  }
  if (info) SNS_HIP_TRY(hipMemcpyAsync(info, w.info, sizeof(sns_info), hipMemcpyDeviceToHost, st));
  return SNS_OK;
}

sns_status sns_lstsq_batched_workspace_size(const sns_problem* probs, int count, size_t* bytes) {
  sns_status s = check_batch(probs, count);
  if (s != SNS_OK) return s;
  if (!bytes) return SNS_ERR_INVALID_ARG;
  Carve c(nullptr, 0);
  BatchWs B;
  carve_batch(c, probs, count, B);
  *bytes = c.off;
  return SNS_OK;
}

sns_status sns_lstsq_batched(const sns_problem* probs, int count, void* workspace,
                             size_t ws_bytes, sns_info* infos, int use_graph, void* stream) {
  sns_status s = check_batch(probs, count);
  if (s != SNS_OK) return s;
  if (!workspace) return SNS_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i)
    if (!probs[i].b || !probs[i].x) return SNS_ERR_INVALID_ARG;
  Carve c(workspace, ws_bytes);
  BatchWs B;
  carve_batch(c, probs, count, B);
  if (!c.ok()) return SNS_ERR_OUT_OF_MEMORY;
  hipStream_t st = (hipStream_t)stream;
  ArgTable t(B.args);
  Jobs J;
  build_batch_jobs(t, J, probs, count, B, true);
  if ((s = t.upload(st)) != SNS_OK) return s;
  if ((s = launch_fused_job(J.fused, st)) != SNS_OK) return s;
  if ((s = run_sketch_jobs(J, st)) != SNS_OK) return s;
  if ((s = launch_qr_job(J.qr, st)) != SNS_OK) return s;
  int max_iters = 0;
  for (int i = 0; i < count; ++i) {
    if (!probs[i].opts.refine)
      SNS_HIP_TRY(hipMemcpyAsync(probs[i].x, B.w[i].q.xw, sizeof(double) * probs[i].A.n,
                                 hipMemcpyDeviceToDevice, st));
    else if (probs[i].opts.max_iters > max_iters)
      max_iters = probs[i].opts.max_iters;
  }
  if ((s = run_batch_lsqr(J.lsqr, max_iters, B.active, use_graph != 0, st)) != SNS_OK) return s;
  if (infos)
    SNS_HIP_TRY(hipMemcpyAsync(infos, B.infos, sizeof(sns_info) * count, hipMemcpyDeviceToHost, st));
  return SNS_OK;
}

}  // extern "C"
