// SAP-SAS refinement: LSQR (Paige and Saunders 1982) on the right-
// preconditioned operator Abar = A R^{-1}, R from the QR of the sketch,
// starting from the sketch-and-solve answer x0 (sketch-and-precondition, as
// named in the paper's solver list).
//
// One pass over A per LSQR iteration.  The bidiagonalisation needs
// u_{i+1} = (Abar v_i - alpha_i u_i) / beta_{i+1} and then Abar^T u_{i+1}.
// The pass computes the unnormalised u' = A w - gamma u (w = R^{-1} v_i,
// gamma = alpha_i / beta_i because u is kept unnormalised), and in the same
// sweep over the rows accumulates A^T u' and ||u'||^2; dividing by
// beta_{i+1} = ||u'|| afterwards gives A^T u_{i+1}.  This is the same
// recurrence as the textbook algorithm with the scaling moved after the
// accumulation.  The residual r0 = b - A x0 and A^T r0 come from the same
// kernel with w = -x0, gamma = -1 and u = b.
//
// Precision: A and the m-vector u are stored in A's dtype; every product and
// accumulation is fp64, and all n-vectors are fp64.
//
// The scalar recurrences, the triangular solves with R and R^T, and the stop
// test run in one work-group (k_lsqr_step).  Once the stop rule holds, a flag
// in device memory makes the remaining launches return at once.
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"
#include "linalg.hpp"

namespace sns {

struct LsqrState {
  double alpha, beta, rhobar, phibar, gamma;
  double ratio;      // alpha_{k+1} |c_k| / sigma_hat at the last iteration
  double stop;       // rtol * sigma_hat (0: run max_iters)
  int iter, max_iters, done, status;
};

namespace {

template <typename T, int VEC>
struct VecT;
template <>
struct VecT<float, 4> { using type = float4; };
template <>
struct VecT<float, 1> { using type = float; };
template <>
struct VecT<double, 2> { using type = double2; };
template <>
struct VecT<double, 1> { using type = double; };

constexpr int kPassWaves = 4;

// Fused pass: for each row i of this work-group's contiguous row range,
//   t = A[i,:] . w;  u'[i] = t - gamma * uin[i];  z += A[i,:]^T u'[i];
//   nrm += u'[i]^2.  Per-group z and nrm go to zpart / npart.
template <typename T, int VEC, int LPR, int NCH>
__global__ __launch_bounds__(kPassWaves * 64) void k_lsqr_pass(
    const T* __restrict__ A, int64_t ld, int64_t m, int n, const LsqrState* __restrict__ st,
    const double* __restrict__ wv, const T* __restrict__ uin, T* __restrict__ uout,
    double* __restrict__ zpart, double* __restrict__ npart) {
  constexpr int RPW = 64 / LPR;
  constexpr int CW = LPR * VEC;        // columns per chunk
  constexpr int NSL = kPassWaves * RPW;  // row slots per group
  __shared__ double zred[kPassWaves][NCH * CW];
  __shared__ double nred[kPassWaves];
  if (st->done) return;
  const double gamma = st->gamma;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int slot = wid * RPW + lane / LPR, lr = lane % LPR;

  double w[NCH][VEC], z[NCH][VEC];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int col = c * CW + lr * VEC + e;
      w[c][e] = col < n ? wv[col] : 0.0;
      z[c][e] = 0.0;
    }
  double nrm = 0.0;

  const int64_t r0 = m * (int64_t)blockIdx.x / gridDim.x;
  const int64_t r1 = m * (int64_t)(blockIdx.x + 1) / gridDim.x;
  for (int64_t i = r0 + slot; i < r1; i += NSL) {
    const T* row = A + i * ld;
    T a[NCH][VEC];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int col = c * CW + lr * VEC;
      if (col + VEC <= n) {
        using V = typename VecT<T, VEC>::type;
        const V x = *reinterpret_cast<const V*>(row + col);
        const T* xe = reinterpret_cast<const T*>(&x);
#pragma unroll
        for (int e = 0; e < VEC; ++e) a[c][e] = xe[e];
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) a[c][e] = (col + e < n) ? row[col + e] : T(0);
      }
    }
    const double ui = (double)uin[i];
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int e = 0; e < VEC; ++e) t = fma((double)a[c][e], w[c][e], t);
#pragma unroll
    for (int off = 1; off < LPR; off <<= 1) t += __shfl_xor(t, off, 64);
    const double up = t - gamma * ui;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int e = 0; e < VEC; ++e) z[c][e] = fma((double)a[c][e], up, z[c][e]);
    if (lr == 0) {
      uout[i] = (T)up;
      nrm = fma(up, up, nrm);
    }
  }
  // combine the row slots of a wave (lanes with equal lr), then the waves
#pragma unroll
  for (int off = LPR; off < 64; off <<= 1)
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int e = 0; e < VEC; ++e) z[c][e] += __shfl_xor(z[c][e], off, 64);
  nrm = wave_sum(nrm);
  if (lane < LPR) {
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int e = 0; e < VEC; ++e) zred[wid][c * CW + lr * VEC + e] = z[c][e];
  }
  if (lane == 0) nred[wid] = nrm;
  __syncthreads();
  for (int col = threadIdx.x; col < n && col < NCH * CW; col += blockDim.x) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kPassWaves; ++q) s += zred[q][col];
    zpart[(size_t)blockIdx.x * n + col] = s;
  }
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kPassWaves; ++q) s += nred[q];
    npart[blockIdx.x] = s;
  }
}

__global__ void k_lsqr_init(int n, int max_iters, double stop, LsqrState* st,
                            const double* __restrict__ x0, double* __restrict__ wpass,
                            double* __restrict__ dy) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    wpass[j] = -x0[j];
    dy[j] = 0.0;
  }
  if (threadIdx.x == 0) {
    st->alpha = st->beta = st->rhobar = st->phibar = 0.0;
    st->gamma = -1.0;
    st->ratio = 0.0;
    st->stop = stop;
    st->iter = -1;  // the next step consumes the residual pass
    st->max_iters = max_iters;
    st->done = max_iters <= 0 ? 1 : 0;
    st->status = SNS_OK;
  }
}

// One LSQR step after a pass.  Vectors (fp64, length n): wpass, v, wd, dy.
__global__ __launch_bounds__(1024) void k_lsqr_step(int n, int G, double sighat,
                                                    const double* __restrict__ R,
                                                    const double* __restrict__ zpart,
                                                    const double* __restrict__ npart,
                                                    LsqrState* __restrict__ st,
                                                    double* __restrict__ wpass,
                                                    double* __restrict__ v,
                                                    double* __restrict__ wd,
                                                    double* __restrict__ dy) {
  extern __shared__ double sh[];
  double* y = sh;                 // n
  double* blk = sh + n;           // 64 x 64
  double* red = blk + 4096;       // 16
  double* part = red + 16;        // up to 1024
  if (st->done) return;
  const int t = threadIdx.x, nt = blockDim.x;
  // z = sum_g zpart[g]: columns are taken in tiles of `nc`; inside a tile,
  // thread t sums column t % nc over the partials g = t / nc (mod K), and the
  // K sums are added in order.
  const int nc = n < nt ? n : nt;
  const int K = nt / nc;
  for (int j0 = 0; j0 < n; j0 += nc) {
    const int jl = t % nc, kk = t / nc, j = j0 + jl;
    double s = 0.0;
    if (kk < K && j < n)
      for (int g = kk; g < G; g += K) s += zpart[(size_t)g * n + j];
    if (kk < K) part[kk * nc + jl] = s;
    __syncthreads();
    if (t < nc && j0 + t < n) {
      double tot = 0.0;
      for (int q = 0; q < K; ++q) tot += part[q * nc + t];
      y[j0 + t] = tot;
    }
    __syncthreads();
  }
  double ps = 0.0;
  for (int g = t; g < G; g += nt) ps += npart[g];
  const double beta = sqrt(block_sum(ps, red));
  const bool first = st->iter < 0;
  if (!isfinite(beta)) {
    if (t == 0) { st->status = SNS_ERR_NUMERICAL; st->done = 1; }
    return;
  }
  // y = R^{-T} (z / beta) - beta v   (first step: without the beta v term)
  if (beta > 0.0) {
    for (int j = t; j < n; j += nt) y[j] /= beta;
    __syncthreads();
    trsv_upper_trans_lds(R, n, n, y, blk);
    if (!first)
      for (int j = t; j < n; j += nt) y[j] -= beta * v[j];
  } else {
    for (int j = t; j < n; j += nt) y[j] = 0.0;
  }
  __syncthreads();
  double ss = 0.0;
  for (int j = t; j < n; j += nt) ss += y[j] * y[j];
  const double alpha = sqrt(block_sum(ss, red));
  if (!isfinite(alpha)) {
    if (t == 0) { st->status = SNS_ERR_NUMERICAL; st->done = 1; }
    return;
  }
  const double inva = alpha > 0.0 ? 1.0 / alpha : 0.0;
  if (first) {
    // beta_1 u_1 = r0, alpha_1 v_1 = Abar^T u_1, wd_1 = v_1, phibar = beta_1, rhobar = alpha_1
    for (int j = t; j < n; j += nt) {
      const double vj = y[j] * inva;
      v[j] = vj;
      wd[j] = vj;
      dy[j] = 0.0;
      y[j] = vj;
    }
    __syncthreads();
    if (t == 0) {
      st->beta = beta;
      st->alpha = alpha;
      st->phibar = beta;
      st->rhobar = alpha;
      st->iter = 0;
      st->gamma = beta > 0.0 ? alpha / beta : 0.0;
      st->ratio = sighat > 0.0 ? alpha / sighat : alpha;
      if (beta == 0.0 || alpha == 0.0 || st->max_iters <= 0) st->done = 1;
    }
  } else {
    const double rhobar = st->rhobar, phibar = st->phibar;
    const double rho = hypot(rhobar, beta);
    const double c = rhobar / rho, s = beta / rho;
    const double theta = s * alpha;
    const double phi = c * phibar;
    const double f1 = phi / rho, f2 = theta / rho;
    for (int j = t; j < n; j += nt) {
      const double vj = y[j] * inva;
      const double wdj = wd[j];
      dy[j] += f1 * wdj;
      wd[j] = vj - f2 * wdj;
      v[j] = vj;
      y[j] = vj;
    }
    __syncthreads();
    if (t == 0) {
      st->beta = beta;
      st->alpha = alpha;
      st->rhobar = -c * alpha;
      st->phibar = s * phibar;
      st->iter += 1;
      st->gamma = beta > 0.0 ? alpha / beta : 0.0;
      const double ratio = alpha * fabs(c);
      st->ratio = sighat > 0.0 ? ratio / sighat : ratio;
      bool stop = beta == 0.0 || alpha == 0.0 || st->iter >= st->max_iters;
      if (st->stop > 0.0 && ratio <= st->stop) stop = true;
      if (stop) {
        st->done = 1;
        if (st->stop > 0.0 && ratio > st->stop && beta != 0.0 && alpha != 0.0)
          st->status = SNS_ERR_NOT_CONVERGED;
      }
    }
  }
  __syncthreads();
  // next pass direction: wpass = R^{-1} v
  trsv_upper_lds(R, n, n, y, blk);
  for (int j = t; j < n; j += nt) wpass[j] = y[j];
}

// x = x0 + R^{-1} dy; report.
__global__ __launch_bounds__(1024) void k_lsqr_final(int n, const double* __restrict__ R,
                                                     const double* __restrict__ x0,
                                                     const double* __restrict__ dy,
                                                     const LsqrState* __restrict__ st,
                                                     double* __restrict__ x,
                                                     sns_info* __restrict__ info) {
  extern __shared__ double sh[];
  double* y = sh;
  double* blk = sh + n;
  for (int j = threadIdx.x; j < n; j += blockDim.x) y[j] = dy[j];
  __syncthreads();
  trsv_upper_lds(R, n, n, y, blk);
  for (int j = threadIdx.x; j < n; j += blockDim.x) x[j] = x0[j] + y[j];
  if (threadIdx.x == 0) {
    info->iters = st->iter < 0 ? 0 : st->iter;
    info->rel_resid_est = st->ratio;
    if (info->status == SNS_OK) info->status = st->status;
  }
}

template <typename T, int VEC, int LPR, int NCH>
void launch_pass_t(const sns_matrix& A, const LsqrPlan& p, const LsqrBufs& l, const void* uin,
                   hipStream_t s) {
  double* vecs = l.vecs;
  SNS_LAUNCH("lsqr_pass", (k_lsqr_pass<T, VEC, LPR, NCH>), dim3(p.grid), dim3(kPassWaves * 64), 0, s,
                     static_cast<const T*>(A.values), A.ld, A.m, (int)A.n,
                     static_cast<const LsqrState*>(l.state), vecs, static_cast<const T*>(uin),
                     static_cast<T*>(l.u), l.zpart, l.npart);
}

template <typename T, int VEC>
void launch_pass_v(const sns_matrix& A, const LsqrPlan& p, const LsqrBufs& l, const void* uin,
                   hipStream_t s) {
  const int nch = p.nch;
  switch (p.lpr * 16 + nch) {
    case 4 * 16 + 1: launch_pass_t<T, VEC, 4, 1>(A, p, l, uin, s); break;
    case 4 * 16 + 2: launch_pass_t<T, VEC, 4, 2>(A, p, l, uin, s); break;
    case 4 * 16 + 4: launch_pass_t<T, VEC, 4, 4>(A, p, l, uin, s); break;
    case 8 * 16 + 4: launch_pass_t<T, VEC, 8, 4>(A, p, l, uin, s); break;
    case 16 * 16 + 4: launch_pass_t<T, VEC, 16, 4>(A, p, l, uin, s); break;
    case 32 * 16 + 4: launch_pass_t<T, VEC, 32, 4>(A, p, l, uin, s); break;
    case 64 * 16 + 4: launch_pass_t<T, VEC, 64, 4>(A, p, l, uin, s); break;
    default: launch_pass_t<T, VEC, 64, 8>(A, p, l, uin, s); break;
  }
}

}  // namespace

// Plan: lanes per row (lpr) and 16-byte column chunks per lane (nch).  The
// element vector width is 16 bytes when rows are 16-byte aligned.
LsqrPlan make_lsqr_plan(const sns_matrix& A) {
  LsqrPlan p;
  const int es = A.dtype == SNS_F64 ? 8 : 4;
  const int vw = 16 / es;
  const int64_t n = A.n;
  int lpr = 4;
  while (lpr < 64 && (int64_t)lpr * vw * 4 < n) lpr <<= 1;
  int64_t nch = (n + (int64_t)lpr * vw - 1) / ((int64_t)lpr * vw);
  if (lpr == 4) nch = nch <= 1 ? 1 : (nch <= 2 ? 2 : 4);
  else nch = nch <= 4 ? 4 : 8;
  p.lpr = lpr;
  p.nch = (int)nch;
  const int64_t rows_per_group = 256;
  int64_t g = (A.m + rows_per_group - 1) / rows_per_group;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  p.grid = (int)g;
  return p;
}

size_t lsqr_workspace_bytes(const sns_matrix& A, const LsqrPlan& p) {
  Carve c(nullptr, 0);
  LsqrBufs l;
  carve_lsqr(c, A, p, l);
  return c.off;
}

void carve_lsqr(Carve& c, const sns_matrix& A, const LsqrPlan& p, LsqrBufs& l) {
  const size_t es = A.dtype == SNS_F64 ? 8 : 4;
  l.u = c.take<char>((size_t)A.m * es);
  l.zpart = c.take<double>((size_t)p.grid * A.n);
  l.npart = c.take<double>((size_t)p.grid);
  l.vecs = c.take<double>((size_t)6 * A.n);
  l.state = c.take<LsqrState>(1);
}

namespace {

// Host-side view of the device stop state, copied after every LSQR step into
// pinned memory so the host can decide how far ahead to enqueue.
struct PollRing {
  static constexpr int kSlots = 8;
  LsqrState* slot = nullptr;  // pinned host memory
  hipEvent_t ev[kSlots] = {};
  bool ok = false;
  PollRing() {
    if (hipHostMalloc((void**)&slot, sizeof(LsqrState) * kSlots, hipHostMallocDefault) !=
        hipSuccess)
      return;
    for (int i = 0; i < kSlots; ++i)
      if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) return;
    ok = true;
  }
};

PollRing& poll_ring() {
  thread_local PollRing r;
  return r;
}

}  // namespace

sns_status launch_sap_refine(const sns_matrix& A, const void* b, const LsqrPlan& p,
                             const LsqrBufs& l, const QrBufs& q, int d, int max_iters,
                             double rtol, double* x, sns_info* info_dev, hipStream_t s) {
  const int n = (int)A.n;
  if (n > 2048) return SNS_ERR_SHAPE;
  const size_t es = A.dtype == SNS_F64 ? 8 : 4;
  if ((uintptr_t)A.values % 16 != 0 || (A.ld * es) % 16 != 0) return SNS_ERR_SHAPE;
  const double sighat = 1.0 - sqrt((double)n / (double)d);
  const double stop = rtol > 0.0 ? rtol * (sighat > 0.0 ? sighat : 1.0) : 0.0;
  double* wpass = l.vecs;
  double* v = l.vecs + n;
  double* wd = l.vecs + 2 * n;
  double* dy = l.vecs + 3 * n;
  LsqrState* st = static_cast<LsqrState*>(l.state);
  SNS_LAUNCH("lsqr_init", k_lsqr_init, dim3(1), dim3(256), 0, s, n, max_iters, stop, st, q.xw, wpass,
             dy);
  const size_t lds_step = ((size_t)n + 4096 + 16 + 1024) * sizeof(double);
  // iteration 0 is the residual pass r0 = b - A x0 plus the start-up step
  auto enqueue = [&](int it) {
    const void* uin = it == 0 ? b : l.u;
    if (A.dtype == SNS_F64) launch_pass_v<double, 2>(A, p, l, uin, s);
    else launch_pass_v<float, 4>(A, p, l, uin, s);
    SNS_LAUNCH("lsqr_step", k_lsqr_step, dim3(1), dim3(1024), lds_step, s, n, p.grid, sighat, q.R,
               l.zpart, l.npart, st, wpass, v, wd, dy);
  };
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  SNS_HIP_TRY(hipStreamIsCapturing(s, &cap));
  PollRing& ring = poll_ring();
  if (cap != hipStreamCaptureStatusNone || stop == 0.0 || !ring.ok) {
    // fixed launch sequence; iterations after the stop rule return at once
    for (int it = 0; it <= max_iters; ++it) enqueue(it);
  } else {
    // Keep at most two iterations in flight.  Before running ahead of an
    // unread iteration, predict from the geometric decay of the stop ratio
    // whether that iteration converges; if so, wait for it instead, so that no
    // launch is issued after the stop rule has fired.
    const int K = PollRing::kSlots;
    auto post = [&](int it) {
      SNS_HIP_TRY(hipMemcpyAsync(&ring.slot[it % K], st, sizeof(LsqrState), hipMemcpyDeviceToHost,
                                 s));
      SNS_HIP_TRY(hipEventRecord(ring.ev[it % K], s));
      return SNS_OK;
    };
    double r_prev = -1.0, r_last = -1.0;
    bool done = false;
    int known = -1;  // last iteration whose state has been read
    auto read = [&](int it) {
      SNS_HIP_TRY(hipEventSynchronize(ring.ev[it % K]));
      const LsqrState& h = ring.slot[it % K];
      done = h.done != 0;
      r_prev = r_last;
      r_last = h.ratio * (sighat > 0.0 ? sighat : 1.0);
      known = it;
      return SNS_OK;
    };
    enqueue(0);
    sns_status e = post(0);
    if (e != SNS_OK) return e;
    int next = 1;
    while (next <= max_iters) {
      if (known < next - 1) {
        // state after next-1 unknown: wait for it if it is predicted to stop
        bool predict_stop = false;
        if (r_last > 0.0 && r_prev > 0.0) {
          double qr = r_last / r_prev;
          qr = qr < 0.2 ? 0.2 : (qr > 0.95 ? 0.95 : qr);
          // iteration next-1 is one step past the last known ratio
          predict_stop = r_last * qr <= 2.0 * stop;
        }
        if (predict_stop || known < next - 2) {
          if ((e = read(known + 1)) != SNS_OK) return e;
          continue;
        }
      }
      if (known == next - 1 && done) break;
      enqueue(next);
      if ((e = post(next)) != SNS_OK) return e;
      ++next;
      if (known < next - 2) {
        if ((e = read(next - 2)) != SNS_OK) return e;
        if (done) break;
      }
    }
  }
  const size_t lds_fin = ((size_t)n + 4096) * sizeof(double);
  SNS_LAUNCH("lsqr_final", k_lsqr_final, dim3(1), dim3(1024), lds_fin, s, n, q.R, q.xw, dy, st, x,
             info_dev);
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace sns
