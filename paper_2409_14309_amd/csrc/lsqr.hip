// SAP-SAS refinement: LSQR (Paige and Saunders 1982) on the right-
// preconditioned operator A X with X = R^{-1}, R from the QR of the sketch,
// starting from the sketch-and-solve answer x0 (sketch-and-precondition, as
// named in the paper's solver list).
//
// X is formed once per solve (k_tri_inv, fp64 back substitution per column)
// and applied as matrix-vector products by many work-groups.  LSQR runs on the
// fixed operator A X and the answer is mapped back with the same X,
// x = x0 + X dy, so x is the least-squares solution of A x = b whatever the
// rounding in X; X only has to keep A X well conditioned.
//
// One pass over A per LSQR iteration.  The bidiagonalisation needs
// u_{i+1} = (Abar v_i - alpha_i u_i) / beta_{i+1} and then Abar^T u_{i+1}.
// The pass computes the unnormalised u' = A w - gamma u (w = X v_i,
// gamma = alpha_i / beta_i because u is kept unnormalised), and in the same
// sweep over the rows accumulates A^T u' and ||u'||^2; dividing by
// beta_{i+1} = ||u'|| afterwards gives A^T u_{i+1}.  This is the same
// recurrence as the textbook algorithm with the scaling moved after the
// accumulation.  The residual r0 = b - A x0 and A^T r0 come from the same
// kernel with w = -x0, gamma = -1 and u = b.
//
// Per iteration: k_lsqr_pass (all of A), k_lsqr_reduce (partials of A^T u'),
// k_lsqr_xtz (y = X^T z / beta - beta v; the last work-group to finish runs
// the scalar recurrences and the n-vector updates), k_lsqr_xv (w = X v).
//
// Precision: A and the m-vector u are stored in A's dtype; every product and
// accumulation is fp64, and all n-vectors are fp64.  Once the stop rule
// holds, a flag in device memory makes the remaining launches return at once.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "common.hpp"
#include "kernels.hpp"
#include "linalg.hpp"

namespace sns {

struct LsqrState {
  double alpha, beta, rhobar, phibar, gamma;
  double ratio;      // alpha_{k+1} |c_k| / sigma_hat at the last iteration
  double stop;       // rtol * sigma_hat (0: run max_iters)
  int iter, max_iters, done, status;
  unsigned int arrived;  // work-groups of k_lsqr_xtz done (reset by the last)
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
constexpr int kRedSplit = 16;      // partial groups left for the step kernel

template <typename T, int VEC, int NCH, int LPR>
__device__ __forceinline__ void load_row_chunks(const T* __restrict__ row, int lr, int n,
                                                T (&a)[NCH][VEC]) {
  constexpr int CW = LPR * VEC;
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
}

// Fused pass: for each row i of this work-group's contiguous row range,
//   t = A[i,:] . w;  u'[i] = t - gamma * uin[i];  z += A[i,:]^T u'[i];
//   nrm += u'[i]^2.  Per-group z and nrm go to zpart / npart.  A row is
// spread over LPR lanes (NCH 16-byte chunks each); each row slot handles two
// rows per step so that two rows' loads are in flight together.
template <typename T, int VEC, int LPR, int NCH, int U>
__global__ __launch_bounds__(kPassWaves * 64) void k_lsqr_pass(
    const T* __restrict__ A, int64_t ld, int64_t m, int n, const LsqrState* __restrict__ st,
    const double* __restrict__ wv, const T* __restrict__ uin, T* __restrict__ uout,
    double* __restrict__ zpart, double* __restrict__ npart) {
  constexpr int RPW = 64 / LPR;
  constexpr int CW = LPR * VEC;          // columns per chunk
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
  if constexpr (U == 1) {
    for (int64_t i = r0 + slot; i < r1; i += NSL) {
      T a0[NCH][VEC];
      load_row_chunks<T, VEC, NCH, LPR>(A + i * ld, lr, n, a0);
      const double u0 = (double)uin[i];
      double t0 = 0.0;
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) t0 = fma((double)a0[c][e], w[c][e], t0);
#pragma unroll
      for (int off = 1; off < LPR; off <<= 1) t0 += __shfl_xor(t0, off, 64);
      const double p0 = t0 - gamma * u0;
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) z[c][e] = fma((double)a0[c][e], p0, z[c][e]);
      if (lr == 0) {
        uout[i] = (T)p0;
        nrm = fma(p0, p0, nrm);
      }
    }
  } else {
    for (int64_t i = r0 + slot; i < r1; i += 2 * NSL) {
      const int64_t i2 = i + NSL;
      const bool has2 = i2 < r1;
      T a0[NCH][VEC], a1[NCH][VEC];
      load_row_chunks<T, VEC, NCH, LPR>(A + i * ld, lr, n, a0);
      if (has2) {
        load_row_chunks<T, VEC, NCH, LPR>(A + i2 * ld, lr, n, a1);
      } else {
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
          for (int e = 0; e < VEC; ++e) a1[c][e] = T(0);
      }
      const double u0 = (double)uin[i];
      const double u1 = has2 ? (double)uin[i2] : 0.0;
      double t0 = 0.0, t1 = 0.0;
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          t0 = fma((double)a0[c][e], w[c][e], t0);
          t1 = fma((double)a1[c][e], w[c][e], t1);
        }
#pragma unroll
      for (int off = 1; off < LPR; off <<= 1) {
        t0 += __shfl_xor(t0, off, 64);
        t1 += __shfl_xor(t1, off, 64);
      }
      const double p0 = t0 - gamma * u0;
      const double p1 = t1 - gamma * u1;
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          z[c][e] = fma((double)a0[c][e], p0, z[c][e]);
          z[c][e] = fma((double)a1[c][e], p1, z[c][e]);
        }
      if (lr == 0) {
        uout[i] = (T)p0;
        nrm = fma(p0, p0, nrm);
        if (has2) {
          uout[i2] = (T)p1;
          nrm = fma(p1, p1, nrm);
        }
      }
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

// First level of the reduction of the G per-group partials: work-group
// (cx, s) sums partials [s G / S, (s+1) G / S) for columns [64 cx, 64 cx + 64)
// into zred2[s][.] (and, for cx = 0, the norms into nred2[s]).  Four thread
// groups take every fourth partial, each with eight running sums (partials
// g, g + 4, ..., g + 28 of a round of 32); all sums are combined in a fixed
// order.
__global__ __launch_bounds__(256) void k_lsqr_reduce(int n, int G,
                                                     const LsqrState* __restrict__ st,
                                                     const double* __restrict__ zpart,
                                                     const double* __restrict__ npart,
                                                     double* __restrict__ zred2,
                                                     double* __restrict__ nred2) {
  __shared__ double part[4][64];
  __shared__ double red[4];
  if (st->done) return;
  const int t = threadIdx.x, cl = t & 63, grp = t >> 6;
  const int s = blockIdx.y;
  const int g0 = (int)((int64_t)G * s / kRedSplit), g1 = (int)((int64_t)G * (s + 1) / kRedSplit);
  const int col = blockIdx.x * 64 + cl;
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  if (col < n) {
    int g = g0 + grp;
    for (; g + 28 < g1; g += 32) {
      double v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = zpart[(size_t)(g + 4 * k) * n + col];
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[k] += v[k];
    }
    for (int k = 0; g < g1; g += 4, ++k) acc[k] += zpart[(size_t)g * n + col];
  }
  part[grp][cl] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (t < 64 && col < n) zred2[(size_t)s * n + col] = ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
  if (blockIdx.x == 0) {
    double a = 0.0;
    for (int g = g0 + t; g < g1; g += 256) a += npart[g];
    a = block_sum(a, red);
    if (t == 0) nred2[s] = a;
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
    st->arrived = 0u;
  }
}

// X = R^{-1}: work-group j solves R x = e_j on the leading (j+1) x (j+1)
// block by back substitution and writes column j of X (column-major Xc and
// row-major Xr; X is upper triangular).
constexpr int kInvThreads = 64;
__global__ __launch_bounds__(kInvThreads) void k_tri_inv(int n, const double* __restrict__ Rc,
                                                         const double* __restrict__ invd,
                                                         double* __restrict__ Xc,
                                                         double* __restrict__ Xr) {
  extern __shared__ double sh[];
  double* x = sh;        // n
  double* blk = sh + n;  // 64 x 64
  const int j = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += kInvThreads) x[i] = i == j ? 1.0 : 0.0;
  __syncthreads();
  trsv_lds<true, kInvThreads>(Rc, n, j + 1, invd, x, blk);
  for (int i = threadIdx.x; i < n; i += kInvThreads) {
    const double v = i <= j ? x[i] : 0.0;
    Xc[(int64_t)j * n + i] = v;
    Xr[(int64_t)i * n + j] = v;
  }
}

constexpr int kGemvThreads = 256;
constexpr int kGemvRows = 16;  // rows per work-group (4 per wave)

// Dot product of row i of a triangular matrix stored row-contiguously
// (M[i * n + j]) with vec over j in [j0, j1), by one wave; all lanes get it.
__device__ __forceinline__ double wave_row_dot(const double* __restrict__ M, int n, int i, int j0,
                                               int j1, const double* __restrict__ vec) {
  const int lane = threadIdx.x & 63;
  const double* row = M + (int64_t)i * n;
  double s = 0.0;
  for (int j = j0 + lane; j < j1; j += 64) s = fma(row[j], vec[j], s);
  return wave_sum(s);
}

// y = X^T (z / beta) - beta v (first step: X^T (z / beta)), z = sum of the
// reduction splits.  X^T row i = X column i = Xc[i * n + j], j <= i.  Each
// group writes its rows of y and its share of ||y||^2; the last group to
// finish (arrival counter) then runs the scalar recurrences and the n-vector
// updates for the whole vector in a fixed order.
__global__ __launch_bounds__(kGemvThreads) void k_lsqr_xtz(
    int n, double sighat, const double* __restrict__ Xc, const double* __restrict__ zred2,
    const double* __restrict__ nred2, LsqrState* __restrict__ st, double* __restrict__ zbuf,
    double* __restrict__ ybuf, double* __restrict__ ypart, double* __restrict__ v,
    double* __restrict__ wd, double* __restrict__ dy) {
  extern __shared__ double sh[];
  double* z = sh;        // n
  double* red = sh + n;  // 16 + kGemvRows
  __shared__ bool last;
  if (st->done) return;
  const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, wv = t >> 6;
  double beta2 = 0.0;
  for (int s = 0; s < kRedSplit; ++s) beta2 += nred2[s];
  const double beta = sqrt(beta2);
  const double invb = beta > 0.0 ? 1.0 / beta : 0.0;
  const bool first = st->iter < 0;
  for (int j = t; j < n; j += nt) {
    double a = 0.0;
    for (int s = 0; s < kRedSplit; ++s) a += zred2[(size_t)s * n + j];
    z[j] = a * invb;
  }
  __syncthreads();
  double ysq = 0.0;
  for (int r = wv; r < kGemvRows; r += nt / 64) {
    const int i = blockIdx.x * kGemvRows + r;
    if (i < n) {
      double yi = wave_row_dot(Xc, n, i, 0, i + 1, z);
      if (!first) yi -= beta * v[i];
      if (lane == 0) {
        ybuf[i] = yi;
        red[16 + r] = yi * yi;
      }
    } else if (lane == 0) {
      red[16 + r] = 0.0;
    }
  }
  __syncthreads();
  if (t == 0) {
    for (int r = 0; r < kGemvRows; ++r) ysq += red[16 + r];
    ypart[blockIdx.x] = ysq;
    __threadfence();
    const unsigned int prev = atomicAdd(&st->arrived, 1u);
    last = prev == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  // ---- last group: scalars and n-vector updates ----
  double a2 = 0.0;
  for (int g = 0; g < (int)gridDim.x; ++g) a2 += ypart[g];  // same value on every thread
  const double alpha = sqrt(a2);
  if (!isfinite(beta) || !isfinite(alpha)) {
    if (t == 0) {
      st->status = SNS_ERR_NUMERICAL;
      st->done = 1;
      st->arrived = 0u;
    }
    return;
  }
  const double inva = alpha > 0.0 ? 1.0 / alpha : 0.0;
  if (first) {
    // beta_1 u_1 = r0, alpha_1 v_1 = Abar^T u_1, wd_1 = v_1, phibar = beta_1, rhobar = alpha_1
    for (int j = t; j < n; j += nt) {
      const double vj = ybuf[j] * inva;
      v[j] = vj;
      wd[j] = vj;
      dy[j] = 0.0;
    }
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
      const double vj = ybuf[j] * inva;
      const double wdj = wd[j];
      dy[j] += f1 * wdj;
      wd[j] = vj - f2 * wdj;
      v[j] = vj;
    }
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
  if (t == 0) st->arrived = 0u;
}

// w = X v for the next pass: row i of X = Xr[i * n + j], j >= i.  `out`
// receives w; with add0 set, out = add0 + X v (the final x = x0 + X dy).
__global__ __launch_bounds__(kGemvThreads) void k_lsqr_xv(int n, const double* __restrict__ Xr,
                                                          const double* __restrict__ vin,
                                                          const double* __restrict__ add0,
                                                          const LsqrState* __restrict__ st,
                                                          int skip_if_done,
                                                          double* __restrict__ out) {
  extern __shared__ double sh[];
  double* vec = sh;  // n
  if (skip_if_done && st->done) return;
  const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, wv = t >> 6;
  for (int j = t; j < n; j += nt) vec[j] = vin[j];
  __syncthreads();
  for (int r = wv; r < kGemvRows; r += nt / 64) {
    const int i = blockIdx.x * kGemvRows + r;
    if (i < n) {
      const double wi = wave_row_dot(Xr, n, i, i, n, vec);
      if (lane == 0) out[i] = add0 ? add0[i] + wi : wi;
    }
  }
}

__global__ void k_lsqr_report(const LsqrState* __restrict__ st, sns_info* __restrict__ info) {
  info->iters = st->iter < 0 ? 0 : st->iter;
  info->rel_resid_est = st->ratio;
  if (info->status == SNS_OK) info->status = st->status;
}

template <typename T, int VEC, int LPR, int NCH, int U>
void launch_pass_t(const sns_matrix& A, const LsqrPlan& p, const LsqrBufs& l, const void* uin,
                   hipStream_t s) {
  double* vecs = l.vecs;
  SNS_LAUNCH("lsqr_pass", (k_lsqr_pass<T, VEC, LPR, NCH, U>), dim3(p.grid), dim3(kPassWaves * 64),
             0, s, static_cast<const T*>(A.values), A.ld, A.m, (int)A.n,
             static_cast<const LsqrState*>(l.state), vecs, static_cast<const T*>(uin),
             static_cast<T*>(l.u), l.zpart, l.npart);
}

template <typename T, int VEC, int U>
void launch_pass_u(const sns_matrix& A, const LsqrPlan& p, const LsqrBufs& l, const void* uin,
                   hipStream_t s) {
  switch (p.lpr * 16 + p.nch) {
    case 4 * 16 + 1: launch_pass_t<T, VEC, 4, 1, U>(A, p, l, uin, s); break;
    case 4 * 16 + 2: launch_pass_t<T, VEC, 4, 2, U>(A, p, l, uin, s); break;
    case 4 * 16 + 4: launch_pass_t<T, VEC, 4, 4, U>(A, p, l, uin, s); break;
    case 8 * 16 + 4: launch_pass_t<T, VEC, 8, 4, U>(A, p, l, uin, s); break;
    case 16 * 16 + 1: launch_pass_t<T, VEC, 16, 1, U>(A, p, l, uin, s); break;
    case 16 * 16 + 2: launch_pass_t<T, VEC, 16, 2, U>(A, p, l, uin, s); break;
    case 16 * 16 + 4: launch_pass_t<T, VEC, 16, 4, U>(A, p, l, uin, s); break;
    case 32 * 16 + 1: launch_pass_t<T, VEC, 32, 1, U>(A, p, l, uin, s); break;
    case 32 * 16 + 2: launch_pass_t<T, VEC, 32, 2, U>(A, p, l, uin, s); break;
    case 32 * 16 + 4: launch_pass_t<T, VEC, 32, 4, U>(A, p, l, uin, s); break;
    case 64 * 16 + 1: launch_pass_t<T, VEC, 64, 1, U>(A, p, l, uin, s); break;
    case 64 * 16 + 2: launch_pass_t<T, VEC, 64, 2, U>(A, p, l, uin, s); break;
    case 64 * 16 + 4: launch_pass_t<T, VEC, 64, 4, U>(A, p, l, uin, s); break;
    default: launch_pass_t<T, VEC, 64, 8, U>(A, p, l, uin, s); break;
  }
}

template <typename T, int VEC>
void launch_pass_v(const sns_matrix& A, const LsqrPlan& p, const LsqrBufs& l, const void* uin,
                   hipStream_t s) {
  if (p.unroll == 2) launch_pass_u<T, VEC, 2>(A, p, l, uin, s);
  else launch_pass_u<T, VEC, 1>(A, p, l, uin, s);
}

}  // namespace

// Plan: lanes per row (lpr) and 16-byte column chunks per lane (nch) such
// that lpr * nch * (16 / element size) covers n; work-groups of the pass.
// SNS_LSQR_PLAN="lpr,nch,grid,unroll" overrides the choice (tuning runs);
// an override that does not cover n is ignored.
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
  p.unroll = 1;
  if (const char* e = getenv("SNS_LSQR_PLAN")) {
    int a = 0, b = 0, c = 0, d = 1;
    if (sscanf(e, "%d,%d,%d,%d", &a, &b, &c, &d) >= 3) {
      const bool lpr_ok = a == 4 || a == 8 || a == 16 || a == 32 || a == 64;
      const bool nch_ok = b == 1 || b == 2 || b == 4 || b == 8;
      if (lpr_ok && nch_ok && (int64_t)a * b * vw >= n && c >= 1 && c <= 65535) {
        p.lpr = a;
        p.nch = b;
        p.grid = c;
        p.unroll = d == 2 ? 2 : 1;
      }
    }
  }
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
  l.zred2 = c.take<double>((size_t)kRedSplit * A.n);
  l.nred2 = c.take<double>((size_t)kRedSplit);
  l.Xc = c.take<double>((size_t)A.n * A.n);
  l.Xr = c.take<double>((size_t)A.n * A.n);
  l.ypart = c.take<double>((size_t)(A.n + kGemvRows - 1) / kGemvRows);
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
  double* ybuf = l.vecs + 4 * n;
  LsqrState* st = static_cast<LsqrState*>(l.state);
  SNS_LAUNCH("lsqr_init", k_lsqr_init, dim3(1), dim3(256), 0, s, n, max_iters, stop, st, q.xw, wpass,
             dy);
  SNS_LAUNCH("tri_inv", k_tri_inv, dim3(n), dim3(kInvThreads), ((size_t)n + 4096) * sizeof(double),
             s, n, q.R, q.invd, l.Xc, l.Xr);
  const unsigned gemv_grid = (unsigned)((n + kGemvRows - 1) / kGemvRows);
  const size_t lds_xtz = ((size_t)n + 16 + kGemvRows) * sizeof(double);
  const size_t lds_xv = (size_t)n * sizeof(double);
  // iteration 0 is the residual pass r0 = b - A x0 plus the start-up step
  auto enqueue = [&](int it) {
    const void* uin = it == 0 ? b : l.u;
    if (A.dtype == SNS_F64) launch_pass_v<double, 2>(A, p, l, uin, s);
    else launch_pass_v<float, 4>(A, p, l, uin, s);
    SNS_LAUNCH("lsqr_reduce", k_lsqr_reduce, dim3((n + 63) / 64, kRedSplit), dim3(256), 0, s, n,
               p.grid, st, l.zpart, l.npart, l.zred2, l.nred2);
    SNS_LAUNCH("lsqr_xtz", k_lsqr_xtz, dim3(gemv_grid), dim3(kGemvThreads), lds_xtz, s, n, sighat,
               l.Xc, l.zred2, l.nred2, st, nullptr, ybuf, l.ypart, v, wd, dy);
    SNS_LAUNCH("lsqr_xv", k_lsqr_xv, dim3(gemv_grid), dim3(kGemvThreads), lds_xv, s, n, l.Xr, v,
               static_cast<const double*>(nullptr), st, 1, wpass);
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
  // x = x0 + X dy
  SNS_LAUNCH("lsqr_final", k_lsqr_xv, dim3(gemv_grid), dim3(kGemvThreads), lds_xv, s, n, l.Xr, dy,
             static_cast<const double*>(q.xw), st, 0, x);
  SNS_LAUNCH("lsqr_report", k_lsqr_report, dim3(1), dim3(1), 0, s, st, info_dev);
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace sns
