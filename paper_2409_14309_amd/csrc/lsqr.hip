// SAP-SAS refinement: LSQR (Paige and Saunders 1982) on the right-
// preconditioned operator A X with X = R^{-1}, R from the QR of the sketch,
// starting from the sketch-and-solve answer x0 (sketch-and-precondition, as
// named in the paper's solver list).
//
// X is formed once per solve (k_tri_inv, fp64 back substitution per column)
// and applied as matrix-vector products: spread over many work-groups for
// n > 256, inside one work-group for smaller n (see below).  LSQR runs on the
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
// the scalar recurrences and the n-vector updates), k_lsqr_xv (w = X v).  For
// n <= 256 the last work-group of k_lsqr_reduce to finish runs the whole step
// after the reduction (both n x n products, the recurrences and the updates),
// so an iteration is two launches.
//
// Precision: A and the m-vector u are stored in A's dtype; every product and
// accumulation is fp64, and all n-vectors are fp64.  Once the stop rule
// holds, a flag in device memory makes the remaining launches return at once;
// for a single problem the device also posts the flag to pinned host memory
// after every iteration, so the host stops enqueuing without a copy.
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
  unsigned int arrived;  // work-groups of k_lsqr_xtz (or k_lsqr_reduce) done; reset by the last
  unsigned int steps;    // iterations launched so far, stopped ones included
};

// Stop state posted by the device into pinned host memory after every
// iteration of a single problem, so the host can poll without a copy.
constexpr int kPollSlots = 8;
struct PollSlot {
  double ratio;
  int done;  // done and step form one 64-bit word, written at once
  int step;  // solve epoch (high 16 bits) and iteration (low 16 bits) the slot describes
};
// The ring of one solve: its slots and the epoch that tags its posts, so
// that a post still in flight from an earlier solve never reads as current.
struct PollRef {
  PollSlot* slot;
  unsigned int epoch;
};
__host__ __device__ inline int poll_tag(unsigned int epoch, unsigned int step) {
  return (int)(((epoch & 0x7FFFu) << 16) | (step & 0xFFFFu));
}

namespace {

// v read from another lane of its 16-lane row by one data-parallel-primitive
// move (CTRL: a rotation, mirror or quad permutation); both 32-bit halves
// move the same way.
template <int CTRL>
__device__ __forceinline__ double dpp_move_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum of t over each aligned group of LPR lanes, in every lane of the group:
// a butterfly whose partner is at lane distance LPR / 2, ..., 2, 1 (every
// lane adds the same pairs in the same order, so all lanes hold the same
// bits).  Steps inside a 16-lane row are register moves: rotations by 8 and
// 4 (partners i ^ 8 and i ^ 4 once the earlier steps made the values
// periodic), the half-row mirror for groups of 8 (partner 7 - i), and quad
// permutations for i ^ 2 and i ^ 1; steps across rows are lane shuffles.
template <int LPR>
__device__ __forceinline__ double lanes_allsum(double t) {
  if constexpr (LPR >= 64) t += __shfl_xor(t, 32, 64);
  if constexpr (LPR >= 32) t += __shfl_xor(t, 16, 64);
  if constexpr (LPR >= 16) {
    t += dpp_move_f64<0x128>(t);  // row_ror:8
    t += dpp_move_f64<0x124>(t);  // row_ror:4
  } else if constexpr (LPR == 8) {
    t += dpp_move_f64<0x141>(t);  // row_half_mirror
  }
  if constexpr (LPR >= 4) t += dpp_move_f64<0x4E>(t);  // quad_perm [2, 3, 0, 1]
  if constexpr (LPR >= 2) t += dpp_move_f64<0xB1>(t);  // quad_perm [1, 0, 3, 2]
  return t;
}


constexpr int kRedSplit = 16;      // partial groups left for the step kernel
constexpr int kFuseMaxN = 256;     // n up to which k_lsqr_reduce also runs the step
constexpr int kRedThreads = 512;  // k_lsqr_reduce work-group (8 waves)
constexpr int kRedGroups = kRedThreads / 64;
constexpr int kFuseParts = kRedThreads / kFuseMaxN;  // threads per column in the fused step
static_assert(kFuseParts >= 1 && kRedGroups % 4 == 0, "combine orders below");

// A is read once per pass: nontemporal loads keep the stream from displacing
// u and the partial sums in the caches.
template <typename T, int VEC, int NCH, int LPR>
__device__ __forceinline__ void load_row_chunks(const T* __restrict__ row, int lr, int n,
                                                T (&a)[NCH][VEC]) {
  constexpr int CW = LPR * VEC;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int col = c * CW + lr * VEC;
    if (col + VEC <= n) {
      typedef T NVT __attribute__((ext_vector_type(VEC)));
      const NVT x = __builtin_nontemporal_load(reinterpret_cast<const NVT*>(row + col));
#pragma unroll
      for (int e = 0; e < VEC; ++e) a[c][e] = x[e];
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) a[c][e] = (col + e < n) ? row[col + e] : T(0);
    }
  }
}

// Fused pass over one work item (a contiguous row range of one problem): for
// each row i,
//   t = A[i,:] . w;  u'[i] = t - gamma * uin[i];  z += A[i,:]^T u'[i];
//   nrm += u'[i]^2.  Per-item z and nrm go to zpart / npart.  A row is spread
// over LPR lanes (NCH 16-byte chunks each); a work-group has W waves.  uin
// is b before the first step (the residual pass) and u afterwards.
template <typename T, int VEC, int LPR, int NCH, int U, int W>
__device__ __forceinline__ void lsqr_pass_item(const LsqrArgs& a, uint32_t loc, double* zred_,
                                               double* nred) {
  constexpr int RPW = 64 / LPR;
  constexpr int CW = LPR * VEC;  // columns per chunk
  constexpr int NSL = W * RPW;   // row slots per group
  double (*zred)[NCH * CW] = reinterpret_cast<double (*)[NCH * CW]>(zred_);
  const LsqrState* __restrict__ st = a.st;
  if (st->done) return;
  const double gamma = st->gamma;
  // SAA-SAS runs the residual pass on A and every later pass on Y = A X
  const bool onY = a.Y != nullptr && st->iter >= 0;
  const T* __restrict__ A = static_cast<const T*>(onY ? a.Y : a.A);
  const T* __restrict__ uin = static_cast<const T*>(st->iter < 0 ? a.b : a.u);
  T* __restrict__ uout = static_cast<T*>(a.u);
  const double* __restrict__ wv = a.vecs;  // w_pass
  const int64_t ld = onY ? a.ldy : a.ld, m = a.m;
  const int n = a.n;
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

  const int64_t r0 = m * (int64_t)loc / a.grid;
  const int64_t r1 = m * (int64_t)(loc + 1) / a.grid;
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
      t0 = lanes_allsum<LPR>(t0);
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
      t0 = lanes_allsum<LPR>(t0);
      t1 = lanes_allsum<LPR>(t1);
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
    for (int q = 0; q < W; ++q) s += zred[q][col];
    a.zpart[(size_t)loc * n + col] = s;
  }
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < W; ++q) s += nred[q];
    a.npart[loc] = s;
  }
}

template <typename T, int VEC, int LPR, int NCH, int U, int W>
__global__ __launch_bounds__(W * 64) void k_lsqr_pass(const LsqrArgs* __restrict__ P, Map mp) {
  constexpr int CW = LPR * VEC;
  __shared__ double zred[W * NCH * CW];
  __shared__ double nred[W];
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const int pi = map_find(mp, it);
  lsqr_pass_item<T, VEC, LPR, NCH, U, W>(P[pi], it - mp.off[pi], zred, nred);
}

// The stop state of the iteration just run, posted to the host ring (one
// thread of one work-group per iteration).  The stop flag and the step number
// travel in one 64-bit store, so the host never pairs a fresh tag with a stale
// flag; the ratio only steers how far the host runs ahead.
// `s` is the state as it now stands (a register copy or *st itself).
__device__ __forceinline__ void post_state(const LsqrState& s, LsqrState* st, PollRef ring) {
  const unsigned int k = s.steps;
  st->steps = k + 1u;
  PollSlot* h = ring.slot + k % kPollSlots;
  h->ratio = s.ratio;
  const unsigned long long tag =
      ((unsigned long long)(unsigned int)poll_tag(ring.epoch, k) << 32) |
      (unsigned long long)(unsigned int)s.done;
  *reinterpret_cast<unsigned long long*>(&h->done) = tag;
}

// Scalar recurrences and n-vector updates of one LSQR step, by one work-group,
// once y = Abar^T u' / beta - beta v (first step: Abar^T u' / beta) is
// complete in y[0, n): alpha = ||y||, v = y / alpha, the plane rotation, dy
// and wd.  `s` is every thread's register copy of the state, updated here and
// written back by thread 0 (no dependent loads of the state on this path).
// With vout (LDS), the new v is also left there.  Returns false, with the
// state marked failed, after a non-finite beta or alpha.
__device__ bool lsqr_update(const LsqrArgs& a, LsqrState& s, const double* y, double beta,
                            double alpha, bool first, double* vout) {
  LsqrState* __restrict__ st = a.st;
  const int n = a.n, t = threadIdx.x, nt = blockDim.x;
  const double sighat = a.sighat;
  double* v = a.vecs + n;
  double* wd = a.vecs + 2 * n;
  double* dy = a.vecs + 3 * n;
  if (!isfinite(beta) || !isfinite(alpha)) {
    s.status = SNS_ERR_NUMERICAL;
    s.done = 1;
    __syncthreads();
    if (t == 0) {
      st->status = s.status;
      st->done = 1;
    }
    return false;
  }
  const double inva = alpha > 0.0 ? 1.0 / alpha : 0.0;
  if (first) {
    // beta_1 u_1 = r0, alpha_1 v_1 = Abar^T u_1, wd_1 = v_1, phibar = beta_1, rhobar = alpha_1
    for (int j = t; j < n; j += nt) {
      const double vj = y[j] * inva;
      v[j] = vj;
      wd[j] = vj;
      dy[j] = 0.0;
      if (vout) vout[j] = vj;
    }
    s.beta = beta;
    s.alpha = alpha;
    s.phibar = beta;
    s.rhobar = alpha;
    s.iter = 0;
    s.gamma = beta > 0.0 ? alpha / beta : 0.0;
    s.ratio = sighat > 0.0 ? alpha / sighat : alpha;
    if (beta == 0.0 || alpha == 0.0 || s.max_iters <= 0) s.done = 1;
  } else {
    const double rhobar = s.rhobar, phibar = s.phibar;
    const double rho = hypot(rhobar, beta);
    const double c = rhobar / rho, sn = beta / rho;
    const double theta = sn * alpha;
    const double phi = c * phibar;
    const double f1 = phi / rho, f2 = theta / rho;
    for (int j = t; j < n; j += nt) {
      const double vj = y[j] * inva;
      const double wdj = wd[j];
      dy[j] += f1 * wdj;
      wd[j] = vj - f2 * wdj;
      v[j] = vj;
      if (vout) vout[j] = vj;
    }
    s.beta = beta;
    s.alpha = alpha;
    s.rhobar = -c * alpha;
    s.phibar = sn * phibar;
    s.iter += 1;
    s.gamma = beta > 0.0 ? alpha / beta : 0.0;
    const double ratio = alpha * fabs(c);
    s.ratio = sighat > 0.0 ? ratio / sighat : ratio;
    bool stop = beta == 0.0 || alpha == 0.0 || s.iter >= s.max_iters;
    if (s.stop > 0.0 && ratio <= s.stop) stop = true;
    if (stop) {
      s.done = 1;
      if (s.stop > 0.0 && ratio > s.stop && beta != 0.0 && alpha != 0.0)
        s.status = SNS_ERR_NOT_CONVERGED;
    }
  }
  __syncthreads();
  if (t == 0) {
    st->beta = s.beta;
    st->alpha = s.alpha;
    st->rhobar = s.rhobar;
    st->phibar = s.phibar;
    st->iter = s.iter;
    st->gamma = s.gamma;
    st->ratio = s.ratio;
    st->done = s.done;
    st->status = s.status;
  }
  return true;
}

// sum_j M[j * n + col] vec[j] over j in [j0, j1), one thread per column, in a
// fixed order (four running sums); consecutive threads read consecutive
// addresses.
__device__ __forceinline__ double col_dot(const double* __restrict__ M, int n, int col, int j0,
                                          int j1, const double* vec) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int j = j0;
  for (; j + 16 <= j1; j += 16) {
    double x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = M[(size_t)(j + k) * n + col];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k & 3] = fma(x[k], vec[j + k], acc[k & 3]);
  }
  for (int k = 0; j < j1; ++j, ++k) acc[k & 3] = fma(M[(size_t)j * n + col], vec[j], acc[k & 3]);
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// The whole step of a problem with n <= kFuseMaxN, run by the last work-group
// of k_lsqr_reduce to finish: z = A^T u' / beta from the reduction groups
// (agent-scope loads: other work-groups wrote them in this launch),
// y = X^T z - beta v (first step: X^T z; SAA-SAS after the residual pass:
// z - beta v), the update, then w = X v for the next pass (SAA-SAS: w = v).
// Each column's sums are split over kFuseParts threads (contiguous ranges of
// j, combined in a fixed order); the triangular products also run over the
// stored zeros of X up to the wave's column block, so every load is coalesced.
__device__ void lsqr_fused_step(const LsqrArgs& a, double* zs, double* ys,
                                double (*pp)[kFuseMaxN], double* red, PollRef ring) {
  LsqrState* __restrict__ st = a.st;
  LsqrState sc = *st;  // register copy, loaded once
  const int n = a.n, t = threadIdx.x;
  const int c = t % kFuseMaxN, q = t / kFuseMaxN;  // column, part
  const int wlo = c & ~63, whi = wlo + 64 < n ? wlo + 64 : n;  // this wave's column block
  double beta2 = 0.0;
  for (int s = 0; s < kRedSplit; ++s)
    beta2 += __hip_atomic_load(&a.nred2[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double beta = sqrt(beta2);
  const double invb = beta > 0.0 ? 1.0 / beta : 0.0;
  const bool first = sc.iter < 0;
  if (t < n) {
    double z = 0.0;
    for (int s = 0; s < kRedSplit; ++s)
      z += __hip_atomic_load(&a.zred2[(size_t)s * n + t], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    zs[t] = z * invb;
  }
  __syncthreads();
  const bool xtz = !(a.Y && !first);  // SAA-SAS after the residual pass: X^T is the identity
  if (xtz && c < n) {
    // X^T row c = X column c: Xr[j * n + c], nonzero for j <= c
    const int j0 = q * whi / kFuseParts, j1 = (q + 1) * whi / kFuseParts;
    pp[q][c] = col_dot(a.Xr, n, c, j0, j1, zs);
  }
  __syncthreads();
  double y = 0.0;
  if (t < n) {
    y = zs[t];
    if (xtz) {
      y = pp[0][t];
      for (int k = 1; k < kFuseParts; ++k) y += pp[k][t];
    }
    if (!first) y -= beta * a.vecs[n + t];
    ys[t] = y;
  }
  const double alpha = sqrt(block_sum(y * y, red));
  if (lsqr_update(a, sc, ys, beta, alpha, first, zs)) {
    if (!a.Y && c < n) {
      // X row c: Xc[j * n + c], nonzero for j >= c
      const int len = n - wlo;
      const int j0 = wlo + q * len / kFuseParts, j1 = wlo + (q + 1) * len / kFuseParts;
      pp[q][c] = col_dot(a.Xc, n, c, j0, j1, zs);
    }
    __syncthreads();
    if (t < n) {
      double w = zs[t];
      if (!a.Y) {
        w = pp[0][t];
        for (int k = 1; k < kFuseParts; ++k) w += pp[k][t];
      }
      a.vecs[t] = w;
    }
  }
  if (t == 0) {
    st->arrived = 0u;
    if (ring.slot) post_state(sc, st, ring);
  }
}

// First level of the reduction of the G per-group partials: item (cx, s)
// sums partials [s G / S, (s+1) G / S) for columns [64 cx, 64 cx + 64) into
// zred2[s][.] (and, for cx = 0, the norms into nred2[s]).  Sixteen thread
// groups take every sixteenth partial, each with eight running sums (partials
// g, g + 16, ..., g + 112 of a round of 128); all sums are combined in a fixed
// order.  For n <= kFuseMaxN the results go to device-coherent memory
// directly and the last item of the problem to finish runs the step.
__device__ __forceinline__ void lsqr_reduce_item(const LsqrArgs& a, uint32_t loc,
                                                 double (*part)[64], double* red, double* zs,
                                                 double* ys, double (*pp)[kFuseMaxN], int* last,
                                                 PollRef ring) {
  const bool fused = a.n <= kFuseMaxN;
  if (a.st->done) {
    if (fused && ring.slot && loc == 0 && threadIdx.x == 0) post_state(*a.st, a.st, ring);
    return;
  }
  const int n = a.n, G = a.grid;
  const uint32_t cxn = (uint32_t)((n + 63) / 64);
  const int cx = (int)(loc % cxn), s = (int)(loc / cxn);
  const int t = threadIdx.x, cl = t & 63, grp = t >> 6;
  const int g0 = (int)((int64_t)G * s / kRedSplit), g1 = (int)((int64_t)G * (s + 1) / kRedSplit);
  const int col = cx * 64 + cl;
  const double* __restrict__ zpart = a.zpart;
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  if (col < n) {
    int g = g0 + grp;
    for (; g + 7 * kRedGroups < g1; g += 8 * kRedGroups) {
      double v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = zpart[(size_t)(g + kRedGroups * k) * n + col];
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[k] += v[k];
    }
    for (int k = 0; g < g1; g += kRedGroups, ++k) acc[k] += zpart[(size_t)g * n + col];
  }
  part[grp][cl] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (t < 64 && col < n) {
    double zr = 0.0;
#pragma unroll
    for (int k = 0; k < kRedGroups; k += 4)
      zr += (part[k][t] + part[k + 1][t]) + (part[k + 2][t] + part[k + 3][t]);
    if (fused)
      __hip_atomic_store(&a.zred2[(size_t)s * n + col], zr, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    else
      a.zred2[(size_t)s * n + col] = zr;
  }
  if (cx == 0) {
    double q = 0.0;
    for (int g = g0 + t; g < g1; g += kRedThreads) q += a.npart[g];
    q = block_sum(q, red);
    if (t == 0) {
      if (fused) __hip_atomic_store(&a.nred2[s], q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else a.nred2[s] = q;
    }
  }
  if (!fused) return;
  // every wave's stores complete before the item reports its arrival
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (t == 0) *last = atomicAdd(&a.st->arrived, 1u) == cxn * kRedSplit - 1u ? 1 : 0;
  __syncthreads();
  if (*last) lsqr_fused_step(a, zs, ys, pp, red, ring);
}

__global__ __launch_bounds__(kRedThreads) void k_lsqr_reduce(const LsqrArgs* __restrict__ P,
                                                             Map mp, PollRef ring) {
  __shared__ double part[kRedGroups][64];
  __shared__ double red[kRedGroups];
  __shared__ double zs[kFuseMaxN], ys[kFuseMaxN];
  __shared__ double pp[kFuseParts][kFuseMaxN];
  __shared__ int last;
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const int pi = map_find(mp, it);
  lsqr_reduce_item(P[pi], it - mp.off[pi], part, red, zs, ys, pp, &last, ring);
}

__global__ void k_lsqr_init(const LsqrArgs* __restrict__ P, Map mp) {
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const LsqrArgs& a = P[map_find(mp, it)];
  const int n = a.n;
  double* wpass = a.vecs;
  double* dy = a.vecs + 3 * n;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    wpass[j] = -a.x0[j];
    dy[j] = 0.0;
  }
  if (threadIdx.x == 0) {
    LsqrState* st = a.st;
    st->alpha = st->beta = st->rhobar = st->phibar = 0.0;
    st->gamma = -1.0;
    st->ratio = 0.0;
    st->stop = a.stop;
    st->iter = -1;  // the next step consumes the residual pass
    st->max_iters = a.max_iters;
    st->done = a.max_iters <= 0 ? 1 : 0;
    st->status = SNS_OK;
    st->arrived = 0u;
    st->steps = 0u;
  }
}

// X = R^{-1}: item j solves R x = e_j on the leading (j+1) x (j+1) block by
// back substitution and writes column j of X (column-major Xc and row-major
// Xr; X is upper triangular).
constexpr int kInvThreads = 256;
__global__ __launch_bounds__(kInvThreads) void k_tri_inv(const LsqrArgs* __restrict__ P, Map mp) {
  extern __shared__ double sh[];
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const int pi = map_find(mp, it);
  const LsqrArgs& a = P[pi];
  const int n = a.n;
  const int j = (int)(it - mp.off[pi]);
  double* x = sh;        // n
  double* blk = sh + n;  // 64 x 64
  for (int i = threadIdx.x; i < n; i += kInvThreads) x[i] = i == j ? 1.0 : 0.0;
  __syncthreads();
  trsv_lds<true, kInvThreads>(a.Rc, n, j + 1, a.invd, x, blk);
  for (int i = threadIdx.x; i < n; i += kInvThreads) {
    const double v = i <= j ? x[i] : 0.0;
    a.Xc[(int64_t)j * n + i] = v;
    a.Xr[(int64_t)i * n + j] = v;
  }
}

constexpr int kGemvThreads = 512;
constexpr int kGemvRows = 8;   // rows per work item (one per wave)

// Dot product of row i of a triangular matrix stored row-contiguously
// (M[i * n + j]) with vec over j in [j0, j1), by one wave; all lanes get it.
// Each lane takes the entries j0 + lane, j0 + lane + 64, ... with eight
// loads in flight and four running sums, combined in a fixed order.
__device__ __forceinline__ double wave_row_dot(const double* __restrict__ M, int n, int i, int j0,
                                               int j1, const double* __restrict__ vec) {
  const int lane = threadIdx.x & 63;
  const double* row = M + (int64_t)i * n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int j = j0 + lane;
  for (; j + 7 * 64 < j1; j += 8 * 64) {
    double x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = row[j + 64 * k];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k & 3] = fma(x[k], vec[j + 64 * k], acc[k & 3]);
  }
  for (int k = 0; j < j1; j += 64, ++k) acc[k & 3] = fma(row[j], vec[j], acc[k & 3]);
  return wave_sum((acc[0] + acc[1]) + (acc[2] + acc[3]));
}

// y = X^T (z / beta) - beta v (first step: X^T (z / beta)), z = sum of the
// reduction splits.  X^T row i = X column i = Xc[i * n + j], j <= i.  Each
// item writes its rows of y and its share of ||y||^2; the last item of the
// problem to finish (arrival counter) then runs the scalar recurrences and
// the n-vector updates for the whole vector in a fixed order.
__device__ __forceinline__ void lsqr_xtz_item(const LsqrArgs& a, uint32_t loc, double* sh,
                                              bool* last, PollRef ring) {
  if (a.n <= kFuseMaxN) return;  // the step ran in k_lsqr_reduce
  LsqrState* __restrict__ st = a.st;
  if (st->done) {
    if (ring.slot && loc == 0 && threadIdx.x == 0) post_state(*st, st, ring);
    return;
  }
  const int n = a.n;
  const uint32_t nitems = (uint32_t)((n + kGemvRows - 1) / kGemvRows);
  double* z = sh;        // n
  double* red = sh + n;  // 16 + kGemvRows
  const double* v = a.vecs + n;
  double* ybuf = a.vecs + 4 * n;
  const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, wv = t >> 6;
  double beta2 = 0.0;
  for (int s = 0; s < kRedSplit; ++s) beta2 += a.nred2[s];
  const double beta = sqrt(beta2);
  const double invb = beta > 0.0 ? 1.0 / beta : 0.0;
  const bool first = st->iter < 0;
  for (int j = t; j < n; j += nt) {
    double q = 0.0;
    for (int s = 0; s < kRedSplit; ++s) q += a.zred2[(size_t)s * n + j];
    z[j] = q * invb;
  }
  __syncthreads();
  double ysq = 0.0;
  for (int r = wv; r < kGemvRows; r += nt / 64) {
    const int i = (int)loc * kGemvRows + r;
    if (i < n) {
      // after the residual pass, SAA-SAS works on Y itself: X^T is the identity
      double yi = (a.Y && !first) ? z[i] : wave_row_dot(a.Xc, n, i, 0, i + 1, z);
      if (!first) yi -= beta * v[i];
      if (lane == 0) red[16 + r] = yi;
    } else if (lane == 0) {
      red[16 + r] = 0.0;
    }
  }
  __syncthreads();
  if (t == 0) {
    // thread 0 stores the item's rows of y, so its release fence covers them
    for (int r = 0; r < kGemvRows; ++r) {
      const double yi = red[16 + r];
      const int i = (int)loc * kGemvRows + r;
      if (i < n) ybuf[i] = yi;
      ysq += yi * yi;
    }
    a.ypart[loc] = ysq;
    __threadfence();
    const unsigned int prev = atomicAdd(&st->arrived, 1u);
    *last = prev == nitems - 1;
  }
  __syncthreads();
  if (!*last) return;
  __threadfence();
  // ---- last item: scalars and n-vector updates ----
  // the items' partial norms are loaded together into LDS (z is no longer
  // needed), then summed in item order: the same value on every thread
  for (uint32_t g = t; g < nitems; g += nt) z[g] = a.ypart[g];
  __syncthreads();
  double a2 = 0.0;
  for (uint32_t g = 0; g < nitems; ++g) a2 += z[g];
  LsqrState sc = *st;
  (void)lsqr_update(a, sc, ybuf, beta, sqrt(a2), first, nullptr);
  if (t == 0) {
    st->arrived = 0u;
    if (ring.slot) post_state(sc, st, ring);
  }
}

__global__ __launch_bounds__(kGemvThreads) void k_lsqr_xtz(const LsqrArgs* __restrict__ P,
                                                           Map mp, PollRef ring) {
  extern __shared__ double sh[];
  __shared__ bool last;
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const int pi = map_find(mp, it);
  lsqr_xtz_item(P[pi], it - mp.off[pi], sh, &last, ring);
}

// mode 0: w_pass = X v for the next pass (skipped once the problem stopped);
// mode 1: x = x0 + X dy.  Row i of X = Xr[i * n + j], j >= i.
__device__ __forceinline__ void lsqr_xv_item(const LsqrArgs& a, uint32_t loc, int mode,
                                             double* vec) {
  if (mode == 0 && (a.st->done || a.n <= kFuseMaxN)) return;  // small n: done in k_lsqr_reduce
  const int n = a.n;
  const double* vin = mode == 0 ? a.vecs + n : a.vecs + 3 * n;
  double* out = mode == 0 ? a.vecs : a.x;
  const double* add0 = mode == 0 ? nullptr : a.x0;
  const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, wv = t >> 6;
  for (int j = t; j < n; j += nt) vec[j] = vin[j];
  __syncthreads();
  for (int r = wv; r < kGemvRows; r += nt / 64) {
    const int i = (int)loc * kGemvRows + r;
    if (i < n) {
      // the passes after the residual pass read Y = A X under SAA-SAS
      const double wi = (mode == 0 && a.Y) ? vec[i] : wave_row_dot(a.Xr, n, i, i, n, vec);
      if (lane == 0) out[i] = add0 ? add0[i] + wi : wi;
    }
  }
}

__global__ __launch_bounds__(kGemvThreads) void k_lsqr_xv(const LsqrArgs* __restrict__ P, Map mp,
                                                          int mode) {
  extern __shared__ double sh[];
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const int pi = map_find(mp, it);
  lsqr_xv_item(P[pi], it - mp.off[pi], mode, sh);
}

__global__ void k_lsqr_report(const LsqrArgs* __restrict__ P, Map mp) {
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const LsqrArgs& a = P[map_find(mp, it)];
  if (threadIdx.x != 0) return;
  const LsqrState* st = a.st;
  sns_info* info = a.info;
  info->iters = st->iter < 0 ? 0 : st->iter;
  info->rel_resid_est = st->ratio;
  if (info->status == SNS_OK) info->status = st->status;
}

// out[p] = 1 once problem p has stopped.
__global__ void k_lsqr_flags(const LsqrArgs* __restrict__ P, int nprob, int* __restrict__ out) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nprob; p += gridDim.x * blockDim.x)
    out[p] = P[p].st->done ? 1 : 0;
}

// Number of problems not yet stopped.
__global__ void k_lsqr_active(const LsqrArgs* __restrict__ P, int nprob, int* __restrict__ out) {
  __shared__ int red[4];
  int c = 0;
  for (int p = threadIdx.x; p < nprob; p += blockDim.x) c += P[p].st->done ? 0 : 1;
  c = block_sum(c, red);
  if (threadIdx.x == 0) *out = c;
}

template <typename T, int VEC, int LPR, int NCH, int U, int W>
void launch_pass_t(const LsqrJob::Cls& c, hipStream_t s) {
  SNS_LAUNCH("lsqr_pass", (k_lsqr_pass<T, VEC, LPR, NCH, U, W>), dim3(grid_for(c.items)),
             dim3(W * 64), 0, s, c.args, c.map);
}

template <typename T, int VEC, int U, int W>
void launch_pass_u(const LsqrJob::Cls& c, hipStream_t s) {
  switch (c.plan.lpr * 16 + c.plan.nch) {
    case 4 * 16 + 1: launch_pass_t<T, VEC, 4, 1, U, W>(c, s); break;
    case 4 * 16 + 2: launch_pass_t<T, VEC, 4, 2, U, W>(c, s); break;
    case 4 * 16 + 4: launch_pass_t<T, VEC, 4, 4, U, W>(c, s); break;
    case 8 * 16 + 4: launch_pass_t<T, VEC, 8, 4, U, W>(c, s); break;
    case 16 * 16 + 1: launch_pass_t<T, VEC, 16, 1, U, W>(c, s); break;
    case 16 * 16 + 2: launch_pass_t<T, VEC, 16, 2, U, W>(c, s); break;
    case 16 * 16 + 4: launch_pass_t<T, VEC, 16, 4, U, W>(c, s); break;
    case 32 * 16 + 1: launch_pass_t<T, VEC, 32, 1, U, W>(c, s); break;
    case 32 * 16 + 2: launch_pass_t<T, VEC, 32, 2, U, W>(c, s); break;
    case 32 * 16 + 4: launch_pass_t<T, VEC, 32, 4, U, W>(c, s); break;
    case 64 * 16 + 1: launch_pass_t<T, VEC, 64, 1, U, W>(c, s); break;
    case 64 * 16 + 2: launch_pass_t<T, VEC, 64, 2, U, W>(c, s); break;
    case 64 * 16 + 4: launch_pass_t<T, VEC, 64, 4, U, W>(c, s); break;
    default: launch_pass_t<T, VEC, 64, 8, U, W>(c, s); break;
  }
}

template <typename T, int VEC, int W>
void launch_pass_w(const LsqrJob::Cls& c, hipStream_t s) {
  if (c.plan.unroll == 2) launch_pass_u<T, VEC, 2, W>(c, s);
  else launch_pass_u<T, VEC, 1, W>(c, s);
}

// Work-groups of 4 or 8 waves (plan.waves): 8 suit large problems (more rows
// in flight per compute unit), 4 the small ones, whose work-groups would
// otherwise hold more row slots than rows.
template <typename T, int VEC>
void launch_pass_v(const LsqrJob::Cls& c, hipStream_t s) {
  if (c.plan.waves == 8) launch_pass_w<T, VEC, 8>(c, s);
  else launch_pass_w<T, VEC, 4>(c, s);
}

}  // namespace

// Plan: lanes per row (lpr) and 16-byte column chunks per lane (nch) such
// that lpr * nch * (16 / element size) covers n; work-groups of the pass.
// SNS_LSQR_PLAN="lpr,nch,grid,unroll[,waves]" overrides the choice (tuning runs);
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
  p.waves = 4;
  LsqrPlan t;
  if (tune_lookup(A.dtype, n, A.m, &t) && lsqr_plan_valid(t.lpr, t.nch) &&
      (int64_t)t.lpr * t.nch * vw >= n && t.grid >= 1 && t.grid <= 65535 &&
      (t.unroll == 1 || t.unroll == 2) && (t.waves == 4 || t.waves == 8))
    p = t;
  if (const char* e = getenv("SNS_LSQR_PLAN")) {
    int a = 0, b = 0, c = 0, d = 1, w = 4;
    if (sscanf(e, "%d,%d,%d,%d,%d", &a, &b, &c, &d, &w) >= 3) {
      if (lsqr_plan_valid(a, b) && (int64_t)a * b * vw >= n && c >= 1 && c <= 65535) {
        p.lpr = a;
        p.nch = b;
        p.grid = c;
        p.unroll = d == 2 ? 2 : 1;
        p.waves = w == 8 ? 8 : 4;
      }
    }
  }
  return p;
}

bool lsqr_plan_valid(int lpr, int nch) {
  switch (lpr) {
    case 4: return nch == 1 || nch == 2 || nch == 4;
    case 8: return nch == 4;
    case 16:
    case 32: return nch == 1 || nch == 2 || nch == 4;
    case 64: return nch == 1 || nch == 2 || nch == 4 || nch == 8;
    default: return false;
  }
}

constexpr int kTuneMaxGrid = 4096;

size_t tune_workspace_bytes(const sns_matrix& A) {
  const size_t es = A.dtype == SNS_F64 ? 8 : 4;
  Carve c(nullptr, 0);
  c.take<char>((size_t)A.m * es);
  c.take<double>((size_t)kTuneMaxGrid * A.n);
  c.take<double>((size_t)kTuneMaxGrid);
  c.take<double>((size_t)6 * A.n);
  c.take<LsqrState>(1);
  c.take<char>(4096);
  return c.off;
}

sns_status time_lsqr_pass(const sns_matrix& A, const LsqrPlan& p, int reps, void* ws,
                          size_t ws_bytes, hipStream_t st, double* us) {
  if (!lsqr_plan_valid(p.lpr, p.nch) || p.grid < 1 || p.grid > kTuneMaxGrid || reps < 1)
    return SNS_ERR_INVALID_ARG;
  const size_t es = A.dtype == SNS_F64 ? 8 : 4;
  const int n = (int)A.n;
  Carve c(ws, ws_bytes);
  LsqrBufs l{};
  l.u = c.take<char>((size_t)A.m * es);
  l.zpart = c.take<double>((size_t)kTuneMaxGrid * n);
  l.npart = c.take<double>((size_t)kTuneMaxGrid);
  l.vecs = c.take<double>((size_t)6 * n);
  l.state = c.take<LsqrState>(1);
  char* args = c.take<char>(4096);
  if (!c.ok()) return SNS_ERR_OUT_OF_MEMORY;
  LsqrState h{};
  h.gamma = 0.5;
  h.iter = 0;  // reads u, not b
  h.max_iters = 1 << 30;
  SNS_HIP_TRY(hipMemcpyAsync(l.state, &h, sizeof(h), hipMemcpyHostToDevice, st));
  SNS_HIP_TRY(hipMemsetAsync(l.u, 0, (size_t)A.m * es, st));
  SNS_HIP_TRY(hipMemsetAsync(l.vecs, 0, sizeof(double) * 6 * n, st));
  LsqrArgs a{};
  a.A = A.values;
  a.ld = A.ld;
  a.m = A.m;
  a.n = n;
  a.grid = p.grid;
  a.b = l.u;
  a.u = l.u;
  a.zpart = l.zpart;
  a.npart = l.npart;
  a.vecs = l.vecs;
  a.st = static_cast<LsqrState*>(l.state);
  ArgTable t(args);
  const LsqrJob j = build_lsqr_job(t, std::vector<LsqrProb>{LsqrProb{p, a}}, A.dtype == SNS_F64);
  if (t.bytes() > 4096) return SNS_ERR_OUT_OF_MEMORY;
  sns_status e = t.upload(st);
  if (e != SNS_OK) return e;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SNS_HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SNS_ERR_HIP;
  }
  auto pass = [&]() {
    if (j.f64) launch_pass_v<double, 2>(j.cls[0], st);
    else launch_pass_v<float, 4>(j.cls[0], st);
  };
  pass();
  float ms = 0.f;
  hipError_t he = hipEventRecord(e0, st);
  for (int r = 0; r < reps && he == hipSuccess; ++r) pass();
  if (he == hipSuccess) he = hipEventRecord(e1, st);
  if (he == hipSuccess) he = hipEventSynchronize(e1);
  if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  SNS_HIP_TRY(he);
  SNS_HIP_TRY(hipGetLastError());
  *us = 1000.0 * ms / reps;  // host h stayed alive until the synchronisation above
  return SNS_OK;
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

LsqrArgs lsqr_args(const sns_matrix& A, const void* b, const LsqrPlan& p, const LsqrBufs& l,
                   const QrBufs& q, int d, int max_iters, double rtol, double* x,
                   sns_info* info, const void* Y, int64_t ldy) {
  LsqrArgs a;
  const int n = (int)A.n;
  a.A = A.values;
  a.ld = A.ld;
  a.m = A.m;
  a.n = n;
  a.grid = p.grid;
  a.max_iters = max_iters;
  a.b = b;
  a.u = l.u;
  a.zpart = l.zpart;
  a.npart = l.npart;
  a.zred2 = l.zred2;
  a.nred2 = l.nred2;
  a.Xc = l.Xc;
  a.Xr = l.Xr;
  a.ypart = l.ypart;
  a.vecs = l.vecs;
  a.st = static_cast<LsqrState*>(l.state);
  a.Rc = q.R;
  a.invd = q.invd;
  a.x0 = q.xw;
  a.x = x;
  a.info = info;
  a.sighat = 1.0 - sqrt((double)n / (double)d);
  a.stop = rtol > 0.0 ? rtol * (a.sighat > 0.0 ? a.sighat : 1.0) : 0.0;
  a.Y = Y;
  a.ldy = ldy;
  return a;
}

LsqrJob build_lsqr_job(ArgTable& t, const std::vector<LsqrProb>& p, bool f64) {
  LsqrJob j;
  j.f64 = f64;
  j.count = (int)p.size();
  if (p.empty()) return j;
  std::vector<LsqrArgs> all;
  std::vector<uint32_t> one, inv, red, gemv;
  for (const LsqrProb& x : p) {
    all.push_back(x.args);
    const int n = x.args.n;
    one.push_back(1u);
    inv.push_back((uint32_t)n);
    red.push_back((uint32_t)(((n + 63) / 64) * kRedSplit));
    gemv.push_back((uint32_t)((n + kGemvRows - 1) / kGemvRows));
    j.maxn = n > j.maxn ? n : j.maxn;
    if (n > kFuseMaxN) j.unfused = true;
  }
  j.all = t.add(all.data(), all.size());
  uint32_t tmp = 0;
  j.mone = t.map(one, &tmp);
  j.minv = t.map(inv, &j.ninv);
  j.mred = t.map(red, &j.nred);
  j.mgemv = t.map(gemv, &j.ngemv);
  std::vector<bool> used(p.size(), false);
  for (size_t i = 0; i < p.size(); ++i) {
    if (used[i]) continue;
    LsqrJob::Cls c;
    c.plan = p[i].plan;
    std::vector<LsqrArgs> sub;
    std::vector<uint32_t> cnt;
    for (size_t k = i; k < p.size(); ++k) {
      const LsqrPlan& q = p[k].plan;
      if (used[k] || q.lpr != c.plan.lpr || q.nch != c.plan.nch || q.unroll != c.plan.unroll ||
          q.waves != c.plan.waves)
        continue;
      used[k] = true;
      sub.push_back(p[k].args);
      cnt.push_back((uint32_t)p[k].args.grid);
    }
    c.args = t.add(sub.data(), sub.size());
    c.map = t.map(cnt, &c.items);
    j.cls.push_back(c);
  }
  if (p.size() == 1) {
    j.state = p[0].args.st;
    j.stop = p[0].args.stop;
    j.sighat = p[0].args.sighat;
  }
  return j;
}

sns_status launch_lsqr_setup(const LsqrJob& j, hipStream_t s) {
  if (j.count == 0) return SNS_OK;
  SNS_LAUNCH("lsqr_init", k_lsqr_init, dim3(grid_for((uint32_t)j.count)), dim3(256), 0, s, j.all,
             j.mone);
  SNS_LAUNCH("tri_inv", k_tri_inv, dim3(grid_for(j.ninv)), dim3(kInvThreads),
             ((size_t)j.maxn + 4096) * sizeof(double), s, j.all, j.minv);
  SNS_HIP_TRY(hipGetLastError());
  return launch_form_y(j.saa, s);
}

sns_status launch_lsqr_iteration(const LsqrJob& j, hipStream_t s, PollSlot* ring,
                                  unsigned int epoch) {
  if (j.count == 0) return SNS_OK;
  for (const LsqrJob::Cls& c : j.cls) {
    if (j.f64) launch_pass_v<double, 2>(c, s);
    else launch_pass_v<float, 4>(c, s);
  }
  const PollRef r{j.count == 1 ? ring : nullptr, epoch};
  SNS_LAUNCH("lsqr_reduce", k_lsqr_reduce, dim3(grid_for(j.nred)), dim3(kRedThreads), 0, s, j.all,
             j.mred, r);
  if (j.unfused) {
    SNS_LAUNCH("lsqr_xtz", k_lsqr_xtz, dim3(grid_for(j.ngemv)), dim3(kGemvThreads),
               ((size_t)j.maxn + 16 + kGemvRows) * sizeof(double), s, j.all, j.mgemv, r);
    SNS_LAUNCH("lsqr_xv", k_lsqr_xv, dim3(grid_for(j.ngemv)), dim3(kGemvThreads),
               (size_t)j.maxn * sizeof(double), s, j.all, j.mgemv, 0);
  }
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

sns_status launch_lsqr_finish(const LsqrJob& j, hipStream_t s) {
  if (j.count == 0) return SNS_OK;
  SNS_LAUNCH("lsqr_final", k_lsqr_xv, dim3(grid_for(j.ngemv)), dim3(kGemvThreads),
             (size_t)j.maxn * sizeof(double), s, j.all, j.mgemv, 1);
  SNS_LAUNCH("lsqr_report", k_lsqr_report, dim3(grid_for((uint32_t)j.count)), dim3(64), 0, s,
             j.all, j.mone);
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

sns_status launch_lsqr_active(const LsqrJob& j, int* out, hipStream_t s) {
  SNS_LAUNCH("lsqr_active", k_lsqr_active, dim3(1), dim3(256), 0, s, j.all, j.count, out);
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

sns_status launch_lsqr_flags(const LsqrJob& j, int* out, hipStream_t s) {
  if (j.count == 0) return SNS_OK;
  SNS_LAUNCH("lsqr_flags", k_lsqr_flags, dim3((j.count + 255) / 256), dim3(256), 0, s, j.all,
             j.count, out);
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

namespace {

// Host-side view of the device stop state: pinned slots that k_lsqr_xtz
// writes after every iteration of a single problem, one event per slot.
struct PollRing {
  PollSlot* slot = nullptr;  // pinned host memory
  hipEvent_t ev[kPollSlots] = {};
  unsigned int epoch = 0;  // solves that used the ring on this thread
  bool ok = false;
  PollRing() {
    if (hipHostMalloc((void**)&slot, sizeof(PollSlot) * kPollSlots, hipHostMallocDefault) !=
        hipSuccess)
      return;
    for (int i = 0; i < kPollSlots; ++i) {
      slot[i].done = 0;
      slot[i].step = -1;
      if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) return;
    }
    ok = true;
  }
};

PollRing& poll_ring() {
  thread_local PollRing r;
  return r;
}

}  // namespace

// One problem: set-up, iterations, final update.  Iteration 0 is the
// residual pass r0 = b - A x0 plus the start-up step.  With `adaptive`, the
// host reads the device stop state while at most two iterations are in
// flight; otherwise all max_iters + 1 steps are enqueued and the ones after
// the stop rule return at once.
sns_status run_lsqr_single(const LsqrJob& j, int max_iters, bool adaptive, hipStream_t s) {
  sns_status e = launch_lsqr_setup(j, s);
  if (e != SNS_OK) return e;
  const LsqrState* st = j.state;
  const double stop = j.stop;
  const double sighat = j.sighat;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  SNS_HIP_TRY(hipStreamIsCapturing(s, &cap));
  PollRing& ring = poll_ring();
  if (!adaptive || !st || cap != hipStreamCaptureStatusNone || stop == 0.0 || !ring.ok) {
    for (int it = 0; it <= max_iters; ++it)
      if ((e = launch_lsqr_iteration(j, s)) != SNS_OK) return e;
  } else {
    // Keep at most two iterations in flight.  Before running ahead of an
    // unread iteration, predict from the geometric decay of the stop ratio
    // whether that iteration converges; if so, wait for it instead, so that no
    // launch is issued after the stop rule has fired.
    const int K = kPollSlots;
    const unsigned int epoch = ++ring.epoch;
    // the {done, step} word of slot k (low half done, high half step)
    auto tag = [&](int k) -> volatile unsigned long long& {
      return *reinterpret_cast<volatile unsigned long long*>(&ring.slot[k].done);
    };
    // Iteration it: clear its slot's step tag, launch, mark with an event.
    auto launch = [&](int it) {
      tag(it % K) = 0xFFFFFFFF00000000ull;
      sns_status r = launch_lsqr_iteration(j, s, ring.slot, epoch);
      if (r != SNS_OK) return r;
      SNS_HIP_TRY(hipEventRecord(ring.ev[it % K], s));
      return SNS_OK;
    };
    double r_prev = -1.0, r_last = -1.0;
    bool done = false;
    int known = -1;  // last iteration whose state has been read
    auto read = [&](int it) {
      SNS_HIP_TRY(hipEventSynchronize(ring.ev[it % K]));
      // the slot normally carries the iteration's tag once its event is done;
      // allow the posted write a moment, then read the device state instead
      const int want = poll_tag(epoch, (unsigned int)it);
      unsigned long long w = tag(it % K);
      for (int spin = 0; (int)(w >> 32) != want && spin < 100000; ++spin) w = tag(it % K);
      double ratio;
      if ((int)(w >> 32) == want) {
        done = (unsigned int)w != 0u;
        ratio = *reinterpret_cast<volatile double*>(&ring.slot[it % K].ratio);
      } else {
        LsqrState d;
        SNS_HIP_TRY(hipStreamSynchronize(s));
        SNS_HIP_TRY(hipMemcpy(&d, st, sizeof(d), hipMemcpyDeviceToHost));
        done = d.done != 0;
        ratio = d.ratio;
      }
      r_prev = r_last;
      r_last = ratio * (sighat > 0.0 ? sighat : 1.0);
      known = it;
      return SNS_OK;
    };
    if ((e = launch(0)) != SNS_OK) return e;
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
      if ((e = launch(next)) != SNS_OK) return e;
      ++next;
      if (known < next - 2) {
        if ((e = read(next - 2)) != SNS_OK) return e;
        if (done) break;
      }
    }
  }
  return launch_lsqr_finish(j, s);
}

}  // namespace sns
