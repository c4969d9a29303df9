// Single-work-group fp64 building blocks used by the QR and LSQR kernels:
// multi-value wave reductions and triangular solves with R (n x n upper
// triangular, column-major, leading dimension ld) on a vector held in LDS.
#pragma once

#include "common.hpp"

namespace sns {

// v moved by one data-parallel-primitive step (row shift or row broadcast,
// `ctrl`), rows outside row_mask and lanes without a source read 0.  Both
// 32-bit halves move the same way.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Sum over each aligned group of G lanes (G a power of two <= 64); the total
// is in the group's last lane (other lanes hold partial sums).  Register-only
// steps in a fixed order: shifts by 1, 2, 4, 8 inside 16-lane rows, then the
// last lane of row 0 (2) is added into row 1 (3), and lane 31 into rows 2-3.
template <int G>
__device__ __forceinline__ double group_sum_last(double s) {
  if constexpr (G >= 2) s += dpp_f64<0x111, 0xF>(s);   // row_shr:1
  if constexpr (G >= 4) s += dpp_f64<0x112, 0xF>(s);   // row_shr:2
  if constexpr (G >= 8) s += dpp_f64<0x114, 0xF>(s);   // row_shr:4
  if constexpr (G >= 16) s += dpp_f64<0x118, 0xF>(s);  // row_shr:8
  if constexpr (G >= 32) s += dpp_f64<0x142, 0xA>(s);  // row_bcast:15 into rows 1, 3
  if constexpr (G >= 64) s += dpp_f64<0x143, 0xC>(s);  // row_bcast:31 into rows 2, 3
  return s;
}

// Sum NB values per thread over a work-group of NT threads; tot[0..NB) (LDS)
// gets the totals, visible to all threads on return.  red: LDS of NB * NT
// doubles.  The values are transposed through LDS: value c is summed by the
// P = NT / NB consecutive threads of group c, thread p adding the stored
// entries p, p + P, ..., p + (NB - 1) P in order (consecutive lanes read
// consecutive words, so the reads are free of bank conflicts), and the group
// finishes with register-only lane steps (group_sum_last) over its P lanes.
// When P exceeds a wave, wave c alone sums value c (NT / 64 entries per
// lane), so the reduction still takes two barriers.
// The order is fixed, so the result is reproducible.
template <int NB, int NT>
__device__ __forceinline__ void block_reduce_multi(const double (&g)[NB], double* red,
                                                   double* tot) {
  static_assert((NB & (NB - 1)) == 0 && NB <= NT && NT % 64 == 0, "NB power of two");
  constexpr int P = NT / NB;
  constexpr int PW = P < 64 ? P : 64;  // lanes of one group inside a wave
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < NB; ++c) red[c * NT + t] = g[c];
  __syncthreads();
  if constexpr (P <= 64) {
    const int c = t / P, p = t % P;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NB; ++q) s += red[c * NT + q * P + p];
    s = group_sum_last<PW>(s);
    if (p == P - 1) tot[c] = s;
  } else {
    // more than a wave per value: wave c alone sums value c, lane l adding
    // the stored entries l, l + 64, ... in order, then the lanes
    const int wv = t >> 6, l = t & 63;
    if (wv < NB) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < NT / 64; ++q) s += red[wv * NT + q * 64 + l];
      s = group_sum_last<64>(s);
      if (l == 63) tot[wv] = s;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Triangular solve in place on a vector x in LDS (length n) by one work-group
// of NT threads, 64 unknowns at a time.  `C` is the triangular factor in
// column-major order with leading dimension ld, `invd` the reciprocals of its
// diagonal.
//   UPPER = true : C = R,   back substitution  R x = c  (last unknown first)
//   UPPER = false: C = R^T (i.e. R stored row-major), forward substitution
//                  R^T y = z (first unknown first)
// The 64 x 64 diagonal block is staged in LDS as blk[j * 64 + l] =
// C[b0 + l, b0 + j] (all loads issued before the stores); wave 0 runs the
// substitution chain, reading each solved unknown with v_readlane; then the
// group updates the remaining rows with coalesced reads of C, 16 loads in
// flight per thread.  The order of operations is fixed.
template <bool UPPER, int NT>
__device__ inline void trsv_lds(const double* __restrict__ C, int64_t ld, int n,
                                const double* __restrict__ invd, double* x, double* blk) {
  static_assert(4096 % NT == 0, "NT divides 4096");
  const int tid = threadIdx.x, lane = tid & 63;
  const int nblk = (n + 63) / 64;
  for (int bi = 0; bi < nblk; ++bi) {
    // UPPER walks the blocks from the bottom; the top block may be partial
    const int b0 = UPPER ? (n - 64 * (bi + 1) > 0 ? n - 64 * (bi + 1) : 0) : 64 * bi;
    const int bend = UPPER ? n - 64 * bi : (b0 + 64 < n ? b0 + 64 : n);
    const int bw = bend - b0;
    {
      constexpr int K = 4096 / NT;
      double tmp[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int e = tid + k * NT, l = e & 63, j = e >> 6;
        tmp[k] = (l < bw && j < bw) ? C[(int64_t)(b0 + j) * ld + b0 + l] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) blk[tid + k * NT] = tmp[k];
    }
    __syncthreads();
    if (tid < 64) {
      double xi = lane < bw ? x[b0 + lane] : 0.0;
      const double di = lane < bw ? invd[b0 + lane] : 0.0;
      // the block's entries are read 16 steps at a time ahead of the steps
      // that use them, so no step waits for its own LDS read
      for (int q0 = 0; q0 < 64; q0 += 16) {
        double cs[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int jl = UPPER ? 63 - (q0 + u) : q0 + u;
          cs[u] = blk[jl * 64 + lane];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int jl = UPPER ? 63 - (q0 + u) : q0 + u;
          if (jl < bw) {
            const double xj = readlane_f64(xi * di, jl);
            const bool upd = UPPER ? lane < jl : lane > jl;
            xi = lane == jl ? xj : (upd ? fma(-cs[u], xj, xi) : xi);
          }
        }
      }
      if (lane < bw) x[b0 + lane] = xi;
    }
    __syncthreads();
    // remaining unknowns: above the block (UPPER) or below it (lower)
    const int r0 = UPPER ? 0 : bend, r1 = UPPER ? b0 : n;
    for (int i = r0 + tid; i < r1; i += NT) {
      double s = 0.0;
      int j = b0;
      for (; j + 16 <= bend; j += 16) {
        double c[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) c[u] = C[(int64_t)(j + u) * ld + i];
#pragma unroll
        for (int u = 0; u < 16; ++u) s = fma(c[u], x[j + u], s);
      }
      for (; j < bend; ++j) s = fma(C[(int64_t)j * ld + i], x[j], s);
      x[i] -= s;
    }
    __syncthreads();
  }
}

}  // namespace sns
