// Single-work-group fp64 building blocks used by the QR and LSQR kernels:
// multi-value wave reductions and triangular solves with R (n x n upper
// triangular, column-major, leading dimension ld) on a vector held in LDS.
#pragma once

#include "common.hpp"

namespace sns {

// Reduce NB values per lane over the 64 lanes of a wave with a butterfly that
// halves the live values at each of the first log2(NB) exchanges.  On return
// `out` on lane L is the wave total of value index `idx(L)`; every index is
// held by 64 / NB lanes.  Exchange order is fixed, so the result is
// reproducible.
template <int NB>
__device__ __forceinline__ double wave_reduce_multi(const double (&g)[NB], int& idx) {
  static_assert(NB >= 1 && NB <= 64 && (NB & (NB - 1)) == 0, "NB power of two");
  const int lane = threadIdx.x & 63;
  double cur[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) cur[q] = g[q];
  int id = 0;
  int s = 0;
#pragma unroll
  for (int len = NB; len > 1; len >>= 1, ++s) {
    const int mask = 32 >> s;
    const bool up = (lane & mask) != 0;
    id = (id << 1) | (up ? 1 : 0);
#pragma unroll
    for (int q = 0; q < len / 2; ++q) {
      const double send = up ? cur[q] : cur[q + len / 2];
      const double keep = up ? cur[q + len / 2] : cur[q];
      cur[q] = keep + __shfl_xor(send, mask, 64);
    }
  }
#pragma unroll
  for (int mask = 32 >> s; mask >= 1; mask >>= 1) cur[0] += __shfl_xor(cur[0], mask, 64);
  idx = id;
  return cur[0];
}

// Sum NB values per thread over the whole work-group; tot[0..NB) (LDS) gets the
// totals, visible to all threads on return.  red: LDS of (blockDim/64) * NB.
template <int NB>
__device__ __forceinline__ void block_reduce_multi(const double (&g)[NB], double* red,
                                                   double* tot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int idx;
  const double v = wave_reduce_multi<NB>(g, idx);
  if ((lane & (64 / NB - 1)) == 0) red[wv * NB + idx] = v;
  __syncthreads();
  if (threadIdx.x < NB) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w * NB + threadIdx.x];
    tot[threadIdx.x] = t;
  }
  __syncthreads();
}

// Solve R x = c in place (x in LDS, length n) by back substitution, 64 rows
// at a time: wave 0 solves the diagonal block from an LDS copy `blk`
// (64 x 64 doubles), then the whole group updates the rows above it.
__device__ inline void trsv_upper_lds(const double* __restrict__ R, int64_t ld, int n,
                                      double* x, double* blk) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
  for (int bend = n; bend > 0; bend -= 64) {
    const int b0 = bend > 64 ? bend - 64 : 0, bw = bend - b0;
    for (int e = tid; e < 64 * 64; e += nt) {
      const int r = e & 63, c = e >> 6;  // blk[c * 64 + r] = R[b0 + r, b0 + c]
      blk[e] = (r < bw && c < bw) ? R[(int64_t)(b0 + c) * ld + b0 + r] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      double xi = lane < bw ? x[b0 + lane] : 0.0;
      for (int jl = bw - 1; jl >= 0; --jl) {
        const double xj = __shfl(xi, jl, 64) / blk[jl * 64 + jl];
        if (lane == jl) xi = xj;
        else if (lane < jl) xi -= blk[jl * 64 + lane] * xj;
      }
      if (lane < bw) x[b0 + lane] = xi;
    }
    __syncthreads();
    for (int i = tid; i < b0; i += nt) {
      double s = 0.0;
      for (int j = b0; j < bend; ++j) s += R[(int64_t)j * ld + i] * x[j];
      x[i] -= s;
    }
    __syncthreads();
  }
}

// Solve R^T y = z in place (y in LDS) by forward substitution, 64 rows at a
// time.  R^T[i, j] = R[j, i] = R[i * ld + j] (column-major R).
__device__ inline void trsv_upper_trans_lds(const double* __restrict__ R, int64_t ld, int n,
                                            double* y, double* blk) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
  for (int b0 = 0; b0 < n; b0 += 64) {
    const int bend = b0 + 64 < n ? b0 + 64 : n, bw = bend - b0;
    for (int e = tid; e < 64 * 64; e += nt) {
      const int r = e & 63, c = e >> 6;  // blk[c * 64 + r] = R^T[b0 + c, b0 + r] = R[b0 + r, b0 + c]
      blk[e] = (r < bw && c < bw) ? R[(int64_t)(b0 + c) * ld + b0 + r] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      double yi = lane < bw ? y[b0 + lane] : 0.0;
      for (int jl = 0; jl < bw; ++jl) {
        const double yj = __shfl(yi, jl, 64) / blk[jl * 64 + jl];
        if (lane == jl) yi = yj;
        else if (lane > jl && lane < bw) yi -= blk[lane * 64 + jl] * yj;  // R[b0+jl, b0+lane]
      }
      if (lane < bw) y[b0 + lane] = yi;
    }
    __syncthreads();
    for (int i = bend + tid; i < n; i += nt) {
      double s = 0.0;
      const double* Ri = R + (int64_t)i * ld;  // column i of R: R[j, i] for j < i
      for (int j = b0; j < bend; ++j) s += Ri[j] * y[j];
      y[i] -= s;
    }
    __syncthreads();
  }
}

}  // namespace sns
