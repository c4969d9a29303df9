// Device-side building blocks shared by the libsns kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sns.h"

namespace sns {
// Reports a failed HIP call on stderr when SNS_DEBUG=1 is set (trace.hip).
void report_hip_error(hipError_t e, const char* what, const char* file, int line);
}  // namespace sns

#define SNS_HIP_TRY(expr)                                                   \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess) {                                                 \
      ::sns::report_hip_error(e_, #expr, __FILE__, __LINE__);               \
      return SNS_ERR_HIP;                                                   \
    }                                                                       \
  } while (0)

namespace sns {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): four 32-bit counter words, two key
// words, ten rounds.  Round: (c0,c1,c2,c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2),
// hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key is bumped by the Weyl constants
// between rounds.  Used for every random quantity of the sketches.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    // one 32 x 32 -> 64-bit multiply gives both halves of each product
    const uint64_t p0 = (uint64_t)M0 * c.x, p1 = (uint64_t)M1 * c.z;
    c = U4{(uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
           (uint32_t)p0};
  }
  return c;
}

// CountSketch bucket and sign of row i (Clarkson-Woodruff, one +-1 per column
// of S).  Rows 2j and 2j+1 share the Philox block j = i >> 1 at counter
// (j lo, j hi, 0, 0): the even row takes words (x, y), the odd row (z, w).
// Bucket = multiply-shift range reduction of the first word to [0, d);
// sign = -1 iff the top bit of the second word is set.
struct Hash { uint32_t h; bool neg; };

__device__ __forceinline__ Hash cs_hash(uint64_t seed, uint32_t d, uint64_t i) {
  const uint64_t j = i >> 1;
  const U4 w = philox4x32_10(U4{(uint32_t)j, (uint32_t)(j >> 32), 0u, 0u},
                             (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint32_t wh = (i & 1) ? w.z : w.x;
  const uint32_t ws = (i & 1) ? w.w : w.y;
  return Hash{(uint32_t)(((uint64_t)wh * d) >> 32), (ws >> 31) != 0u};
}

// Both rows of one Philox block at once (rows 2j, 2j+1).
__device__ __forceinline__ void cs_hash_pair(uint64_t seed, uint32_t d, uint64_t j,
                                             Hash& even, Hash& odd) {
  const U4 w = philox4x32_10(U4{(uint32_t)j, (uint32_t)(j >> 32), 0u, 0u},
                             (uint32_t)seed, (uint32_t)(seed >> 32));
  even = Hash{(uint32_t)(((uint64_t)w.x * d) >> 32), (w.y >> 31) != 0u};
  odd = Hash{(uint32_t)(((uint64_t)w.z * d) >> 32), (w.w >> 31) != 0u};
}

// ---------------------------------------------------------------------------
// Reductions.  All of them combine values in a fixed order that depends only
// on the launch shape, so results are reproducible bit for bit.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Sum over the whole work-group; every thread receives the total.
// `red` is LDS scratch of at least blockDim.x / 64 entries.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  T t = 0;
  for (int k = 0; k < nw; ++k) t += red[k];
  return t;
}

template <typename T>
__device__ __forceinline__ T block_max(T v, T* red) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  T t = red[0];
  for (int k = 1; k < nw; ++k) t = fmax(t, red[k]);
  return t;
}

}  // namespace sns
