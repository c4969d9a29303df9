// Hadamard sketch (subsampled randomized Hadamard transform, the second
// dense operator of Sec. 1.2.1): SA = d^{-1/2} (H D A)[r_0 .. r_{d-1}], Sb
// likewise, with A zero-padded to m' = 2^L rows, D = diag(s(i)) random signs,
// H the unnormalised Sylvester-Hadamard matrix (H[r, i] = (-1)^popcount(r & i))
// and rows r_k drawn uniformly from [0, m') with replacement.
//   s(i): top bit of word (i & 3) of Philox4x32-10 at counter
//         (i >> 2 mod 2^32, i >> 34, 0, 2) clear -> +1, set -> -1;
//   r_k  = (w * m') >> 32, w word (k & 3) of Philox4x32-10 at counter
//         (k >> 2 mod 2^32, k >> 34, 0, 3); key = seed.
//
// H = H_top (x) H_low splits the row index i = (i_top, i_low) with i_low
// the low b = min(L, 10) bits.  Pass 1 (k_srht_block) transforms each block
// of 2^b consecutive rows of D [A | b] in LDS (b butterfly stages) and writes
// the result B (m' x C, A's dtype, C = n + 1 with b).  Pass 2
// (k_srht_sample) forms each sampled row r = (r_top, r_low) as
// sum over i_top of (-1)^popcount(r_top & i_top) B[(i_top, r_low)], in fp64,
// and scales by d^{-1/2}.  Bytes: pass 1 reads A and writes B, pass 2 reads
// d 2^(L-b) rows of B (about all of B once when d ~ 2^b).
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace sns {

namespace {

constexpr int kHThreads = 256;
constexpr int kHBlockBits = 10;

__device__ __forceinline__ uint32_t had_word(uint64_t seed, uint64_t idx, uint32_t tag) {
  const uint64_t q = idx >> 2;
  const U4 w = philox4x32_10(U4{(uint32_t)q, (uint32_t)(q >> 32), 0u, tag}, (uint32_t)seed,
                             (uint32_t)(seed >> 32));
  switch (idx & 3) {
    case 0: return w.x;
    case 1: return w.y;
    case 2: return w.z;
    default: return w.w;
  }
}

// One block of BR = 2^bits rows x CW columns of D [A | b]: load (signs,
// zero rows past m), `bits` butterfly stages in LDS, store to B.
template <typename T, int CW>
__global__ __launch_bounds__(kHThreads) void k_srht_block(const T* __restrict__ A, int64_t ld,
                                                          int64_t m, int n, const T* __restrict__ b,
                                                          uint64_t seed, int bits, int ctiles,
                                                          T* __restrict__ B, int C) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  T* tile = reinterpret_cast<T*>(smem);  // [BR][CW]
  const int BR = 1 << bits;
  const int t = threadIdx.x;
  const int ct = (int)(blockIdx.x % (unsigned)ctiles);
  const int64_t blk = blockIdx.x / (unsigned)ctiles;
  const int c0 = ct * CW;
  const int64_t i0 = blk << bits;
  for (int e = t; e < BR * CW; e += kHThreads) {
    const int r = e / CW, c = e % CW, col = c0 + c;
    const int64_t i = i0 + r;
    T v = T(0);
    if (i < m && col <= n) {
      if (col < n) v = A[i * ld + col];
      else if (b) v = b[i];
      if ((had_word(seed, (uint64_t)i, 2u) >> 31) != 0u) v = -v;
    }
    tile[e] = v;
  }
  __syncthreads();
  for (int s = 0; s < bits; ++s) {
    const int h = 1 << s;
    for (int q = t; q < (BR / 2) * CW; q += kHThreads) {
      const int c = q % CW, p = q / CW;
      const int r = ((p >> s) << (s + 1)) | (p & (h - 1));
      const T x = tile[r * CW + c], y = tile[(r + h) * CW + c];
      tile[r * CW + c] = x + y;
      tile[(r + h) * CW + c] = x - y;
    }
    __syncthreads();
  }
  for (int e = t; e < BR * CW; e += kHThreads) {
    const int r = e / CW, c = e % CW, col = c0 + c;
    if (col < C) B[(i0 + r) * C + col] = tile[e];
  }
}

// Sampled row k, columns [256 ct, 256 ct + 256): sum over i_top of
// (-1)^popcount(r_top & i_top) B[(i_top << bits) | r_low], eight running fp64
// sums per thread combined in a fixed order.
template <typename T>
__global__ __launch_bounds__(kHThreads) void k_srht_sample(const T* __restrict__ B, int C,
                                                           int bits, int L, uint64_t seed,
                                                           int ctiles, int n, double scale,
                                                           T* __restrict__ SA, T* __restrict__ Sb) {
  const int ct = (int)(blockIdx.x % (unsigned)ctiles);
  const int64_t k = blockIdx.x / (unsigned)ctiles;
  const int col = ct * kHThreads + threadIdx.x;
  if (col >= C) return;
  const uint64_t mp = uint64_t(1) << L;
  const uint64_t r = ((uint64_t)had_word(seed, (uint64_t)k, 3u) * mp) >> 32;
  const uint64_t rlow = r & ((uint64_t(1) << bits) - 1), rtop = r >> bits;
  const int64_t ntop = int64_t(1) << (L - bits);
  double acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = 0.0;
  int64_t it = 0;
  for (; it + 8 <= ntop; it += 8) {
    T v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = B[(((it + j) << bits) | rlow) * C + col];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double x = (double)v[j];
      acc[j] += (__popcll(rtop & (uint64_t)(it + j)) & 1) ? -x : x;
    }
  }
  for (int j = 0; it < ntop; ++it, ++j) {
    const double x = (double)B[((it << bits) | rlow) * C + col];
    acc[j] += (__popcll(rtop & (uint64_t)it) & 1) ? -x : x;
  }
  const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  if (col < n) SA[k * n + col] = (T)(s * scale);
  else if (Sb) Sb[k] = (T)(s * scale);
}

struct HadPlan {
  int L, bits, C;
  uint64_t mp;
};

HadPlan had_plan(const sns_matrix& A, bool with_b) {
  HadPlan p;
  p.L = 0;
  while ((int64_t(1) << p.L) < A.m) ++p.L;
  p.mp = uint64_t(1) << p.L;
  p.bits = p.L < kHBlockBits ? p.L : kHBlockBits;
  p.C = (int)A.n + (with_b ? 1 : 0);
  return p;
}

template <typename T, int CW>
sns_status launch_had(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b, void* SA,
                      void* Sb, void* ws, hipStream_t st) {
  const HadPlan p = had_plan(A, b != nullptr);
  T* B = static_cast<T*>(ws);
  const int ctiles = (p.C + CW - 1) / CW;
  const uint64_t blocks = (p.mp >> p.bits) * (uint64_t)ctiles;
  if (blocks > 0x7FFFFFFFull) return SNS_ERR_SHAPE;
  const size_t lds = ((size_t)1 << p.bits) * CW * sizeof(T);
  SNS_LAUNCH("srht_block", (k_srht_block<T, CW>), dim3((unsigned)blocks), dim3(kHThreads), lds, st,
             static_cast<const T*>(A.values), A.ld, A.m, (int)A.n, static_cast<const T*>(b), seed,
             p.bits, ctiles, B, p.C);
  const int stiles = (p.C + kHThreads - 1) / kHThreads;
  SNS_LAUNCH("srht_sample", k_srht_sample<T>, dim3((unsigned)(d * (uint64_t)stiles)),
             dim3(kHThreads), 0, st, (const T*)B, p.C, p.bits, p.L, seed, stiles, (int)A.n,
             1.0 / sqrt((double)d), static_cast<T*>(SA), static_cast<T*>(Sb));
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace

size_t hadamard_workspace_bytes(const sns_matrix& A, uint32_t /*d*/) {
  const HadPlan p = had_plan(A, true);
  return align_up((size_t)p.mp * p.C * (A.dtype == SNS_F64 ? 8 : 4));
}

sns_status launch_hadamard_sketch(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b,
                                  void* SA, void* Sb, void* ws, hipStream_t st) {
  if (A.layout != SNS_DENSE_ROWMAJOR) return SNS_ERR_DTYPE;
  if (A.dtype == SNS_F64) return launch_had<double, 8>(A, d, seed, b, SA, Sb, ws, st);
  return launch_had<float, 16>(A, d, seed, b, SA, Sb, ws, st);
}

}  // namespace sns
