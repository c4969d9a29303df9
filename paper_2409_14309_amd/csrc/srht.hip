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
// H is the Kronecker product of 2 x 2 factors, one per bit of the row index,
// so the transform is a sequence of butterfly stages, one per bit, in any
// order.  Full passes (k_srht_pass) each apply the stages of up to 8
// consecutive bits [lo, lo + nb): a work-group loads the 2^nb rows that differ
// only in those bits (row segments of 32 columns: 128 bytes fp32, two columns
// per lane; 256 bytes fp64),
// applies the stages in registers and one LDS exchange, and writes the result
// back in place of the same rows (pass 1 reads D [A | b], zero-padded; later
// passes ping-pong between two m' x C buffers, C = n + 1 with b, rows padded
// to 32 values so that every segment is aligned).  The last at most 8 bits
// are never transformed in full: each sampled row r is formed directly
// (k_srht_sample) as the sum over the top index i_top of
// (-1)^popcount(r_top & i_top) B[(i_top, r_low)], in fp64, scaled by d^{-1/2}.
// Bytes for m' = 2^L rows: ceil(L / 8) - 1 full passes (at least one), each
// reading and writing m' x C values, plus d 2^(L - 8 P) rows for the samples.
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace sns {

namespace {

constexpr int kHThreads = 256;

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

// VW consecutive columns of one row, moved with one load or store (8 bytes for
// two fp32 values).
template <typename T, int VW>
struct Pk {
  T e[VW];
};

template <typename T, int VW>
__device__ __forceinline__ Pk<T, VW> pk_load(const T* p) {
  Pk<T, VW> r;
  if constexpr (VW == 1) {
    r.e[0] = *p;
  } else {
    typedef T VT __attribute__((ext_vector_type(VW)));
    const VT v = *reinterpret_cast<const VT*>(p);
#pragma unroll
    for (int e = 0; e < VW; ++e) r.e[e] = v[e];
  }
  return r;
}

template <typename T, int VW>
__device__ __forceinline__ void pk_store(T* p, const Pk<T, VW>& x) {
  if constexpr (VW == 1) {
    *p = x.e[0];
  } else {
    typedef T VT __attribute__((ext_vector_type(VW)));
    VT v;
#pragma unroll
    for (int e = 0; e < VW; ++e) v[e] = x.e[e];
    *reinterpret_cast<VT*>(p) = v;
  }
}

template <typename T, int VW>
__device__ __forceinline__ void pk_butterfly(Pk<T, VW>& a, Pk<T, VW>& b) {
#pragma unroll
  for (int e = 0; e < VW; ++e) {
    const T x = a.e[e], y = b.e[e];
    a.e[e] = x + y;
    b.e[e] = x - y;
  }
}

// One full pass over the bits [lo, lo + NB): work-group (o, ct) transforms
// the 2^NB rows row(j) = (o mod 2^lo) + (j << lo) + ((o >> lo) << (lo + NB))
// over columns [CW VW ct, CW VW (ct + 1)), VW columns per thread.  Thread
// (g, c), g < RT, holds j = g + RT k and applies the stages of the bits of k
// in registers; one LDS exchange (row stride CW + 1 packs) then gives each
// thread groups of RT consecutive j for the stages of the bits of g.
// src == nullptr: the first pass, reading D [A | b] (rows past m are zero);
// `avec`: A's rows allow VW-wide loads (base and row stride aligned).
template <typename T, int VW, int CW, int NB>
__global__ __launch_bounds__(kHThreads) void k_srht_pass(const T* __restrict__ src,
                                                         const T* __restrict__ A, int64_t ld,
                                                         int64_t m, int n, const T* __restrict__ b,
                                                         uint64_t seed, int lo, int ctiles,
                                                         T* __restrict__ dst, int C, int ldb,
                                                         bool avec) {
  typedef Pk<T, VW> P;
  constexpr int BR = 1 << NB;
  constexpr int RT0 = kHThreads / CW;
  constexpr int RT = RT0 < BR ? RT0 : BR, NV = BR / RT, LDT = CW + 1;
  __shared__ P tile[BR * LDT];
  __shared__ unsigned char neg[BR];  // first pass: sign bits of the block's rows
  const int t = threadIdx.x, g = t / CW, c = t % CW;
  const int ct = (int)(blockIdx.x % (unsigned)ctiles);
  const int64_t o = blockIdx.x / (unsigned)ctiles;
  const int64_t olow = o & ((int64_t(1) << lo) - 1), ohigh = o >> lo;
  auto row = [&](int j) -> int64_t { return olow + ((int64_t)j << lo) + (ohigh << (lo + NB)); };
  const int col = (ct * CW + c) * VW;  // first column of this thread's pack
  const bool active = g < RT;
  if (!src) {  // lo = 0: the block's rows are consecutive, one Philox call per 4 rows
    for (int j = t; j < BR; j += kHThreads) neg[j] = (unsigned char)(had_word(seed, (uint64_t)row(j), 2u) >> 31);
    __syncthreads();
  }
  // Loads: the common cases have no branch inside the loop, so every load of
  // the block is in flight before the first use.  Columns past C (inside the
  // padded row of the work buffers) carry zeros or values nobody reads.
  P v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int e = 0; e < VW; ++e) v[k].e[e] = T(0);
  if (active) {
    if (src) {
      if (col < C) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = pk_load<T, VW>(src + row(g + RT * k) * ldb + col);
      }
    } else {
      const bool full = row(BR - 1) < m;  // the first pass reads consecutive rows
      if (full && col + VW <= n && (VW == 1 || avec)) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = pk_load<T, VW>(A + row(g + RT * k) * ld + col);
      } else if (col <= n) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          const int64_t i = row(g + RT * k);
          if (i < m) {
#pragma unroll
            for (int e = 0; e < VW; ++e) {
              const int cc = col + e;
              v[k].e[e] = cc < n ? A[i * ld + cc] : (cc == n && b ? b[i] : T(0));
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < NV; ++k)
        if (neg[g + RT * k])
#pragma unroll
          for (int e = 0; e < VW; ++e) v[k].e[e] = -v[k].e[e];
    }
  }
#pragma unroll
  for (int h = 1; h < NV; h <<= 1)
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if ((k & h) == 0) pk_butterfly<T, VW>(v[k], v[k + h]);
  if constexpr (RT == 1) {
    if (active && col < C) {
#pragma unroll
      for (int k = 0; k < NV; ++k) pk_store<T, VW>(dst + row(k) * ldb + col, v[k]);
    }
  } else {
    if (active) {
#pragma unroll
      for (int k = 0; k < NV; ++k) tile[(g + RT * k) * LDT + c] = v[k];
    }
    __syncthreads();
    for (int q = t; q < NV * CW; q += kHThreads) {
      const int grp = q / CW, cc = q % CW, ccol = (ct * CW + cc) * VW;
      P w[RT];
#pragma unroll
      for (int r = 0; r < RT; ++r) w[r] = tile[(grp * RT + r) * LDT + cc];
#pragma unroll
      for (int h = 1; h < RT; h <<= 1)
#pragma unroll
        for (int r = 0; r < RT; ++r)
          if ((r & h) == 0) pk_butterfly<T, VW>(w[r], w[r + h]);
      if (ccol < C) {
#pragma unroll
        for (int r = 0; r < RT; ++r) pk_store<T, VW>(dst + row(grp * RT + r) * ldb + ccol, w[r]);
      }
    }
  }
}

// Sampled row k, columns [256 ct, 256 ct + 256): sum over i_top of
// (-1)^popcount(r_top & i_top) B[(i_top << bits) | r_low], eight running fp64
// sums per thread combined in a fixed order.
template <typename T>
__global__ __launch_bounds__(kHThreads) void k_srht_sample(const T* __restrict__ B, int C, int ldb,
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
    for (int j = 0; j < 8; ++j) v[j] = B[(((it + j) << bits) | rlow) * ldb + col];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double x = (double)v[j];
      acc[j] += (__popcll(rtop & (uint64_t)(it + j)) & 1) ? -x : x;
    }
  }
  for (int j = 0; it < ntop; ++it, ++j) {
    const double x = (double)B[((it << bits) | rlow) * ldb + col];
    acc[j] += (__popcll(rtop & (uint64_t)it) & 1) ? -x : x;
  }
  const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  if (col < n) SA[k * n + col] = (T)(s * scale);
  else if (Sb) Sb[k] = (T)(s * scale);
}

struct HadPlan {
  int L, P, C, ldb;  // m' = 2^L rows, P full passes over bits [0, 8 P) (the last may be shorter)
  uint64_t mp;
};

HadPlan had_plan(const sns_matrix& A, bool with_b) {
  HadPlan p;
  p.L = 0;
  while ((int64_t(1) << p.L) < A.m) ++p.L;
  p.mp = uint64_t(1) << p.L;
  p.P = (p.L + 7) / 8 - 1;
  if (p.P < 1) p.P = 1;
  p.C = (int)A.n + (with_b ? 1 : 0);
  p.ldb = (int)((A.n + 1 + 31) / 32 * 32);  // B rows start on 128-byte boundaries
  return p;
}

template <typename T, int VW, int CW, int NB>
void launch_pass(dim3 grid, hipStream_t st, const T* src, const sns_matrix& A, const void* b,
                 uint64_t seed, int lo, int ctiles, T* dst, int C, int ldb, bool avec) {
  SNS_LAUNCH(src ? "srht_pass" : "srht_pass1", (k_srht_pass<T, VW, CW, NB>), grid,
             dim3(kHThreads), 0, st, src, static_cast<const T*>(A.values), A.ld, A.m, (int)A.n,
             static_cast<const T*>(b), seed, lo, ctiles, dst, C, ldb, avec);
}

// VW columns per thread, CW packs per work-group (a row segment of CW VW
// values: 128 bytes for fp32, 256 for fp64).
template <typename T, int VW, int CW>
sns_status launch_had(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b, void* SA,
                      void* Sb, void* ws, hipStream_t st) {
  const HadPlan p = had_plan(A, b != nullptr);
  const size_t buf = align_up((size_t)p.mp * p.ldb * sizeof(T));
  T* Bs[2] = {static_cast<T*>(ws), reinterpret_cast<T*>(static_cast<char*>(ws) + buf)};
  static_assert(32 % (CW * VW) == 0 || (CW * VW) % 32 == 0, "tiles inside the padded rows");
  const int ctiles = (p.C + CW * VW - 1) / (CW * VW);
  const bool avec = reinterpret_cast<uintptr_t>(A.values) % (VW * sizeof(T)) == 0 && A.ld % VW == 0;
  const T* src = nullptr;
  int lo = 0;
  for (int q = 0; q < p.P; ++q) {
    const int nb = (p.L - lo) < 8 ? (p.L - lo) : 8;
    T* dst = Bs[q & 1];
    const uint64_t blocks = (p.mp >> nb) * (uint64_t)ctiles;
    if (blocks > 0x7FFFFFFFull) return SNS_ERR_SHAPE;
    const dim3 grid((unsigned)blocks);
#define SNS_PASS(NBV) \
  launch_pass<T, VW, CW, NBV>(grid, st, src, A, b, seed, lo, ctiles, dst, p.C, p.ldb, avec)
    switch (nb) {
      case 0: SNS_PASS(0); break;
      case 1: SNS_PASS(1); break;
      case 2: SNS_PASS(2); break;
      case 3: SNS_PASS(3); break;
      case 4: SNS_PASS(4); break;
      case 5: SNS_PASS(5); break;
      case 6: SNS_PASS(6); break;
      case 7: SNS_PASS(7); break;
      default: SNS_PASS(8); break;
    }
#undef SNS_PASS
    src = dst;
    lo += nb;
  }
  const int stiles = (p.C + kHThreads - 1) / kHThreads;
  SNS_LAUNCH("srht_sample", k_srht_sample<T>, dim3((unsigned)(d * (uint64_t)stiles)),
             dim3(kHThreads), 0, st, src, p.C, p.ldb, lo, p.L, seed, stiles, (int)A.n,
             1.0 / sqrt((double)d), static_cast<T*>(SA), static_cast<T*>(Sb));
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace

size_t hadamard_workspace_bytes(const sns_matrix& A, uint32_t /*d*/) {
  const HadPlan p = had_plan(A, true);
  const size_t buf = align_up((size_t)p.mp * p.ldb * (A.dtype == SNS_F64 ? 8 : 4));
  return p.P > 1 ? 2 * buf : buf;
}

sns_status launch_hadamard_sketch(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b,
                                  void* SA, void* Sb, void* ws, hipStream_t st) {
  if (A.layout != SNS_DENSE_ROWMAJOR) return SNS_ERR_DTYPE;
  if (A.dtype == SNS_F64) return launch_had<double, 1, 32>(A, d, seed, b, SA, Sb, ws, st);
  return launch_had<float, 2, 32>(A, d, seed, b, SA, Sb, ws, st);
}

}  // namespace sns
