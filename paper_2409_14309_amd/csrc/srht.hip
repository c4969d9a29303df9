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
// back in place of the same rows (pass 1 reads D A or D [A | b], zero-padded;
// later passes ping-pong between two m' x C buffers, rows padded to 32 values
// so that every segment is aligned).  b is column n of the work buffers (C =
// n + 1) when n is not a multiple of the tile width, so it shares the last
// tile; otherwise it would take a tile of its own with one scattered 4- or
// 8-byte access per row, and b is transformed as a vector of its own instead
// (C = n): its first 8 bits by k_srht_vpass1 (for m' < 256, the pass kernel
// on b as an m x 1 matrix), each later pass over bits [lo, lo + nb) by the
// pass kernel on b as an (m' >> lo) x 2^lo matrix (row-contiguous, so its
// bits [0, nb) are the vector's bits [lo, lo + nb)).  The stages run in the
// same order for b as for the columns of A.  The last at most 8 bits
// are never transformed in full: each sampled row r is formed directly
// (k_srht_sample) as the sum over the top index i_top of
// (-1)^popcount(r_top & i_top) B[(i_top, r_low)], in fp64, scaled by d^{-1/2}.
// Bytes for m' = 2^L rows: ceil(L / 8) - 1 full passes (at least one), each
// reading and writing m' x (n + 1) values, plus d 2^(L - 8 P) rows for the
// samples.
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

// The first pass over b when it is a vector of its own (bits [0, 8) of the
// index, m' >= 256): one wave per block of 256 consecutive entries, lane l
// holding entries l + 64 k, k < 4.  The stages run in the order that
// k_srht_pass applies with 8 row groups (index bits 3 to 7, then 0 to 2),
// each pair giving (lower + upper, lower - upper), so b comes out bit for bit
// as it would as a column of the work buffers.
template <typename T>
__global__ __launch_bounds__(kHThreads) void k_srht_vpass1(const T* __restrict__ b, int64_t m,
                                                           uint64_t seed, uint64_t nblk,
                                                           T* __restrict__ dst) {
  const uint64_t blk = (uint64_t)blockIdx.x * (kHThreads / 64) + (threadIdx.x >> 6);
  if (blk >= nblk) return;  // uniform over the wave
  const int lane = threadIdx.x & 63;
  const int64_t base = (int64_t)blk * 256 + lane;
  T v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + 64 * k;
    const T x = i < m ? b[i] : T(0);
    v[k] = (had_word(seed, (uint64_t)i, 2u) >> 31) ? -x : x;
  }
  // index bits 3, 4, 5: partners 8, 16, 32 lanes away
#pragma unroll
  for (int s = 8; s <= 32; s <<= 1)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T y = __shfl_xor(v[k], s, 64);
      v[k] = (lane & s) ? y - v[k] : v[k] + y;
    }
  // index bits 6, 7: in registers
  Pk<T, 1> r[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k].e[0] = v[k];
  pk_butterfly<T, 1>(r[0], r[1]);
  pk_butterfly<T, 1>(r[2], r[3]);
  pk_butterfly<T, 1>(r[0], r[2]);
  pk_butterfly<T, 1>(r[1], r[3]);
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = r[k].e[0];
  // index bits 0, 1, 2
#pragma unroll
  for (int s = 1; s <= 4; s <<= 1)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T y = __shfl_xor(v[k], s, 64);
      v[k] = (lane & s) ? y - v[k] : v[k] + y;
    }
#pragma unroll
  for (int k = 0; k < 4; ++k) dst[base + 64 * k] = v[k];
}

// Sampled row k, columns [256 ct, 256 ct + 256) of [A | b]: sum over i_top
// of (-1)^popcount(r_top & i_top) B[(i_top << bits) | r_low], eight running
// fp64 sums per thread combined in a fixed order.  Columns of A come from B
// (row stride ldb), column n (b) from the vector Bv if there is one, else
// from column n of B.
template <typename T>
__global__ __launch_bounds__(kHThreads) void k_srht_sample(const T* __restrict__ Bm,
                                                           const T* __restrict__ Bv, int C, int ldb,
                                                           int bits, int L, uint64_t seed,
                                                           int ctiles, int n, double scale,
                                                           T* __restrict__ SA, T* __restrict__ Sb) {
  const int ct = (int)(blockIdx.x % (unsigned)ctiles);
  const int64_t k = blockIdx.x / (unsigned)ctiles;
  const int col = ct * kHThreads + threadIdx.x;
  if (col >= C) return;
  const bool vec = col == n && Bv;
  const T* __restrict__ B = vec ? Bv : Bm + col;
  const int64_t stride = vec ? 1 : ldb;
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
    for (int j = 0; j < 8; ++j) v[j] = B[(((it + j) << bits) | rlow) * stride];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double x = (double)v[j];
      acc[j] += (__popcll(rtop & (uint64_t)(it + j)) & 1) ? -x : x;
    }
  }
  for (int j = 0; it < ntop; ++it, ++j) {
    const double x = (double)B[((it << bits) | rlow) * stride];
    acc[j] += (__popcll(rtop & (uint64_t)it) & 1) ? -x : x;
  }
  const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  if (col < n) SA[k * n + col] = (T)(s * scale);
  else if (Sb) Sb[k] = (T)(s * scale);
}

struct HadPlan {
  int L, P, ldb;  // m' = 2^L rows, P full passes over bits [0, 8 P) (the last may be shorter)
  uint64_t mp;
  int nbuf;       // work buffers of each kind (ping-pong from the second pass on)
  bool bvec;      // b transformed as a vector of its own, not as column n
};

// Columns per work-group of the full passes (CW packs of VW values; the
// launches below instantiate these widths).
template <typename T>
constexpr int had_tile_of() {
  return sizeof(T) == 8 ? 32 : 64;
}
int had_tile(const sns_matrix& A) {
  return A.dtype == SNS_F64 ? had_tile_of<double>() : had_tile_of<float>();
}

HadPlan had_plan(const sns_matrix& A) {
  HadPlan p;
  p.L = 0;
  while ((int64_t(1) << p.L) < A.m) ++p.L;
  p.mp = uint64_t(1) << p.L;
  p.P = (p.L + 7) / 8 - 1;
  if (p.P < 1) p.P = 1;
  p.bvec = A.n % had_tile(A) == 0;
  p.ldb = (int)((A.n + (p.bvec ? 0 : 1) + 31) / 32 * 32);  // B rows start on 128-byte boundaries
  p.nbuf = p.P > 1 ? 2 : 1;
  return p;
}

// Work space: nbuf m' x ldb buffers, then (bvec) nbuf m'-vectors for b.
size_t had_matrix_bytes(const HadPlan& p, size_t es) { return align_up((size_t)p.mp * p.ldb * es); }
size_t had_vector_bytes(const HadPlan& p, size_t es) {
  return p.bvec ? align_up((size_t)p.mp * es) : 0;
}

template <typename T, int VW, int CW, int NB>
void launch_pass(dim3 grid, hipStream_t st, bool view, const T* src, const T* A, int64_t ld,
                 int64_t m, int n, const T* b, uint64_t seed, int lo, int ctiles, T* dst, int C,
                 int ldb, bool avec) {
  if (view)
    SNS_LAUNCH(src ? "srht_vpass" : "srht_vpass1", (k_srht_pass<T, VW, CW, NB>), grid,
               dim3(kHThreads), 0, st, src, A, ld, m, n, b, seed, lo, ctiles, dst, C, ldb, avec);
  else
    SNS_LAUNCH(src ? "srht_pass" : "srht_pass1", (k_srht_pass<T, VW, CW, NB>), grid,
               dim3(kHThreads), 0, st, src, A, ld, m, n, b, seed, lo, ctiles, dst, C, ldb, avec);
}

// The P full passes over the columns [0, C) of [X | b] (X: m x n, row stride
// ld; b, if given, is column n = C - 1; pass 1 reads them with the signs D),
// ping-ponging between bufs[0] and bufs[1] (row stride ldb), VW columns per
// thread and CW packs per work-group.  view = true: X is a vector (n = C = 1,
// no b) and each pass after the first works on it as an (m' >> lo) x 2^lo
// matrix (bits [lo, lo + nb) of the index are bits [0, nb) of the view's
// row).  Returns the buffer holding the result.
template <typename T, int VW, int CW>
const T* had_passes(const HadPlan& p, const T* X, int64_t ld, int64_t m, int n, const T* b, int C,
                    bool view, uint64_t seed, T* const bufs[2], int ldb, bool avec, hipStream_t st,
                    sns_status* err) {
  const T* src = nullptr;
  int lo = 0, q0 = 0;
  if (view && p.L >= 8) {  // the vector's first pass over 8 bits
    const uint64_t nblk = p.mp >> 8, waves = kHThreads / 64;
    if ((nblk + waves - 1) / waves > 0x7FFFFFFFull) {
      *err = SNS_ERR_SHAPE;
      return nullptr;
    }
    SNS_LAUNCH("srht_vpass1", k_srht_vpass1<T>, dim3((unsigned)((nblk + waves - 1) / waves)),
               dim3(kHThreads), 0, st, X, m, seed, nblk, bufs[0]);
    src = bufs[0];
    lo = 8;
    q0 = 1;
  }
  for (int q = q0; q < p.P; ++q) {
    const int nb = (p.L - lo) < 8 ? (p.L - lo) : 8;
    T* dst = bufs[q & 1];
    if (view && lo > 24) {  // the view's row length 2^lo stays an int
      *err = SNS_ERR_SHAPE;
      return nullptr;
    }
    // view passes: lo' = 0 on a matrix of 2^lo columns
    const int vc = view && src ? (1 << lo) : C, vld = view && src ? (1 << lo) : ldb;
    const int vlo = view && src ? 0 : lo;
    const uint64_t vrows = view && src ? (p.mp >> lo) : p.mp;
    const int ctiles = (vc + CW * VW - 1) / (CW * VW);
    const uint64_t blocks = (vrows >> nb) * (uint64_t)ctiles;
    if (blocks > 0x7FFFFFFFull) {
      *err = SNS_ERR_SHAPE;
      return nullptr;
    }
    const dim3 grid((unsigned)blocks);
#define SNS_PASS(NBV)                                                                      \
  launch_pass<T, VW, CW, NBV>(grid, st, view, src, X, ld, m, n, b, seed, vlo, ctiles, dst, vc, \
                              vld, avec)
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
  return src;
}

// VW columns per thread, CW packs per work-group (a row segment of CW VW
// values: 128 bytes for fp32 with one column per thread, 256 with two, 256
// for fp64); b's vector passes take one column per thread.
template <typename T, int VW, int CW>
sns_status launch_had(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b, void* SA,
                      void* Sb, void* ws, hipStream_t st) {
  const HadPlan p = had_plan(A);
  const size_t mb = had_matrix_bytes(p, sizeof(T)), vb = had_vector_bytes(p, sizeof(T));
  char* w = static_cast<char*>(ws);
  T* const Bm[2] = {reinterpret_cast<T*>(w), reinterpret_cast<T*>(w + (p.nbuf - 1) * mb)};
  char* wv = w + p.nbuf * mb;
  T* const Bv[2] = {reinterpret_cast<T*>(wv), reinterpret_cast<T*>(wv + (p.nbuf - 1) * vb)};
  static_assert(32 % (CW * VW) == 0 || (CW * VW) % 32 == 0, "tiles inside the padded rows");
  static_assert(CW * VW == had_tile_of<T>(), "the plan's tile width");
  const int n = (int)A.n;
  const bool avec = reinterpret_cast<uintptr_t>(A.values) % (VW * sizeof(T)) == 0 && A.ld % VW == 0;
  const T* bt = static_cast<const T*>(b);
  const bool bcol = bt && !p.bvec;  // b as column n of the work buffers
  const int C = n + (b ? 1 : 0);
  sns_status err = SNS_OK;
  const T* rm = had_passes<T, VW, CW>(p, static_cast<const T*>(A.values), A.ld, A.m, n,
                                      bcol ? bt : nullptr, bcol ? C : n, false, seed, Bm, p.ldb,
                                      avec, st, &err);
  if (err != SNS_OK) return err;
  const T* rv = nullptr;
  if (bt && p.bvec) {
    rv = had_passes<T, 1, 32>(p, bt, 1, A.m, 1, nullptr, 1, true, seed, Bv, 1, true, st, &err);
    if (err != SNS_OK) return err;
  }
  const int stiles = (C + kHThreads - 1) / kHThreads;
  int lo = 0;
  for (int q = 0; q < p.P; ++q) lo += (p.L - lo) < 8 ? (p.L - lo) : 8;
  SNS_LAUNCH("srht_sample", k_srht_sample<T>, dim3((unsigned)(d * (uint64_t)stiles)),
             dim3(kHThreads), 0, st, rm, rv, C, p.ldb, lo, p.L, seed, stiles, n,
             1.0 / sqrt((double)d), static_cast<T*>(SA), static_cast<T*>(Sb));
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace

size_t hadamard_workspace_bytes(const sns_matrix& A, uint32_t /*d*/) {
  const HadPlan p = had_plan(A);
  const size_t es = A.dtype == SNS_F64 ? 8 : 4;
  return p.nbuf * (had_matrix_bytes(p, es) + had_vector_bytes(p, es));
}

sns_status launch_hadamard_sketch(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b,
                                  void* SA, void* Sb, void* ws, hipStream_t st) {
  if (A.layout != SNS_DENSE_ROWMAJOR) return SNS_ERR_DTYPE;
  if (A.dtype == SNS_F64) return launch_had<double, 1, 32>(A, d, seed, b, SA, Sb, ws, st);
  return launch_had<float, 2, 32>(A, d, seed, b, SA, Sb, ws, st);
}

}  // namespace sns
