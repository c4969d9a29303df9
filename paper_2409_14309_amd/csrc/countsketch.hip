// CountSketch apply (Clarkson-Woodruff sketch): SA[k, :] = sum over rows i in
// bucket k of s(i) A[i, :], and Sb[k] likewise, for a dense row-major A.
//
// After the stable bucket sort, bucket k's rows are a contiguous run of perm
// (ascending row id).  One work-group reduces one bucket (or one segment of a
// bucket when buckets are few and long) over one tile of columns: row-slots of
// LPR lanes stream whole rows (VEC elements per lane, coalesced), accumulate in
// registers in ascending perm order, and the slots are combined in LDS in a
// fixed order.  There are no atomics; the result depends only on the data,
// the seed and the launch shape.
#include "common.hpp"
#include "kernels.hpp"

namespace sns {

namespace {

template <typename T, int VEC>
struct Vec;
template <>
struct Vec<float, 4> { using type = float4; };
template <>
struct Vec<float, 2> { using type = float2; };
template <>
struct Vec<float, 1> { using type = float; };
template <>
struct Vec<double, 2> { using type = double2; };
template <>
struct Vec<double, 1> { using type = double; };

template <typename T, int VEC>
__device__ __forceinline__ void load_row(const T* __restrict__ p, int col, int n, T (&v)[VEC]) {
  if (col + VEC <= n) {
    using V = typename Vec<T, VEC>::type;
    const V x = *reinterpret_cast<const V*>(p + col);
    const T* e = reinterpret_cast<const T*>(&x);
#pragma unroll
    for (int q = 0; q < VEC; ++q) v[q] = e[q];
  } else {
#pragma unroll
    for (int q = 0; q < VEC; ++q) v[q] = (col + q < n) ? p[col + q] : T(0);
  }
}

template <typename T, typename Acc, int VEC, int LPR, int WAVES, int U>
__global__ __launch_bounds__(WAVES * 64) void k_cs_gather(
    const T* __restrict__ A, int64_t ld, int n, const uint32_t* __restrict__ perm,
    const T* __restrict__ bperm, const uint32_t* __restrict__ bucket_ptr, uint32_t d, int nseg,
    T* __restrict__ SA, T* __restrict__ Sb, Acc* __restrict__ partA, Acc* __restrict__ partB) {
  constexpr int RPW = 64 / LPR;
  constexpr int CT = LPR * VEC;
  constexpr int NS = WAVES * RPW;
  __shared__ Acc red[NS * CT];
  __shared__ Acc redb[NS];

  const uint32_t k = blockIdx.x / nseg;
  const int sg = blockIdx.x % nseg;
  const int64_t p0 = bucket_ptr[k], p1 = bucket_ptr[k + 1], len = p1 - p0;
  const int64_t s0 = p0 + len * sg / nseg, s1 = p0 + len * (sg + 1) / nseg;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int slot = wv * RPW + lane / LPR, lr = lane % LPR;
  const int col = blockIdx.y * CT + lr * VEC;
  const bool do_b = (bperm != nullptr) && blockIdx.y == 0;

  Acc acc[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q) acc[q] = Acc(0);
  Acc accb = Acc(0);

  for (int64_t p = s0 + slot; p < s1; p += (int64_t)NS * U) {
    uint32_t e[U];
    T v[U][VEC];
    T bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t pu = p + (int64_t)u * NS;
      e[u] = pu < s1 ? perm[pu] : 0xFFFFFFFFu;
      bv[u] = (do_b && pu < s1) ? bperm[pu] : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (e[u] != 0xFFFFFFFFu) {
        const int64_t i = e[u] & 0x7FFFFFFFu;
        load_row<T, VEC>(A + i * ld, col, n, v[u]);
      } else {
#pragma unroll
        for (int q = 0; q < VEC; ++q) v[u][q] = T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool neg = (e[u] >> 31) && e[u] != 0xFFFFFFFFu;
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        const Acc x = (Acc)v[u][q];
        acc[q] += neg ? -x : x;
      }
      accb += (Acc)bv[u];
    }
  }

#pragma unroll
  for (int q = 0; q < VEC; ++q) red[slot * CT + lr * VEC + q] = acc[q];
  if (lr == 0) redb[slot] = accb;
  __syncthreads();
  for (int t = threadIdx.x; t < CT; t += blockDim.x) {
    Acc s = Acc(0);
    for (int q = 0; q < NS; ++q) s += red[q * CT + t];
    const int c = blockIdx.y * CT + t;
    if (c < n) {
      if (nseg == 1) SA[(size_t)k * n + c] = (T)s;
      else partA[((size_t)sg * d + k) * n + c] = s;
    }
  }
  if (do_b && threadIdx.x == 0) {
    Acc s = Acc(0);
    for (int q = 0; q < NS; ++q) s += redb[q];
    if (nseg == 1) Sb[k] = (T)s;
    else partB[(size_t)sg * d + k] = s;
  }
}

// SA = sum over segments (ascending) of the partial sketches.
template <typename T, typename Acc>
__global__ void k_seg_reduce(int64_t dn, int64_t d, int nseg, const Acc* __restrict__ partA,
                             const Acc* __restrict__ partB, T* __restrict__ SA,
                             T* __restrict__ Sb) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < dn + d;
       t += (int64_t)gridDim.x * blockDim.x) {
    if (t < dn) {
      Acc s = Acc(0);
      for (int g = 0; g < nseg; ++g) s += partA[(size_t)g * dn + t];
      SA[t] = (T)s;
    } else if (partB) {
      const int64_t k = t - dn;
      Acc s = Acc(0);
      for (int g = 0; g < nseg; ++g) s += partB[(size_t)g * d + k];
      Sb[k] = (T)s;
    }
  }
}

constexpr int kWaves = 4;
constexpr int kUnroll = 4;

template <typename T, typename Acc, int VEC, int LPR>
void launch_one(const GatherPlan& g, const sns_matrix& A, uint32_t d, const SortBufs& s,
                bool with_b, void* SA, void* Sb, void* part, hipStream_t st) {
  const dim3 grid(d * g.nseg, g.coltiles);
  Acc* pa = g.nseg > 1 ? static_cast<Acc*>(part) : nullptr;
  Acc* pb = (g.nseg > 1 && with_b) ? pa + (size_t)g.nseg * d * A.n : nullptr;
  SNS_LAUNCH("cs_gather", (k_cs_gather<T, Acc, VEC, LPR, kWaves, kUnroll>), grid, dim3(kWaves * 64), 0,
                     st, static_cast<const T*>(A.values), A.ld, (int)A.n, s.perm,
                     with_b ? static_cast<const T*>(s.bperm) : nullptr, s.bucket_ptr, d, g.nseg,
                     static_cast<T*>(SA), static_cast<T*>(Sb), pa, pb);
  if (g.nseg > 1) {
    const int64_t dn = (int64_t)d * A.n;
    int64_t blocks = (dn + d + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    SNS_LAUNCH("seg_reduce", (k_seg_reduce<T, Acc>), dim3((unsigned)blocks), dim3(256), 0, st, dn,
                       (int64_t)d, g.nseg, pa, pb, static_cast<T*>(SA),
                       with_b ? static_cast<T*>(Sb) : nullptr);
  }
}

template <typename T, typename Acc, int VEC>
void dispatch_lpr(const GatherPlan& g, const sns_matrix& A, uint32_t d, const SortBufs& s,
                  bool with_b, void* SA, void* Sb, void* part, hipStream_t st) {
  switch (g.lpr) {
    case 4: launch_one<T, Acc, VEC, 4>(g, A, d, s, with_b, SA, Sb, part, st); break;
    case 8: launch_one<T, Acc, VEC, 8>(g, A, d, s, with_b, SA, Sb, part, st); break;
    case 16: launch_one<T, Acc, VEC, 16>(g, A, d, s, with_b, SA, Sb, part, st); break;
    case 32: launch_one<T, Acc, VEC, 32>(g, A, d, s, with_b, SA, Sb, part, st); break;
    default: launch_one<T, Acc, VEC, 64>(g, A, d, s, with_b, SA, Sb, part, st); break;
  }
}

}  // namespace

GatherPlan make_gather_plan(const sns_matrix& A, uint32_t d, bool acc64) {
  GatherPlan g;
  const size_t es = A.dtype == SNS_F64 ? 8 : 4;
  const int vmax = (int)(16 / es);
  const bool aligned = ((uintptr_t)A.values % 16 == 0) && (A.ld % vmax == 0);
  g.vec = aligned ? vmax : 1;
  const int64_t lanes = (A.n + g.vec - 1) / g.vec;
  int lpr = 4;
  while (lpr < 64 && lpr < lanes) lpr <<= 1;
  g.lpr = lpr;
  g.ct = lpr * g.vec;
  g.coltiles = (int)((A.n + g.ct - 1) / g.ct);
  g.acc64 = acc64 || A.dtype == SNS_F64;
  // enough work-groups to fill the device, each segment keeping >= 256 rows
  const int64_t wgs = (int64_t)d * g.coltiles;
  int64_t nseg = (1024 + wgs - 1) / wgs;
  const int64_t maxseg = A.m / ((int64_t)d * 256);
  if (nseg > maxseg) nseg = maxseg;
  if (nseg < 1) nseg = 1;
  if (nseg > 64) nseg = 64;
  g.nseg = (int)nseg;
  return g;
}

size_t gather_partial_bytes(const GatherPlan& g, const sns_matrix& A, uint32_t d) {
  if (g.nseg <= 1) return 0;
  return (size_t)g.nseg * d * (A.n + 1) * (g.acc64 ? 8 : 4);
}

sns_status launch_cs_gather(const GatherPlan& g, const sns_matrix& A, uint32_t d,
                            const SortBufs& s, bool with_b, void* SA, void* Sb, void* part,
                            hipStream_t st) {
  if (A.dtype == SNS_F64) {
    if (g.vec == 2) dispatch_lpr<double, double, 2>(g, A, d, s, with_b, SA, Sb, part, st);
    else dispatch_lpr<double, double, 1>(g, A, d, s, with_b, SA, Sb, part, st);
  } else if (g.acc64) {
    if (g.vec == 4) dispatch_lpr<float, double, 4>(g, A, d, s, with_b, SA, Sb, part, st);
    else dispatch_lpr<float, double, 1>(g, A, d, s, with_b, SA, Sb, part, st);
  } else {
    if (g.vec == 4) dispatch_lpr<float, float, 4>(g, A, d, s, with_b, SA, Sb, part, st);
    else dispatch_lpr<float, float, 1>(g, A, d, s, with_b, SA, Sb, part, st);
  }
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace sns
