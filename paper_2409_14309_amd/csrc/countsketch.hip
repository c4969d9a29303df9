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

// Rows of A are read once per sketch: nontemporal loads keep the stream from
// displacing the partial sums and permutation in the caches.
template <typename T, int VEC>
__device__ __forceinline__ void load_row(const T* __restrict__ p, int col, int n, T (&v)[VEC]) {
  if (col + VEC <= n) {
    typedef T NVT __attribute__((ext_vector_type(VEC)));
    const NVT x = __builtin_nontemporal_load(reinterpret_cast<const NVT*>(p + col));
#pragma unroll
    for (int q = 0; q < VEC; ++q) v[q] = x[q];
  } else {
#pragma unroll
    for (int q = 0; q < VEC; ++q) v[q] = (col + q < n) ? p[col + q] : T(0);
  }
}

// One work item: bucket k, segment sg, column tile ct of one problem.
template <typename T, typename Acc, int VEC, int LPR, int WAVES, int U>
__device__ __forceinline__ void cs_gather_item(const GatherArgs& a, uint32_t loc, Acc* red,
                                               Acc* redb) {
  constexpr int RPW = 64 / LPR;
  constexpr int CT = LPR * VEC;
  constexpr int NS = WAVES * RPW;
  const T* __restrict__ A = static_cast<const T*>(a.A);
  const T* __restrict__ bperm = static_cast<const T*>(a.bperm);
  const int64_t ld = a.ld;
  const int n = a.n, nseg = a.nseg;
  const uint32_t d = a.d;
  const uint32_t bx = loc % (d * (uint32_t)nseg), ct = loc / (d * (uint32_t)nseg);
  const uint32_t k = bx / nseg;
  const int sg = bx % nseg;
  const int64_t p0 = a.bucket_ptr[k], p1 = a.bucket_ptr[k + 1], len = p1 - p0;
  const int64_t s0 = p0 + len * sg / nseg, s1 = p0 + len * (sg + 1) / nseg;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int slot = wv * RPW + lane / LPR, lr = lane % LPR;
  const int col = ct * CT + lr * VEC;
  const bool do_b = (bperm != nullptr) && ct == 0;

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
      e[u] = pu < s1 ? a.perm[pu] : 0xFFFFFFFFu;
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
    const int c = ct * CT + t;
    if (c < n) {
      if (nseg == 1) static_cast<T*>(a.SA)[(size_t)k * n + c] = (T)s;
      else static_cast<Acc*>(a.partA)[((size_t)sg * d + k) * n + c] = s;
    }
  }
  if (do_b && threadIdx.x == 0) {
    Acc s = Acc(0);
    for (int q = 0; q < NS; ++q) s += redb[q];
    if (nseg == 1) static_cast<T*>(a.Sb)[k] = (T)s;
    else static_cast<Acc*>(a.partB)[(size_t)sg * d + k] = s;
  }
}

template <typename T, typename Acc, int VEC, int LPR, int WAVES, int U>
__global__ __launch_bounds__(WAVES * 64) void k_cs_gather(const GatherArgs* __restrict__ P,
                                                          Map mp) {
  constexpr int CT = LPR * VEC;
  constexpr int NS = WAVES * (64 / LPR);
  __shared__ Acc red[NS * CT];
  __shared__ Acc redb[NS];
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const int pi = map_find(mp, it);
  cs_gather_item<T, Acc, VEC, LPR, WAVES, U>(P[pi], it - mp.off[pi], red, redb);
}

// SA = sum over segments (ascending) of the partial sketches.  A work item is
// 256 consecutive outputs of one problem.
template <typename T, typename Acc>
__global__ void k_seg_reduce(const GatherArgs* __restrict__ P, Map mp) {
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const int pi = map_find(mp, it);
  const GatherArgs& a = P[pi];
  const uint32_t loc = it - mp.off[pi];
  const int64_t d = a.d, dn = d * a.n;
  const Acc* partA = static_cast<const Acc*>(a.partA);
  const Acc* partB = static_cast<const Acc*>(a.partB);
  for (int64_t t = (int64_t)loc * blockDim.x + threadIdx.x; t < dn + d;
       t += (int64_t)a.red_blocks * blockDim.x) {
    if (t < dn) {
      Acc s = Acc(0);
      for (int g = 0; g < a.nseg; ++g) s += partA[(size_t)g * dn + t];
      static_cast<T*>(a.SA)[t] = (T)s;
    } else if (a.bperm) {
      const int64_t k = t - dn;
      Acc s = Acc(0);
      for (int g = 0; g < a.nseg; ++g) s += partB[(size_t)g * d + k];
      static_cast<T*>(a.Sb)[k] = (T)s;
    }
  }
}

constexpr int kWaves = 4;
constexpr int kUnroll = 4;

template <typename T, typename Acc, int VEC, int LPR>
void launch_one(const GatherLaunch& g, hipStream_t st) {
  SNS_LAUNCH("cs_gather", (k_cs_gather<T, Acc, VEC, LPR, kWaves, kUnroll>), dim3(grid_for(g.items)),
             dim3(kWaves * 64), 0, st, g.args, g.map);
  if (g.ritems)
    SNS_LAUNCH("seg_reduce", (k_seg_reduce<T, Acc>), dim3(grid_for(g.ritems)), dim3(256), 0, st,
               g.rargs, g.rmap);
}

template <typename T, typename Acc, int VEC>
void dispatch_lpr(const GatherLaunch& g, hipStream_t st) {
  switch (g.plan.lpr) {
    case 4: launch_one<T, Acc, VEC, 4>(g, st); break;
    case 8: launch_one<T, Acc, VEC, 8>(g, st); break;
    case 16: launch_one<T, Acc, VEC, 16>(g, st); break;
    case 32: launch_one<T, Acc, VEC, 32>(g, st); break;
    default: launch_one<T, Acc, VEC, 64>(g, st); break;
  }
}

}  // namespace

GatherPlan gather_plan_with(const sns_matrix& A, uint32_t d, bool acc64, int64_t keys, int lpr,
                            int nseg) {
  GatherPlan g;
  const size_t es = A.dtype == SNS_F64 ? 8 : 4;
  const int vmax = (int)(16 / es);
  const bool aligned = ((uintptr_t)A.values % 16 == 0) && (A.ld % vmax == 0);
  g.vec = aligned ? vmax : 1;
  g.lpr = lpr < 4 ? 4 : (lpr > 64 ? 64 : lpr);
  g.ct = g.lpr * g.vec;
  g.coltiles = (int)((A.n + g.ct - 1) / g.ct);
  g.acc64 = acc64 || A.dtype == SNS_F64;
  const int64_t maxseg = (keys >= 0 ? keys : A.m) / ((int64_t)d * 256);
  int64_t ns = nseg;
  if (ns > maxseg) ns = maxseg;
  if (ns < 1) ns = 1;
  if (ns > 64) ns = 64;
  g.nseg = (int)ns;
  return g;
}

GatherPlan make_gather_plan(const sns_matrix& A, uint32_t d, bool acc64, int64_t keys) {
  const size_t es = A.dtype == SNS_F64 ? 8 : 4;
  const int vmax = (int)(16 / es);
  const bool aligned = ((uintptr_t)A.values % 16 == 0) && (A.ld % vmax == 0);
  const int vec = aligned ? vmax : 1;
  int tl = 0, ts = 0;
  if (tune_gather_lookup(A.dtype, A.n, d, keys >= 0 ? keys : A.m, &tl, &ts))
    return gather_plan_with(A, d, acc64, keys, tl, ts);
  // built-in rule: the fewest lanes per row that cover n in one column tile,
  // and enough work-groups to fill the device, each segment keeping >= 256 rows
  const int64_t lanes = (A.n + vec - 1) / vec;
  int lpr = 4;
  while (lpr < 64 && lpr < lanes) lpr <<= 1;
  const int64_t coltiles = (A.n + (int64_t)lpr * vec - 1) / ((int64_t)lpr * vec);
  const int64_t wgs = (int64_t)d * coltiles;
  int64_t nseg = (1024 + wgs - 1) / wgs;
  return gather_plan_with(A, d, acc64, keys, lpr, (int)(nseg > 64 ? 64 : nseg));
}

size_t gather_partial_bytes(const GatherPlan& g, const sns_matrix& A, uint32_t d) {
  if (g.nseg <= 1) return 0;
  return (size_t)g.nseg * d * (A.n + 1) * (g.acc64 ? 8 : 4);
}

GatherArgs gather_args(const GatherPlan& g, const sns_matrix& A, uint32_t d, const SortBufs& s,
                       bool with_b, void* SA, void* Sb, void* part) {
  GatherArgs a;
  a.A = A.values;
  a.ld = A.ld;
  a.n = (int)A.n;
  a.nseg = g.nseg;
  a.coltiles = g.coltiles;
  a.d = d;
  a.perm = s.perm;
  a.bperm = with_b ? s.bperm : nullptr;
  a.bucket_ptr = s.bucket_ptr;
  a.SA = SA;
  a.Sb = with_b ? Sb : nullptr;
  const size_t ab = g.acc64 ? 8 : 4;
  a.partA = g.nseg > 1 ? part : nullptr;
  a.partB = (g.nseg > 1 && with_b) ? static_cast<char*>(part) + (size_t)g.nseg * d * A.n * ab
                                   : nullptr;
  const int64_t dn = (int64_t)d * A.n;
  int64_t blocks = (dn + d + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  a.red_blocks = (int)blocks;
  return a;
}

std::vector<GatherLaunch> build_gather_job(ArgTable& t, const std::vector<GatherProb>& p) {
  std::vector<GatherLaunch> out;
  std::vector<bool> used(p.size(), false);
  for (size_t i = 0; i < p.size(); ++i) {
    if (used[i]) continue;
    GatherLaunch g;
    g.plan = p[i].plan;
    g.dtype = p[i].dtype;
    std::vector<GatherArgs> args, rargs;
    std::vector<uint32_t> cnt, rcnt;
    for (size_t k = i; k < p.size(); ++k) {
      const GatherPlan& q = p[k].plan;
      if (used[k] || p[k].dtype != g.dtype || q.vec != g.plan.vec || q.lpr != g.plan.lpr ||
          q.acc64 != g.plan.acc64)
        continue;
      used[k] = true;
      args.push_back(p[k].args);
      cnt.push_back(p[k].args.d * (uint32_t)q.nseg * (uint32_t)q.coltiles);
      if (q.nseg > 1) {
        rargs.push_back(p[k].args);
        rcnt.push_back((uint32_t)p[k].args.red_blocks);
      }
    }
    g.args = t.add(args.data(), args.size());
    g.map = t.map(cnt, &g.items);
    g.rargs = nullptr;
    g.rmap = Map{nullptr, 0};
    g.ritems = 0;
    if (!rargs.empty()) {
      g.rargs = t.add(rargs.data(), rargs.size());
      g.rmap = t.map(rcnt, &g.ritems);
    }
    out.push_back(g);
  }
  return out;
}

sns_status launch_gather_job(const std::vector<GatherLaunch>& j, hipStream_t st) {
  for (const GatherLaunch& g : j) {
    if (g.dtype == SNS_F64) {
      if (g.plan.vec == 2) dispatch_lpr<double, double, 2>(g, st);
      else dispatch_lpr<double, double, 1>(g, st);
    } else if (g.plan.acc64) {
      if (g.plan.vec == 4) dispatch_lpr<float, double, 4>(g, st);
      else dispatch_lpr<float, double, 1>(g, st);
    } else {
      if (g.plan.vec == 4) dispatch_lpr<float, float, 4>(g, st);
      else dispatch_lpr<float, float, 1>(g, st);
    }
  }
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace sns
