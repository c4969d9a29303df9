// CountSketch of a sparse matrix in CSR form (Clarkson-Woodruff sketch over
// the rows of A): SA[k, j] = sum over rows i with h(i) = k of s(i) A[i, j],
// Sb[k] = sum over all rows with h(i) = k of s(i) b[i].
//
// Only rows that hold nonzeros touch SA.  They are compacted in ascending
// order (block counts, scan, ordered write), sorted by bucket with the same
// stable counting sort as the dense path (fed the compacted row list; its
// length stays on the device), and each bucket is reduced by one work-group.
// Each wave takes a contiguous share of the bucket's rows, 64 rows at a time:
// the rows' nonzeros are enumerated as one flat sequence (prefix sum of the
// row lengths across lanes, binary search per lane), 64 nonzeros per step,
// and added into a private LDS copy of the output row.
//
// Sb covers every row of b.  Each wave streams a contiguous range of rows,
// 128 at a time (one Philox call per pair of rows), into a private LDS copy of
// Sb; per-group partials are summed in order by a two-stage reduction.
//
// Lanes of one step that hit the same LDS slot are resolved in rounds: each
// round the lowest such lane (integer LDS min on a tag array) adds, so equal
// keys add in ascending lane order, which is ascending row order.  No
// floating-point atomics anywhere; the result depends only on the inputs, the
// seed and the launch shape.
#include "common.hpp"
#include "kernels.hpp"

namespace sns {

namespace {

constexpr int kRowsPerBlock = 8192;  // rows per compaction work-group
constexpr int kCompactThreads = 256;
constexpr size_t kLdsBudget = 65536;  // bytes of LDS per work-group

// per-block counts of nonempty rows
__global__ __launch_bounds__(kCompactThreads) void k_csr_count(int64_t m,
                                                               const int32_t* __restrict__ rp,
                                                               uint32_t* __restrict__ bcount) {
  __shared__ uint32_t red[kCompactThreads / 64];
  const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock;
  const int64_t r1 = r0 + kRowsPerBlock < m ? r0 + kRowsPerBlock : m;
  uint32_t c = 0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += kCompactThreads) c += rp[i + 1] > rp[i] ? 1u : 0u;
  c = block_sum(c, red);
  if (threadIdx.x == 0) bcount[blockIdx.x] = c;
}

// exclusive scan of the block counts (one work-group); total -> *total
__global__ __launch_bounds__(1024) void k_csr_scan(int nb, uint32_t* __restrict__ bcount,
                                                   uint32_t* __restrict__ total) {
  __shared__ uint32_t wsum[16];
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (nb + nt - 1) / nt;
  const int b0 = t * per < nb ? t * per : nb, b1 = b0 + per < nb ? b0 + per : nb;
  uint32_t local = 0;
  for (int k = b0; k < b1; ++k) local += bcount[k];
  const int lane = t & 63, wv = t >> 6;
  uint32_t incl = local;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  uint32_t run = incl - local;
  for (int w = 0; w < wv; ++w) run += wsum[w];
  for (int k = b0; k < b1; ++k) {
    const uint32_t c = bcount[k];
    bcount[k] = run;
    run += c;
  }
  if (t == nt - 1) *total = run;
}

// Ascending list of nonempty rows.  A block takes kRowsPerBlock rows in
// rounds of 256 (coalesced loads, all issued up front); a row's slot is the
// block offset plus the nonempty rows before it in round-major order.
__global__ __launch_bounds__(kCompactThreads) void k_csr_compact(int64_t m,
                                                                 const int32_t* __restrict__ rp,
                                                                 const uint32_t* __restrict__ boff,
                                                                 uint32_t* __restrict__ list) {
  constexpr int kRounds = kRowsPerBlock / kCompactThreads;
  constexpr int kWaves = kCompactThreads / 64;
  __shared__ uint32_t wcnt[kRounds][kWaves];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock + t;
  uint32_t fl = 0;
#pragma unroll
  for (int q = 0; q < kRounds; ++q) {
    const int64_t i = r0 + (int64_t)q * kCompactThreads;
    if (i < m && rp[i + 1] > rp[i]) fl |= 1u << q;
  }
  const uint64_t below = (uint64_t(1) << lane) - 1;
#pragma unroll
  for (int q = 0; q < kRounds; ++q) {
    const uint64_t bq = __ballot((fl >> q) & 1u);
    if (lane == 0) wcnt[q][wv] = (uint32_t)__popcll(bq);
  }
  __syncthreads();
  uint32_t run = boff[blockIdx.x];
  for (int q = 0; q < kRounds; ++q) {
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wcnt[q][w];
      before += w < wv ? c : 0u;
      tot += c;
    }
    const uint64_t bq = __ballot((fl >> q) & 1u);
    if ((fl >> q) & 1u)
      list[run + before + (uint32_t)__popcll(bq & below)] = (uint32_t)(r0 + (int64_t)q * kCompactThreads);
    run += tot;
  }
}

// acc[key] += x for every active lane of the wave.  Lanes with equal keys add
// one per round, lowest lane first.  tag is the wave's own scratch, indexed
// like acc; no initial contents are assumed.
template <typename Acc>
__device__ __forceinline__ void wave_scatter_add(Acc* acc, uint32_t* tag, bool act, uint32_t key,
                                                 Acc x, uint32_t lane) {
  while (__ballot(act)) {
    if (act) tag[key] = 0xFFFFFFFFu;
    if (act) atomicMin(&tag[key], lane);
    if (act && tag[key] == lane) {
      acc[key] += x;
      act = false;
    }
  }
}

// SA[k, :] for bucket k = blockIdx.x, `waves` waves each with n accumulators
// and n tags in LDS.
template <typename T, typename Acc>
__global__ __launch_bounds__(256) void k_csr_gather(
    int n, int waves, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
    const T* __restrict__ vals, const uint32_t* __restrict__ perm,
    const uint32_t* __restrict__ bucket_ptr, T* __restrict__ SA) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  Acc* acc = reinterpret_cast<Acc*>(lds_raw);
  uint32_t* tag = reinterpret_cast<uint32_t*>(lds_raw + (size_t)waves * n * sizeof(Acc));
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const uint32_t k = blockIdx.x;
  for (int j = t; j < waves * n; j += blockDim.x) acc[j] = Acc(0);
  __syncthreads();
  Acc* mine = acc + (size_t)wv * n;
  uint32_t* mytag = tag + (size_t)wv * n;
  const uint32_t p0 = bucket_ptr[k], p1 = bucket_ptr[k + 1];
  const uint64_t cnt = p1 - p0;
  const uint32_t r0 = p0 + (uint32_t)(cnt * wv / waves), r1 = p0 + (uint32_t)(cnt * (wv + 1) / waves);
  for (uint32_t r = r0; r < r1; r += 64) {
    const uint32_t p = r + lane;
    int s0 = 0, len = 0, neg = 0;
    if (p < r1) {
      const uint32_t e = perm[p];
      const int64_t i = e & 0x7FFFFFFFu;
      neg = (int)(e >> 31);
      s0 = rp[i];
      len = rp[i + 1] - s0;
    }
    int P = len;  // inclusive prefix of the row lengths over lanes
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(P, off, 64);
      if (lane >= off) P += y;
    }
    const int E = P - len;
    const int total = __shfl(P, 63, 64);
    // flat nonzero e -> its index q in ci/vals and its row's sign
    auto locate = [&](int e, int& q, int& nq) {
      int pos = 0;  // number of lanes whose inclusive prefix is <= e
#pragma unroll
      for (int s = 32; s >= 1; s >>= 1)
        if (__shfl(P, pos + s - 1, 64) <= e) pos += s;
      q = __shfl(s0, pos, 64) + (e - __shfl(E, pos, 64));
      nq = __shfl(neg, pos, 64);
    };
    int q, nq;
    bool valid = lane < total;
    locate(lane, q, nq);
    uint32_t j = 0;
    T v = T(0);
    if (valid) {
      j = (uint32_t)ci[q];
      v = vals[q];
    }
    for (int c = 0; c < total; c += 64) {
      // the next step's nonzeros are in flight while this step adds
      const int e2 = c + 64 + lane;
      const bool valid2 = e2 < total;
      int q2, nq2;
      locate(e2, q2, nq2);
      uint32_t j2 = 0;
      T v2 = T(0);
      if (valid2) {
        j2 = (uint32_t)ci[q2];
        v2 = vals[q2];
      }
      const Acc x = nq ? -(Acc)v : (Acc)v;
      // columns outside [0, n) are ignored
      wave_scatter_add(mine, mytag, valid && j < (uint32_t)n, j, x, (uint32_t)lane);
      j = j2;
      v = v2;
      valid = valid2;
      nq = nq2;
    }
  }
  __syncthreads();
  for (int j = t; j < n; j += blockDim.x) {
    Acc s = Acc(0);
    for (int w = 0; w < waves; ++w) s += acc[(size_t)w * n + j];
    SA[(size_t)k * n + j] = (T)s;
  }
}

// Partial Sb of a contiguous range of 128-row batches per wave, for buckets
// [k0, k0 + span).  part[blockIdx.x * d + k].
template <typename T, typename Acc>
__global__ __launch_bounds__(256) void k_vec_sketch(int64_t m, uint32_t d, uint64_t seed, int waves,
                                                    uint32_t span, const T* __restrict__ b,
                                                    Acc* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  Acc* acc = reinterpret_cast<Acc*>(lds_raw);
  uint32_t* tag = reinterpret_cast<uint32_t*>(lds_raw + (size_t)waves * span * sizeof(Acc));
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const uint32_t k0 = blockIdx.y * span;
  const uint32_t kn = d - k0 < span ? d - k0 : span;
  for (uint32_t j = t; j < (uint32_t)waves * span; j += blockDim.x) acc[j] = Acc(0);
  __syncthreads();
  Acc* mine = acc + (size_t)wv * span;
  uint32_t* mytag = tag + (size_t)wv * span;
  const int64_t nbat = (m + 127) / 128;
  const int64_t W = (int64_t)gridDim.x * waves, gw = (int64_t)blockIdx.x * waves + wv;
  const int64_t b0 = nbat * gw / W, b1 = nbat * (gw + 1) / W;
  T ve = T(0), vo = T(0);
  if (b0 < b1) {
    const int64_t i = 2 * (b0 * 64 + lane);
    if (i < m) ve = b[i];
    if (i + 1 < m) vo = b[i + 1];
  }
  for (int64_t bt = b0; bt < b1; ++bt) {
    const int64_t j = bt * 64 + lane, i = 2 * j;
    const T ce = ve, co = vo;
    if (bt + 1 < b1) {  // next batch in flight while this one is added
      const int64_t in = i + 128;
      ve = in < m ? b[in] : T(0);
      vo = in + 1 < m ? b[in + 1] : T(0);
    }
    Hash he, ho;
    cs_hash_pair(seed, d, (uint64_t)j, he, ho);
    const uint32_t ke = he.h - k0, ko = ho.h - k0;
    const Acc xe = he.neg ? -(Acc)ce : (Acc)ce, xo = ho.neg ? -(Acc)co : (Acc)co;
    wave_scatter_add(mine, mytag, i < m && ke < kn, ke, xe, (uint32_t)lane);
    wave_scatter_add(mine, mytag, i + 1 < m && ko < kn, ko, xo, (uint32_t)lane);
  }
  __syncthreads();
  for (uint32_t k = t; k < kn; k += blockDim.x) {
    Acc s = Acc(0);
    for (int w = 0; w < waves; ++w) s += acc[(size_t)w * span + k];
    part[(size_t)blockIdx.x * d + k0 + k] = s;
  }
}

// out[y * d + k] = sum of in[g * d + k] over g in [y * chunk, (y + 1) * chunk)
// (ascending g), for k < d.
template <typename Acc, typename O>
__global__ __launch_bounds__(256) void k_vec_reduce(uint32_t d, int G, int chunk,
                                                    const Acc* __restrict__ in, O* __restrict__ out) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d) return;
  const int g0 = blockIdx.y * chunk, g1 = g0 + chunk < G ? g0 + chunk : G;
  Acc s = Acc(0);
#pragma unroll 8
  for (int g = g0; g < g1; ++g) s += in[(size_t)g * d + k];
  out[(size_t)blockIdx.y * d + k] = (O)s;
}

constexpr int kReduceChunk = 32;

struct CsrPlan {
  int nb = 0;          // compaction blocks
  SortPlan sp;         // sort of up to m keys
  int gwaves = 1;      // waves per bucket work-group
  int vgrid = 1;       // Sb work-groups (row ranges)
  int vwaves = 1;      // waves (LDS copies) per Sb work-group
  int vsplit = 1;      // bucket ranges when one copy of Sb does not fit LDS
  uint32_t vspan = 0;  // buckets per range
  int rsplit = 1;      // first-stage reduction outputs
};

CsrPlan make_csr_plan(const sns_matrix& A, uint32_t d, bool acc64) {
  CsrPlan c;
  const size_t per = (acc64 ? 8 : 4) + 4;  // accumulator + tag bytes
  c.nb = (int)((A.m + kRowsPerBlock - 1) / kRowsPerBlock);
  // at most min(m, nnz) rows hold nonzeros; the exact count stays on the device
  const int64_t keys = A.nnz < A.m ? A.nnz : A.m;
  c.sp = make_sort_plan(keys > 0 ? keys : 1, d);
  size_t gw = kLdsBudget / ((size_t)A.n * per);
  c.gwaves = (int)(gw < 1 ? 1 : (gw > 4 ? 4 : gw));
  const size_t cap = kLdsBudget / per;  // buckets one work-group can hold
  if (d <= cap) {
    const size_t w = cap / d;
    c.vwaves = (int)(w > 4 ? 4 : w);
    c.vsplit = 1;
    c.vspan = d;
  } else {
    c.vwaves = 1;
    c.vsplit = (int)((d + cap - 1) / cap);
    c.vspan = (d + c.vsplit - 1) / c.vsplit;
  }
  // about 8K rows per wave, at most 2048 waves in all
  int64_t g = (A.m + 8192 * c.vwaves - 1) / (8192 * c.vwaves);
  const int64_t gmax = 2048 / c.vwaves;
  c.vgrid = (int)(g < 1 ? 1 : (g > gmax ? gmax : g));
  c.rsplit = (c.vgrid + kReduceChunk - 1) / kReduceChunk;
  return c;
}

constexpr size_t kCsrArgBytes = 4096;  // argument table of the row sort

struct CsrBufs {
  char* args;
  uint32_t* bcount;
  uint32_t* total;
  uint32_t* list;
  SortBufs sb;
  void* vpart;
  void* vpart2;
};

void carve_csr(Carve& c, const sns_matrix& A, uint32_t d, bool acc64, const CsrPlan& p,
               CsrBufs& b) {
  const size_t ab = acc64 ? 8 : 4;
  b.args = c.take<char>(kCsrArgBytes);
  b.bcount = c.take<uint32_t>((size_t)p.nb + 1);
  b.total = c.take<uint32_t>(1);
  b.list = c.take<uint32_t>((size_t)A.m);
  carve_sort(c, p.sp, 0, b.sb);
  b.vpart = c.take<char>((size_t)p.vgrid * d * ab);
  b.vpart2 = c.take<char>((size_t)p.rsplit * d * ab);
}

template <typename T, typename Acc>
void launch_csr_t(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b, void* SA, void* Sb,
                  const CsrPlan& p, const CsrBufs& bf, hipStream_t st) {
  const size_t lds_g = (size_t)p.gwaves * A.n * (sizeof(Acc) + 4);
  SNS_LAUNCH("csr_gather", (k_csr_gather<T, Acc>), dim3(d), dim3(p.gwaves * 64), lds_g, st,
             (int)A.n, p.gwaves, A.row_ptr, A.col_idx, static_cast<const T*>(A.values), bf.sb.perm,
             bf.sb.bucket_ptr, static_cast<T*>(SA));
  if (!b) return;
  const size_t lds_v = (size_t)p.vwaves * p.vspan * (sizeof(Acc) + 4);
  SNS_LAUNCH("vec_sketch", (k_vec_sketch<T, Acc>), dim3(p.vgrid, p.vsplit), dim3(p.vwaves * 64),
             lds_v, st, A.m, d, seed, p.vwaves, p.vspan, static_cast<const T*>(b),
             static_cast<Acc*>(bf.vpart));
  const dim3 rg((d + 255) / 256, p.rsplit);
  SNS_LAUNCH("vec_reduce", (k_vec_reduce<Acc, Acc>), rg, dim3(256), 0, st, d, p.vgrid, kReduceChunk,
             static_cast<const Acc*>(bf.vpart), static_cast<Acc*>(bf.vpart2));
  SNS_LAUNCH("vec_reduce", (k_vec_reduce<Acc, T>), dim3((d + 255) / 256, 1), dim3(256), 0, st, d,
             p.rsplit, p.rsplit, static_cast<const Acc*>(bf.vpart2), static_cast<T*>(Sb));
}

}  // namespace

// The CSR sketch always accumulates in fp64 (acc64 is accepted for the
// dense path's signature and ignored): each entry of Sb sums about m / d
// values of b (4,200 at 2^24 rows, d = 4000) with heavy cancellation, and fp32
// partial sums of that length move x0 by more than 1e-5.  The sketch here is
// bound by row_ptr and b traffic and by latency, not by the accumulator width.
size_t csr_workspace_bytes(const sns_matrix& A, uint32_t d, bool acc64) {
  (void)acc64;
  const bool a64 = true;
  Carve c(nullptr, 0);
  const CsrPlan p = make_csr_plan(A, d, a64);
  CsrBufs b;
  carve_csr(c, A, d, a64, p, b);
  return c.off;
}

sns_status launch_csr_sketch(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b,
                             void* SA, void* Sb, bool acc64, void* ws, size_t ws_bytes,
                             hipStream_t st) {
  (void)acc64;
  const bool a64 = true;
  // one wave's accumulators and tags for an output row must fit in LDS
  if ((size_t)A.n * ((a64 ? 8 : 4) + 4) > kLdsBudget) return SNS_ERR_SHAPE;
  Carve c(ws, ws_bytes);
  const CsrPlan p = make_csr_plan(A, d, a64);
  CsrBufs bf;
  carve_csr(c, A, d, a64, p, bf);
  if (!c.ok()) return SNS_ERR_OUT_OF_MEMORY;
  region_begin("csr_sketch", st);
  SNS_LAUNCH("csr_count", k_csr_count, dim3(p.nb), dim3(kCompactThreads), 0, st, A.m, A.row_ptr,
             bf.bcount);
  SNS_LAUNCH("csr_scan", k_csr_scan, dim3(1), dim3(1024), 0, st, p.nb, bf.bcount, bf.total);
  SNS_LAUNCH("csr_compact", k_csr_compact, dim3(p.nb), dim3(kCompactThreads), 0, st, A.m,
             A.row_ptr, bf.bcount, bf.list);
  ArgTable t(bf.args);
  const std::vector<SortArgs> sa{sort_args(p.sp, seed, nullptr, bf.sb, bf.list, bf.total)};
  const SortJob job = build_sort_job(t, sa, A.dtype == SNS_F64);
  sns_status s = t.bytes() > kCsrArgBytes ? SNS_ERR_OUT_OF_MEMORY : t.upload(st);
  if (s == SNS_OK) s = launch_sort_job(job, st);
  if (s == SNS_OK) {
    if (A.dtype == SNS_F64) launch_csr_t<double, double>(A, d, seed, b, SA, Sb, p, bf, st);
    else launch_csr_t<float, double>(A, d, seed, b, SA, Sb, p, bf, st);
  }
  region_end(st);
  if (s != SNS_OK) return s;
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace sns
