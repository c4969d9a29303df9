// Sketch and QR of many small problems in one persistent launch.
//
// For a problem whose sketched system [SA | Sb] (d x (n + 1), fp64) fits in
// LDS (d <= 256, n <= 64) the whole set-up of sketch-and-solve (Sec. 1.2
// steps 1-3: CountSketch of [A | b], Householder QR, x0 = R^{-1} c) runs in
// k_fused_sq.  Every problem of the batch is cut into row chunks; a fixed
// grid of work-groups (one per compute unit) claims chunks from one device
// queue, so uneven problems share the launch without a per-problem grid.
//
// A chunk is sketched in sub-blocks of 4096 rows: the rows are hashed and
// counting-sorted by bucket in LDS (per-wave histograms, a scan in
// bucket-major then wave order, a stable scatter ranked by ballot), then
// thread t accumulates the (bucket, column) outputs t, t + 512, ... in fp64
// registers over the rows of that bucket in ascending row order.  A chunk's
// partial goes to memory; chunks are summed in ascending order in two
// levels: the last chunk of each group of kFusedGroup to arrive adds the
// group, the last group to arrive adds the groups (a problem with one chunk
// skips both).  The work-group that completes a problem's sum holds
// [SA | Sb] in LDS and factors it there.  No floating-point atomics: every
// sum has a fixed order, so the result depends only on the problem and its
// seed, never on the batch or on which work-group ran what.
#include "common.hpp"
#include "kernels.hpp"
#include "linalg.hpp"

namespace sns {

namespace {

constexpr int kFusedThreads = 512;
constexpr int kFusedWaves = kFusedThreads / 64;
constexpr int kFusedSub = 4096;     // rows sorted in LDS at a time
constexpr int kFusedMaxD = 256;
constexpr int kFusedMaxCols = 65;   // n + 1
constexpr int kFusedU = (kFusedMaxD * kFusedMaxCols + kFusedThreads - 1) / kFusedThreads;
constexpr int kFusedGroup = 16;     // chunks summed by one group reducer
constexpr int kFusedMaxChunks = 128;

// LDS: the sort phase and the QR phase use the same bytes.
struct FusedSortLds {
  uint32_t hist[kFusedWaves][kFusedMaxD];
  uint32_t cur[kFusedWaves][kFusedMaxD];
  uint32_t bptr[kFusedMaxD + 1];
  uint32_t wsum[4];
  uint32_t perm[kFusedSub];
};
constexpr int kQrLd = kFusedMaxCols;  // odd row stride of M in LDS
constexpr size_t kFusedQrBytes =
    sizeof(double) * ((size_t)kFusedMaxD * kQrLd + 16 * kFusedMaxCols + kFusedMaxCols + 64);
constexpr size_t kFusedLds =
    sizeof(FusedSortLds) > kFusedQrBytes ? sizeof(FusedSortLds) : kFusedQrBytes;

template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every wave's stores of the hand-over values (st_agent) have completed
// before thread 0 counts the work-group in; true in every thread of the
// work-group that arrives last.
__device__ __forceinline__ bool arrive_last(unsigned* cnt, unsigned expect, int* flag) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) *flag = atomicAdd(cnt, 1u) == expect - 1u ? 1 : 0;
  __syncthreads();
  return *flag != 0;
}

// Sketch of rows [s0, s1) (at most kFusedSub) added into acc: acc[u] holds
// output e = t + kFusedThreads u, bucket e / ncol, column e % ncol (column n
// is b).
template <typename T>
__device__ __forceinline__ void sketch_sub(const FusedArgs& a, int64_t s0, int64_t s1,
                                           FusedSortLds& L, double (&acc)[kFusedU]) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint32_t d = (uint32_t)a.d;
  const int ncol = a.n + 1;
  const int len = (int)(s1 - s0);
  const int per = (((len + kFusedWaves - 1) / kFusedWaves) + 63) / 64 * 64;  // rows per wave
  const int w0 = w * per < len ? w * per : len, w1 = w0 + per < len ? w0 + per : len;
  for (uint32_t k = lane; k < d; k += 64) L.hist[w][k] = 0u;
  __builtin_amdgcn_wave_barrier();
  for (int r = w0 + lane; r < w1; r += 64) atomicAdd(&L.hist[w][cs_hash(a.seed, d, s0 + r).h], 1u);
  __syncthreads();
  // bucket starts: exclusive scan of the bucket totals (d <= 256: the first
  // four waves), then each wave's cursor inside its buckets
  uint32_t tot = 0, incl = 0;
  if (t < 256) {
    if ((uint32_t)t < d)
      for (int q = 0; q < kFusedWaves; ++q) tot += L.hist[q][t];
    incl = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(incl, off, 64);
      if (lane >= off) incl += y;
    }
    if (lane == 63) L.wsum[w] = incl;
  }
  __syncthreads();
  if ((uint32_t)t < d) {
    uint32_t run = incl - tot;
    for (int q = 0; q < (t >> 6); ++q) run += L.wsum[q];
    L.bptr[t] = run;
    for (int q = 0; q < kFusedWaves; ++q) {
      const uint32_t cq = L.hist[q][t];
      L.cur[q][t] = run;
      run += cq;
    }
  }
  if (t == 0) L.bptr[d] = (uint32_t)len;
  __syncthreads();
  // stable scatter: wave w's rows in ascending order, ranked inside each
  // batch of 64 by the lanes below with the same bucket
  const int nbits = d > 1 ? 32 - __clz((int)(d - 1)) : 0;
  for (int r0 = w0; r0 < w1; r0 += 64) {
    const int r = r0 + lane;
    const bool valid = r < w1;
    const Hash hs = cs_hash(a.seed, d, (uint64_t)(s0 + (valid ? r : w0)));
    const uint32_t h = valid ? hs.h : 0u;
    uint64_t peers = __ballot(valid);
    for (int bit = 0; bit < nbits; ++bit) {
      const bool on = (h >> bit) & 1u;
      const uint64_t bal = __ballot(on);
      peers &= on ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
    const bool last = lane == 63 || (peers >> (lane + 1)) == 0ull;
    if (valid) {
      const uint32_t pos = L.cur[w][h] + rank;
      L.perm[pos] = (uint32_t)r | (hs.neg ? 0x80000000u : 0u);
      if (last) L.cur[w][h] = pos + 1;
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // gather: output e sums its bucket's rows in ascending order, 8 loads in flight
  const T* __restrict__ A = static_cast<const T*>(a.A);
  const T* __restrict__ b = static_cast<const T*>(a.b);
  const int dn = (int)d * ncol;
#pragma unroll
  for (int u = 0; u < kFusedU; ++u) {
    const int e = t + kFusedThreads * u;
    if (e >= dn) break;
    const int k = e / ncol, j = e - k * ncol;
    const int p0 = (int)L.bptr[k], p1 = (int)L.bptr[k + 1];
    double s = acc[u];
    for (int p = p0; p < p1; p += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        v[q] = 0.0;
        if (p + q < p1) {
          const uint32_t pr = L.perm[p + q];
          const int64_t i = s0 + (int64_t)(pr & 0x7FFFFFFFu);
          const double x = j < a.n ? (double)A[i * a.ld + j] : (double)b[i];
          v[q] = (pr >> 31) ? -x : x;
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) s += v[q];
    }
    acc[u] = s;
  }
  __syncthreads();  // the LDS is reused by the next sub-block
}

// Householder QR (LAPACK convention, as the blocked QR) of [SA | Sb] held in
// LDS (M[i * kQrLd + c], d x ncol), then rho, rank and finiteness checks and
// x0 = R^{-1} c.  Thread (c, q) = (t % ncol, t / ncol) owns column c on the
// rows q, q + nq, ...; each column step takes the products of column k below
// its pivot with every later column (one work-group sum), then updates.
// Only R, c and rho leave the factorisation, so the reflectors are not kept:
// column k keeps x below the diagonal and gets beta on it.
__device__ __forceinline__ void lds_qr(const FusedArgs& a, double* sh) {
  const int t = threadIdx.x;
  const int d = a.d, n = a.n, ncol = n + 1;
  const int nq = kFusedThreads / ncol;
  const int c = t % ncol, q = t / ncol;
  const bool act = q < nq;
  double* M = sh;
  double* gp = M + (size_t)kFusedMaxD * kQrLd;  // [16][ncol] group partials
  double* piv = gp + 16 * kFusedMaxCols;        // [ncol] pivot row
  double* red = piv + kFusedMaxCols;            // [3]: rho, rank-deficient, non-finite
  bool bad = false;
  for (int k = 0; k < n; ++k) {
    // products of x = column k below the pivot with the columns c >= k
    double g = 0.0;
    if (act && c >= k)
      for (int i = k + 1 + q; i < d; i += nq) g = fma(M[i * kQrLd + k], M[i * kQrLd + c], g);
    // fold the nq row-group partials into 16 slots in a fixed order
    if (act) {
      if (q < 16) gp[q * kFusedMaxCols + c] = g;
    }
    if (t < ncol) piv[t] = M[k * kQrLd + t];
    __syncthreads();
    for (int qq = 16; qq < nq; qq += 16) {
      if (act && q >= qq && q < qq + 16) gp[(q - qq) * kFusedMaxCols + c] += g;
      __syncthreads();
    }
    auto total = [&](int col) {
      double s = 0.0;
      const int ns = nq < 16 ? nq : 16;
      for (int z = 0; z < ns; ++z) s += gp[z * kFusedMaxCols + col];
      return s;
    };
    const double alpha = piv[k];
    const double nu = sqrt(alpha * alpha + total(k));
    double beta = 0.0, tk = 0.0, scale = 0.0;
    if (nu != 0.0) {
      beta = alpha >= 0.0 ? -nu : nu;
      tk = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    if (!isfinite(nu)) bad = true;
    if (act && c > k) {
      const double wc = piv[c] + scale * total(c);
      // row k (v = 1) by its row group, rows below with v_i = scale x_i
      if (q == 0) M[k * kQrLd + c] = fma(-tk, wc, piv[c]);
      for (int i = k + 1 + q; i < d; i += nq)
        M[i * kQrLd + c] = fma(-tk * scale * M[i * kQrLd + k], wc, M[i * kQrLd + c]);
    }
    __syncthreads();  // every read of column k and of the pivot row is done
    if (t == 0) M[k * kQrLd + k] = beta;
    __syncthreads();
  }
  // rho = ||M[n:, n]||, rank and finiteness, on the first wave
  const int lane = t & 63;
  if (t < 64) {
    double s = 0.0;
    for (int i = n + lane; i < d; i += 64) s += M[i * kQrLd + n] * M[i * kQrLd + n];
    double mx = 0.0;
    bool nf = false;
    for (int i = lane; i < n; i += 64) {
      const double r = M[i * kQrLd + i];
      mx = fmax(mx, fabs(r));
      if (!isfinite(r)) nf = true;
    }
    s = wave_sum(s);
    mx = wave_max(mx);
    const double thr = 10.0 * (double)n * 1.1102230246251565e-16 * mx;
    bool small = false;
    for (int i = lane; i < n; i += 64)
      if (fabs(M[i * kQrLd + i]) <= thr) small = true;
    const bool rankdef = __ballot(small) != 0ull;
    const bool nonfin = __ballot(nf) != 0ull;
    if (lane == 0) {
      red[0] = sqrt(s);
      red[1] = rankdef ? 1.0 : 0.0;
      red[2] = nonfin ? 1.0 : 0.0;
    }
  }
  const bool anybad = __syncthreads_or(bad ? 1 : 0) != 0;  // also orders red[] for all
  const double rho = red[0];
  const bool nonfin = red[2] > 0.0 || anybad || !isfinite(rho);
  // R out (column-major for the refinement, ld n) and 1 / diag
  for (int e = t; e < n * n; e += kFusedThreads) {
    const int i = e % n, j = e / n;
    a.R[e] = i <= j ? M[i * kQrLd + j] : 0.0;
  }
  if (t < n) a.invd[t] = 1.0 / M[t * kQrLd + t];
  // x0 = R^{-1} c on the first wave (n <= 64): back substitution, lane i
  // keeps its running right-hand side
  if (t < 64) {
    double xi = lane < n ? M[lane * kQrLd + n] : 0.0;
    for (int j = n - 1; j >= 0; --j) {
      const double xj = readlane_f64(xi, j) / M[j * kQrLd + j];
      if (lane == j) xi = xj;
      else if (lane < j) xi = fma(-M[lane * kQrLd + j], xj, xi);
    }
    if (lane < n) a.x0[lane] = xi;
  }
  if (t == 0) {
    a.scal[0] = rho;
    a.scal[1] = red[1];
    a.scal[2] = nonfin ? 1.0 : 0.0;
    sns_info* info = a.info;
    info->status = nonfin ? SNS_ERR_NUMERICAL : (red[1] > 0.0 ? SNS_ERR_RANK_DEFICIENT : SNS_OK);
    info->iters = 0;
    info->rel_resid_est = 0.0;
    info->sketch_resid = rho;
  }
}

template <typename T>
__global__ __launch_bounds__(kFusedThreads) void k_fused_sq(FusedArgs* __restrict__ P, Map mp,
                                                            FusedCtl* __restrict__ ctl) {
  __shared__ __attribute__((aligned(16))) unsigned char lds_raw[kFusedLds];
  __shared__ unsigned s_item;
  __shared__ int s_flag;
  FusedSortLds& L = *reinterpret_cast<FusedSortLds*>(lds_raw);
  double* sh = reinterpret_cast<double*>(lds_raw);
  const int t = threadIdx.x;
  const unsigned total = mp.off[mp.nprob];
  for (;;) {
    if (t == 0) s_item = atomicAdd(&ctl->head, 1u);
    __syncthreads();
    const unsigned item = s_item;
    __syncthreads();
    if (item >= total) break;
    const int pi = map_find(mp, item);
    FusedArgs& a = P[pi];
    const int chunk = (int)(item - mp.off[pi]);
    const int ncol = a.n + 1, dn = a.d * ncol;
    double acc[kFusedU];
#pragma unroll
    for (int u = 0; u < kFusedU; ++u) acc[u] = 0.0;
    const int64_t r0 = (int64_t)chunk * a.rc;
    const int64_t r1 = r0 + a.rc < a.m ? r0 + a.rc : a.m;
    for (int64_t s0 = r0; s0 < r1; s0 += kFusedSub)
      sketch_sub<T>(a, s0, s0 + kFusedSub < r1 ? s0 + kFusedSub : r1, L, acc);
    if (a.nchunk > 1) {
      // chunk partial, then the group sum by the group's last chunk
      double* part = a.part + (size_t)chunk * dn;
#pragma unroll
      for (int u = 0; u < kFusedU; ++u) {
        const int e = t + kFusedThreads * u;
        if (e < dn) st_agent(&part[e], acc[u]);
      }
      const int grp = chunk / kFusedGroup;
      const int c0 = grp * kFusedGroup;
      const int c1 = c0 + kFusedGroup < a.nchunk ? c0 + kFusedGroup : a.nchunk;
      if (!arrive_last(&a.cnt[1 + grp], (unsigned)(c1 - c0), &s_flag)) continue;
#pragma unroll
      for (int u = 0; u < kFusedU; ++u) {
        const int e = t + kFusedThreads * u;
        double s = 0.0;
        if (e < dn)
          for (int cc = c0; cc < c1; ++cc) s += ld_agent(&a.part[(size_t)cc * dn + e]);
        acc[u] = s;
      }
      if (t == 0) a.cnt[1 + grp] = 0u;
      if (a.ngroup > 1) {
#pragma unroll
        for (int u = 0; u < kFusedU; ++u) {
          const int e = t + kFusedThreads * u;
          if (e < dn) st_agent(&a.gpart[(size_t)grp * dn + e], acc[u]);
        }
        if (!arrive_last(&a.cnt[0], (unsigned)a.ngroup, &s_flag)) continue;
#pragma unroll
        for (int u = 0; u < kFusedU; ++u) {
          const int e = t + kFusedThreads * u;
          double s = 0.0;
          if (e < dn)
            for (int g = 0; g < a.ngroup; ++g) s += ld_agent(&a.gpart[(size_t)g * dn + e]);
          acc[u] = s;
        }
        if (t == 0) a.cnt[0] = 0u;
      }
    }
    // this work-group holds the problem's whole [SA | Sb]
#pragma unroll
    for (int u = 0; u < kFusedU; ++u) {
      const int e = t + kFusedThreads * u;
      if (e < dn) sh[(e / ncol) * kQrLd + e % ncol] = acc[u];
    }
    __syncthreads();
    lds_qr(a, sh);
    __syncthreads();  // the LDS is reused by the next item
  }
}

// Copies a batch's argument table from pinned host memory into its device
// table (the replayed graph's first node; its counters arrive zeroed).
__global__ void k_fused_stage(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst,
                              const uint64_t* __restrict__ words) {
  const uint64_t nw = *words;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nw;
       i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

int fused_grid() {
  static int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      n = 256;
    return n > 0 ? n : 256;
  }();
  return cus;
}

}  // namespace

bool fused_eligible(const sns_sketch& sk, const sns_matrix& A) {
  return sk.kind == SNS_SKETCH_COUNT && A.layout == SNS_DENSE_ROWMAJOR && sk.d <= kFusedMaxD &&
         A.n + 1 <= kFusedMaxCols && A.m <= kMaxFusedRows;
}

FusedPlan make_fused_plan(const sns_sketch& sk, const sns_matrix& A) {
  FusedPlan p;
  // sub-blocks per chunk: as few as keep the chunk count within the limit
  const int64_t subs = (A.m + kFusedSub - 1) / kFusedSub;
  const int64_t spc = (subs + kFusedMaxChunks - 1) / kFusedMaxChunks;
  p.rc = spc * kFusedSub;
  p.nchunk = (int)((A.m + p.rc - 1) / p.rc);
  p.ngroup = (p.nchunk + kFusedGroup - 1) / kFusedGroup;
  p.dn = sk.d * (A.n + 1);
  return p;
}

void carve_fused(Carve& c, const FusedPlan& p, double*& part, double*& gpart) {
  part = p.nchunk > 1 ? c.take<double>((size_t)p.nchunk * p.dn) : nullptr;
  gpart = p.ngroup > 1 ? c.take<double>((size_t)p.ngroup * p.dn) : nullptr;
}

FusedArgs fused_args(const FusedPlan& p, const sns_sketch& sk, const sns_matrix& A, const void* b,
                     double* part, double* gpart, const QrBufs& q, double* x0, sns_info* info) {
  FusedArgs a{};
  a.A = A.values;
  a.b = b;
  a.ld = A.ld;
  a.m = A.m;
  a.n = (int)A.n;
  a.d = (int)sk.d;
  a.seed = sk.seed;
  a.rc = p.rc;
  a.nchunk = p.nchunk;
  a.ngroup = p.ngroup;
  a.part = part;
  a.gpart = gpart;
  a.R = q.R;
  a.invd = q.invd;
  a.x0 = x0;
  a.scal = q.scal;
  a.info = info;
  return a;
}

FusedJob build_fused_job(ArgTable& t, const std::vector<FusedArgs>& a, bool f64) {
  FusedJob j;
  j.f64 = f64;
  j.count = (int)a.size();
  if (a.empty()) return j;
  std::vector<uint32_t> cnt;
  for (const FusedArgs& x : a) cnt.push_back((uint32_t)x.nchunk);
  j.ctl = t.add(std::vector<FusedCtl>(1).data(), 1);
  j.args = t.add(a.data(), a.size());
  j.map = t.map(cnt, &j.items);
  return j;
}

sns_status launch_fused_job(const FusedJob& j, hipStream_t st) {
  if (j.count == 0) return SNS_OK;
  const int grid = (int)(j.items < (uint32_t)fused_grid() ? j.items : (uint32_t)fused_grid());
  region_begin("fused", st);
  if (j.f64)
    SNS_LAUNCH("fused_sq", k_fused_sq<double>, dim3(grid), dim3(kFusedThreads), 0, st,
               const_cast<FusedArgs*>(j.args), j.map, const_cast<FusedCtl*>(j.ctl));
  else
    SNS_LAUNCH("fused_sq", k_fused_sq<float>, dim3(grid), dim3(kFusedThreads), 0, st,
               const_cast<FusedArgs*>(j.args), j.map, const_cast<FusedCtl*>(j.ctl));
  region_end(st);
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

sns_status launch_fused_stage(const void* host_src, void* dev_dst, const uint64_t* host_words,
                              hipStream_t st) {
  SNS_LAUNCH("fused_stage", k_fused_stage, dim3(8), dim3(256), 0, st,
             static_cast<const uint64_t*>(host_src), static_cast<uint64_t*>(dev_dst), host_words);
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

size_t fused_lds_bytes() { return kFusedLds; }

}  // namespace sns
