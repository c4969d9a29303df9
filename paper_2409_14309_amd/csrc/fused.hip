// Sketch and QR of many small problems in one persistent launch.
//
// For a problem whose sketched system [SA | Sb] (d x (n + 1), fp64) fits in
// LDS (d <= 256, n <= 64) and whose data is small (m (n + 1) <= 2^21), the
// whole set-up of sketch-and-solve (Sec. 1.2
// steps 1-3: CountSketch of [A | b], Householder QR, x0 = R^{-1} c) runs in
// k_fused_sq.  Every problem of the batch is cut into row chunks; a fixed
// grid of work-groups (one per compute unit) claims chunks from one device
// queue, so uneven problems share the launch without a per-problem grid.
//
// A chunk is sketched in sub-blocks of 4096 rows: the rows are hashed and
// counting-sorted by bucket in LDS (per-wave histograms, a scan in
// bucket-major then wave order, a stable scatter ranked by ballot), then
// thread t accumulates the (bucket, four-column quad) outputs t, t + 512, ...
// in fp64 registers over the rows of that bucket in ascending row order, the
// quad's four entries of a row in one vector load.  A chunk's
// partial goes to memory; chunks are summed in ascending order in two
// levels: the last chunk of each group of kFusedGroup to arrive adds the
// group, the last group to arrive adds the groups (a problem with one chunk
// skips both).  The work-group that completes a problem's sum holds
// [SA | Sb] in LDS and factors it there.  No floating-point atomics: every
// sum has a fixed order, so the result depends only on the problem and its
// seed, never on the batch or on which work-group ran what.
#include <string.h>

#include <atomic>

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
constexpr int kFusedQuads = (kFusedMaxCols + 3) / 4;  // column quads of [A | b]
constexpr int kFusedU = (kFusedMaxD * kFusedQuads + kFusedThreads - 1) / kFusedThreads;
constexpr int kFusedGroup = 16;     // chunks summed by one group reducer
constexpr int kGV = 2;              // quads a thread gathers together
constexpr int kFusedMaxChunks = 128;

// LDS: the sort phase and the QR phase use the same bytes.
struct FusedSortLds {
  uint32_t hist[kFusedWaves][kFusedMaxD];
  uint32_t cur[kFusedWaves][kFusedMaxD];
  uint32_t bptr[kFusedMaxD + 1];
  uint32_t wsum[4];
  uint32_t perm[kFusedSub];
};
// LDS of the QR: x and the pivot row (double-buffered), row-group partials,
// flags, and R with c for the triangular solve
constexpr size_t kFusedQrBytes =
    sizeof(double) * (2 * (kFusedMaxD + 1) + 2 * kFusedMaxCols + 16 * kFusedMaxCols + 4 +
                      (kFusedMaxCols - 1) * kFusedMaxCols);
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

// Sketch of rows [s0, s1) (at most kFusedSub) added into acc: acc[u][i]
// holds column 4 jq + i of bucket k for the quad e = t + kFusedThreads u =
// k ncq + jq (ncq = ceil((n + 1) / 4); column n is b).
template <typename T>
__device__ __forceinline__ void sketch_sub(const FusedArgs& a, int64_t s0, int64_t s1,
                                           FusedSortLds& L, double (&acc)[kFusedU][4]) {
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
  // gather: each quad of outputs sums its bucket's rows in ascending row
  // order; a row's four entries come in one vector load where A allows it,
  // and two quads advance together, eight rows each (four in fp64)
  const T* __restrict__ A = static_cast<const T*>(a.A);
  const T* __restrict__ b = static_cast<const T*>(a.b);
  constexpr int kGR = sizeof(T) == 4 ? 8 : 4;  // rows of each quad in flight
  const int ncq = (ncol + 3) / 4, dq = (int)d * ncq;
#pragma unroll
  for (int ug = 0; ug < kFusedU; ug += kGV) {
    if (t + kFusedThreads * ug >= dq) break;
    int p0[kGV], p1[kGV], c0[kGV];
    int len = 0;
#pragma unroll
    for (int v = 0; v < kGV; ++v) {
      const int e = t + kFusedThreads * (ug + v);
      p0[v] = p1[v] = 0;
      c0[v] = 0;
      if (ug + v < kFusedU && e < dq) {
        const int k = e / ncq;
        c0[v] = 4 * (e - k * ncq);
        p0[v] = (int)L.bptr[k];
        p1[v] = (int)L.bptr[k + 1];
      }
      len = max(len, p1[v] - p0[v]);
    }
    for (int r = 0; r < len; r += kGR) {
      T x[kGV][kGR][4];  // signed entries, exact in A's type
#pragma unroll
      for (int v = 0; v < kGV; ++v)
#pragma unroll
        for (int q = 0; q < kGR; ++q) {
#pragma unroll
          for (int c = 0; c < 4; ++c) x[v][q][c] = T(0);
          const int p = p0[v] + r + q;
          if (p < p1[v]) {
            const uint32_t pr = L.perm[p];
            const int64_t i = s0 + (int64_t)(pr & 0x7FFFFFFFu);
            const T* row = A + i * a.ld;
            const int cb = c0[v];
            if (a.vec && cb + 4 <= a.n) {
              if constexpr (sizeof(T) == 4) {
                const float4 f = *reinterpret_cast<const float4*>(row + cb);
                x[v][q][0] = f.x; x[v][q][1] = f.y; x[v][q][2] = f.z; x[v][q][3] = f.w;
              } else {
                const double2 f0 = *reinterpret_cast<const double2*>(row + cb);
                const double2 f1 = *reinterpret_cast<const double2*>(row + cb + 2);
                x[v][q][0] = f0.x; x[v][q][1] = f0.y; x[v][q][2] = f1.x; x[v][q][3] = f1.y;
              }
            } else {
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                const int col = cb + c;
                x[v][q][c] = col < a.n ? row[col] : (col == a.n ? b[i] : T(0));
              }
            }
            if (pr >> 31)
#pragma unroll
              for (int c = 0; c < 4; ++c) x[v][q][c] = -x[v][q][c];
          }
        }
#pragma unroll
      for (int v = 0; v < kGV; ++v)
        if (ug + v < kFusedU) {
#pragma unroll
          for (int q = 0; q < kGR; ++q)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[ug + v][c] += (double)x[v][q][c];
        }
    }
  }
  __syncthreads();  // the LDS is reused by the next sub-block
}

// Householder QR (LAPACK convention, as the blocked QR) of [SA | Sb], then
// rho, rank and finiteness checks and x0 = R^{-1} c.  On entry a.msys
// (row-major d x ncol) holds the system; thread (c, q) = (t % ncol,
// t / ncol) takes column c on the rows q, q + nq, ... into registers, so the
// factorisation reads LDS only for the column being eliminated: each step
// publishes x = column k below its pivot and the pivot row, takes the
// products of x with every later column (one work-group sum over the row
// groups, in a fixed order), and updates.  Only R, c and rho leave the
// factorisation, so the reflectors are not kept.
// Rows per thread for the widest system of each column class (ncol <= 17,
// 33, 65): the row loops are unrolled to exactly that many rows, and rows past
// d read the zero entry x[d] (their registers hold zeros), so no iteration is
// predicated.
template <int RM>
__device__ __forceinline__ void lds_qr_t(const FusedArgs& a, double* sh) {
  const int t = threadIdx.x;
  const int d = a.d, n = a.n, ncol = n + 1;
  const int nq = kFusedThreads / ncol;
  const int c = t % ncol, q = t / ncol;
  const bool act = q < nq;
  double Mr[RM];
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    const int i = q + nq * r;
    Mr[r] = (act && i < d) ? a.msys[i * ncol + c] : 0.0;
  }
  double* xs = sh;                              // [2][kFusedMaxD + 1] column k below its pivot; x[d] = 0
  double* pv = xs + 2 * (kFusedMaxD + 1);       // [2][kFusedMaxCols] pivot rows
  double* gp = pv + 2 * kFusedMaxCols;          // [16][kFusedMaxCols] row-group partials
  double* red = gp + 16 * kFusedMaxCols;        // [4]: rho, rank-deficient, non-finite
  double* Rl = red + 4;                         // [n][n + 1]: R and c for x0
  if (t < 2) xs[t * (kFusedMaxD + 1) + d] = 0.0;  // the pad row, read by rows past d
  bool bad = false;
  for (int k = 0; k < n; ++k) {
    double* x = xs + (k & 1) * (kFusedMaxD + 1);
    double* piv = pv + (k & 1) * kFusedMaxCols;
    const int qk = k % nq, rk = k / nq;  // owner of row k
    if (act && c == k)
#pragma unroll
      for (int r = 0; r < RM; ++r) {
        const int i = q + nq * r;
        if (i < d) x[i] = i > k ? Mr[r] : 0.0;
      }
    if (act && q == qk)
#pragma unroll
      for (int r = 0; r < RM; ++r)
        if (r == rk) piv[c] = Mr[r];
    __syncthreads();
    // products of x with the columns c >= k, folded into 16 row-group slots
    double g = 0.0;
    if (act && c >= k)
#pragma unroll
      for (int r = 0; r < RM; ++r) g = fma(x[min(q + nq * r, d)], Mr[r], g);
    if (act && q < 16) gp[q * kFusedMaxCols + c] = g;
    __syncthreads();
    for (int qq = 16; qq < nq; qq += 16) {
      if (act && q >= qq && q < qq + 16) gp[(q - qq) * kFusedMaxCols + c] += g;
      __syncthreads();
    }
    const int ns = nq < 16 ? nq : 16;
    auto total = [&](int col) {
      double sum = 0.0;
      for (int z = 0; z < ns; ++z) sum += gp[z * kFusedMaxCols + col];
      return sum;
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
      // w_c = v . M[:, c] with v_k = 1, v_i = scale x_i below; M -= tau v w_c
      const double wc = piv[c] + scale * total(c);
      const double f = tk * scale * wc;
#pragma unroll
      for (int r = 0; r < RM; ++r) Mr[r] = fma(-f, x[min(q + nq * r, d)], Mr[r]);
      if (q == qk)
#pragma unroll
        for (int r = 0; r < RM; ++r)
          if (r == rk) Mr[r] = fma(-tk, wc, piv[c]);
    }
    if (act && c == k && q == qk)
#pragma unroll
      for (int r = 0; r < RM; ++r)
        if (r == rk) Mr[r] = beta;
    __syncthreads();  // gp, x and piv of this step are read
  }
  // R (upper triangle) and c to LDS for x0; R out (column-major, ld n)
  if (act)
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      const int i = q + nq * r;
      if (i < n && i <= c) Rl[i * ncol + c] = Mr[r];
    }
  // rho = ||M[n:, n]|| from the last column's threads
  double sq = 0.0;
  if (act && c == n)
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      const int i = q + nq * r;
      if (i >= n && i < d) sq += Mr[r] * Mr[r];
    }
  if (act && q < 16) gp[q * kFusedMaxCols + c] = c == n ? sq : 0.0;
  __syncthreads();
  for (int qq = 16; qq < nq; qq += 16) {
    if (act && c == n && q >= qq && q < qq + 16) gp[(q - qq) * kFusedMaxCols + c] += sq;
    __syncthreads();
  }
  for (int e = t; e < n * n; e += kFusedThreads) {
    const int i = e % n, j = e / n;
    a.R[e] = i <= j ? Rl[i * ncol + j] : 0.0;
  }
  if (t < n) a.invd[t] = 1.0 / Rl[t * ncol + t];
  const int lane = t & 63;
  if (t < 64) {
    double s2 = 0.0;
    const int ns = nq < 16 ? nq : 16;
    for (int z = 0; z < ns; ++z) s2 += gp[z * kFusedMaxCols + n];
    double mx = 0.0;
    bool nf = false;
    for (int i = lane; i < n; i += 64) {
      const double r = Rl[i * ncol + i];
      mx = fmax(mx, fabs(r));
      if (!isfinite(r)) nf = true;
    }
    mx = wave_max(mx);
    const double thr = 10.0 * (double)n * 1.1102230246251565e-16 * mx;
    bool small = false;
    for (int i = lane; i < n; i += 64)
      if (fabs(Rl[i * ncol + i]) <= thr) small = true;
    const bool rankdef = __ballot(small) != 0ull;
    const bool nonfin = __ballot(nf) != 0ull;
    // x0 = R^{-1} c (n <= 64): back substitution, lane i keeps its running
    // right-hand side
    double xi = lane < n ? Rl[lane * ncol + n] : 0.0;
    for (int j2 = n - 1; j2 >= 0; --j2) {
      const double xj = readlane_f64(xi, j2) / Rl[j2 * ncol + j2];
      if (lane == j2) xi = xj;
      else if (lane < j2) xi = fma(-Rl[lane * ncol + j2], xj, xi);
    }
    if (lane < n) a.x0[lane] = xi;
    if (lane == 0) {
      red[0] = sqrt(s2);
      red[1] = rankdef ? 1.0 : 0.0;
      red[2] = nonfin ? 1.0 : 0.0;
    }
  }
  const bool anybad = __syncthreads_or(bad ? 1 : 0) != 0;  // also orders red[] for all
  const double rho = red[0];
  const bool nonfin = red[2] > 0.0 || anybad || !isfinite(rho);
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


// The QR of the problem's system, unrolled for its column class.
__device__ __forceinline__ void lds_qr(const FusedArgs& a, double* sh) {
  const int ncol = a.n + 1;
  if (ncol <= 17) lds_qr_t<(kFusedMaxD + kFusedThreads / 17 - 1) / (kFusedThreads / 17)>(a, sh);
  else if (ncol <= 33) lds_qr_t<(kFusedMaxD + kFusedThreads / 33 - 1) / (kFusedThreads / 33)>(a, sh);
  else lds_qr_t<(kFusedMaxD + kFusedThreads / kFusedMaxCols - 1) / (kFusedThreads / kFusedMaxCols)>(a, sh);
}

// The problem count is read from the control block, so a captured launch
// serves any batch up to the table's capacity.
template <typename T>
__global__ __launch_bounds__(kFusedThreads) void k_fused_sq(FusedArgs* __restrict__ P,
                                                            const uint32_t* __restrict__ off,
                                                            FusedCtl* __restrict__ ctl) {
  __shared__ __attribute__((aligned(16))) unsigned char lds_raw[kFusedLds];
  __shared__ unsigned s_item;
  __shared__ int s_flag;
  FusedSortLds& L = *reinterpret_cast<FusedSortLds*>(lds_raw);
  double* sh = reinterpret_cast<double*>(lds_raw);
  const int t = threadIdx.x;
  const Map mp{off, ctl->nprob};
  const unsigned total = mp.nprob > 0 ? mp.off[mp.nprob] : 0u;
  for (;;) {
    if (t == 0) s_item = atomicAdd(&ctl->head, 1u);
    __syncthreads();
    const unsigned item = s_item;
    __syncthreads();
    if (item >= total) break;
    const int pi = map_find(mp, item);
    FusedArgs& a = P[pi];
    const int chunk = (int)(item - mp.off[pi]);
    const int ncol = a.n + 1, dn = a.d * ncol, ncq = (ncol + 3) / 4, dq = a.d * ncq;
    double acc[kFusedU][4];
#pragma unroll
    for (int u = 0; u < kFusedU; ++u)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[u][c] = 0.0;
    // element (bucket, column) of quad slot (u, c), or -1
    auto elem = [&](int u, int c) {
      const int e = t + kFusedThreads * u;
      if (e >= dq) return -1;
      const int k = e / ncq, col = 4 * (e - k * ncq) + c;
      return col < ncol ? k * ncol + col : -1;
    };
    const int64_t r0 = (int64_t)chunk * a.rc;
    const int64_t r1 = r0 + a.rc < a.m ? r0 + a.rc : a.m;
    for (int64_t s0 = r0; s0 < r1; s0 += kFusedSub)
      sketch_sub<T>(a, s0, s0 + kFusedSub < r1 ? s0 + kFusedSub : r1, L, acc);
    if (a.nchunk > 1) {
      // chunk partial, then the group sum by the group's last chunk
      double* part = a.part + (size_t)chunk * dn;
#pragma unroll
      for (int u = 0; u < kFusedU; ++u)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int e = elem(u, c);
          if (e >= 0) st_agent(&part[e], acc[u][c]);
        }
      const int grp = chunk / kFusedGroup;
      const int c0 = grp * kFusedGroup;
      const int c1 = c0 + kFusedGroup < a.nchunk ? c0 + kFusedGroup : a.nchunk;
      if (!arrive_last(&a.cnt[1 + grp], (unsigned)(c1 - c0), &s_flag)) continue;
      // the group's partials in ascending chunk order; each step loads all
      // of this thread's entries of one chunk before adding them
#pragma unroll
      for (int u = 0; u < kFusedU; ++u)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[u][c] = 0.0;
      for (int cc = c0; cc < c1; ++cc) {
        const double* pc = a.part + (size_t)cc * dn;
        double v[kFusedU][4];
#pragma unroll
        for (int u = 0; u < kFusedU; ++u)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int e = elem(u, c);
            v[u][c] = e >= 0 ? ld_agent(&pc[e]) : 0.0;
          }
#pragma unroll
        for (int u = 0; u < kFusedU; ++u)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[u][c] += v[u][c];
      }
      if (t == 0) a.cnt[1 + grp] = 0u;
      if (a.ngroup > 1) {
#pragma unroll
        for (int u = 0; u < kFusedU; ++u)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int e = elem(u, c);
            if (e >= 0) st_agent(&a.gpart[(size_t)grp * dn + e], acc[u][c]);
          }
        if (!arrive_last(&a.cnt[0], (unsigned)a.ngroup, &s_flag)) continue;
#pragma unroll
        for (int u = 0; u < kFusedU; ++u)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[u][c] = 0.0;
        for (int g = 0; g < a.ngroup; ++g) {
          const double* pg = a.gpart + (size_t)g * dn;
          double v[kFusedU][4];
#pragma unroll
          for (int u = 0; u < kFusedU; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const int e = elem(u, c);
              v[u][c] = e >= 0 ? ld_agent(&pg[e]) : 0.0;
            }
#pragma unroll
          for (int u = 0; u < kFusedU; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[u][c] += v[u][c];
        }
        if (t == 0) a.cnt[0] = 0u;
      }
    }
    // this work-group holds the problem's whole [SA | Sb]; it passes through
    // memory (read back by the same work-group) into the QR's layout
#pragma unroll
    for (int u = 0; u < kFusedU; ++u)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int e = elem(u, c);
        if (e >= 0) a.msys[e] = acc[u][c];
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

namespace {
std::atomic<bool> g_fused_on{false};
}  // namespace

// Small systems whose data is small too: one work-group sketches a chunk at
// a few tens of GB/s, so larger matrices stream faster through the blocked
// path's many work-groups per problem.
bool fused_eligible(const sns_sketch& sk, const sns_matrix& A) {
  return g_fused_on.load(std::memory_order_relaxed) && sk.kind == SNS_SKETCH_COUNT &&
         A.layout == SNS_DENSE_ROWMAJOR && sk.d <= kFusedMaxD && A.n + 1 <= kFusedMaxCols &&
         A.m * (A.n + 1) <= kMaxFusedElems;
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

void carve_fused(Carve& c, const FusedPlan& p, FusedBufs& f) {
  f.part = p.nchunk > 1 ? c.take<double>((size_t)p.nchunk * p.dn) : nullptr;
  f.gpart = p.ngroup > 1 ? c.take<double>((size_t)p.ngroup * p.dn) : nullptr;
  f.msys = c.take<double>((size_t)p.dn);
}

FusedArgs fused_args(const FusedPlan& p, const sns_sketch& sk, const sns_matrix& A, const void* b,
                     const FusedBufs& f, const QrBufs& q, double* x0, sns_info* info) {
  FusedArgs a{};
  a.A = A.values;
  a.b = b;
  a.ld = A.ld;
  a.m = A.m;
  a.n = (int)A.n;
  a.d = (int)sk.d;
  a.seed = sk.seed;
  a.vec = ((uintptr_t)A.values % 16 == 0 && (A.ld * (A.dtype == SNS_F64 ? 8 : 4)) % 16 == 0) ? 1 : 0;
  a.rc = p.rc;
  a.nchunk = p.nchunk;
  a.ngroup = p.ngroup;
  a.part = f.part;
  a.gpart = f.gpart;
  a.msys = f.msys;
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
  FusedCtl c{};
  c.nprob = (int)a.size();
  j.ctl = t.add(&c, 1);
  j.args = t.add(a.data(), a.size());
  j.map = t.map(cnt, &j.items);
  return j;
}

FusedTableLayout fused_table_layout(int max_probs) {
  FusedTableLayout L;
  L.max_probs = max_probs;
  size_t o = align_up(sizeof(FusedCtl), 16);
  L.args_off = o;
  o = align_up(o + sizeof(FusedArgs) * (size_t)max_probs, 16);
  L.off_off = o;
  o = align_up(o + sizeof(uint32_t) * ((size_t)max_probs + 1), 16);
  L.bytes = o;
  return L;
}

bool fused_table_fill(void* img, const FusedTableLayout& L, const std::vector<FusedArgs>& a,
                      uint64_t* words) {
  if ((int)a.size() > L.max_probs) return false;
  char* base = static_cast<char*>(img);
  FusedCtl c{};
  c.nprob = (int)a.size();
  memcpy(base, &c, sizeof(c));
  if (!a.empty()) memcpy(base + L.args_off, a.data(), sizeof(FusedArgs) * a.size());
  uint32_t* off = reinterpret_cast<uint32_t*>(base + L.off_off);
  off[0] = 0u;
  for (size_t i = 0; i < a.size(); ++i) off[i + 1] = off[i] + (uint32_t)a[i].nchunk;
  *words = L.bytes / 8;
  return true;
}

sns_status fused_graph_create(void* dev_tab, const FusedTableLayout& L, const void* host_img,
                              const uint64_t* host_words, bool f64, hipStream_t st,
                              hipGraphExec_t* exec) {
  char* base = static_cast<char*>(dev_tab);
  FusedCtl* ctl = reinterpret_cast<FusedCtl*>(base);
  FusedArgs* args = reinterpret_cast<FusedArgs*>(base + L.args_off);
  const uint32_t* off = reinterpret_cast<const uint32_t*>(base + L.off_off);
  hipGraph_t g = nullptr;
  SNS_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  hipLaunchKernelGGL(k_fused_stage, dim3(8), dim3(256), 0, st,
                     static_cast<const uint64_t*>(host_img), reinterpret_cast<uint64_t*>(base),
                     host_words);
  if (f64)
    hipLaunchKernelGGL(k_fused_sq<double>, dim3(fused_grid()), dim3(kFusedThreads), 0, st, args,
                       off, ctl);
  else
    hipLaunchKernelGGL(k_fused_sq<float>, dim3(fused_grid()), dim3(kFusedThreads), 0, st, args,
                       off, ctl);
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipStreamEndCapture(st, &g);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return SNS_ERR_HIP;
  }
  const hipError_t e3 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e3 == hipSuccess ? SNS_OK : SNS_ERR_HIP;
}

sns_status launch_fused_job(const FusedJob& j, hipStream_t st) {
  if (j.count == 0) return SNS_OK;
  const int grid = (int)(j.items < (uint32_t)fused_grid() ? j.items : (uint32_t)fused_grid());
  region_begin("fused", st);
  if (j.f64)
    SNS_LAUNCH("fused_sq", k_fused_sq<double>, dim3(grid), dim3(kFusedThreads), 0, st,
               const_cast<FusedArgs*>(j.args), j.map.off, const_cast<FusedCtl*>(j.ctl));
  else
    SNS_LAUNCH("fused_sq", k_fused_sq<float>, dim3(grid), dim3(kFusedThreads), 0, st,
               const_cast<FusedArgs*>(j.args), j.map.off, const_cast<FusedCtl*>(j.ctl));
  region_end(st);
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

size_t fused_lds_bytes() { return kFusedLds; }

}  // namespace sns

extern "C" void sns_fused_enable(int on) { sns::g_fused_on.store(on != 0); }
extern "C" int sns_fused_enabled(void) { return sns::g_fused_on.load() ? 1 : 0; }
