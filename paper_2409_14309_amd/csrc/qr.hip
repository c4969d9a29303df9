// Householder QR of the augmented sketch [SA | Sb] (d x (n+1)) in fp64 and
// the triangular solve R x0 = c, c = (Q^T Sb)[:n]: step 3 of sketch-and-solve.
//
// Layout: the working copy M is column-major with leading dimension d.
// Blocked right-looking algorithm: for each panel of nb columns,
//   k_qr_panel    one work-group (256 or 512 threads) holds the panel rows in
//                 registers and factors it column by column.  Each column
//                 needs one work-group reduction, which yields the norm, the
//                 products of the column with the remaining panel columns
//                 (for the rank-1 update) and with the earlier Householder
//                 vectors (for the compact-WY factor T).
//   k_qr_trailing applies (I - V T V^T)^T to the trailing columns, Sb
//                 included; a work-group keeps V in registers and takes
//                 groups of one (or two) columns in turn.
// then k_qr_extract copies R out (tiled transposes) and k_qr_finish checks
// rank and finiteness and solves R x0 = c on one work-group.
// Reflector convention (LAPACK): beta = -sign(alpha) ||x|| (sign(0) = +1),
// tau = (beta - alpha) / beta, v = x / (alpha - beta) with v[0] = 1.
#include <atomic>

#include "common.hpp"
#include "kernels.hpp"
#include "linalg.hpp"

namespace sns {

namespace {


// M[j * d + i] = SA[i * ld + j] (j < n), M[n * d + i] = Sb[i], via 32x32 tiles
// (a work item is one tile).  The first tile also clears the scalar flags.
template <typename T>
__global__ void k_qr_load(const QrArgs* __restrict__ P, Map mp) {
  __shared__ double tile[32][33];
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const int pi = map_find(mp, it);
  const QrArgs& a = P[pi];
  const uint32_t loc = it - mp.off[pi];
  const int64_t d = a.d, n = a.n, ld = a.ld_sa;
  const T* __restrict__ SA = static_cast<const T*>(a.SA);
  const T* __restrict__ Sb = static_cast<const T*>(a.Sb);
  const uint32_t tiles_i = (uint32_t)((d + 31) / 32);
  const int64_t i0 = (int64_t)(loc % tiles_i) * 32, j0 = (int64_t)(loc / tiles_i) * 32;
  if (loc == 0 && ty == 0 && tx < 8) a.scal[tx] = 0.0;
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + r, j = j0 + tx;
    double v = 0.0;
    if (i < d && j < n) v = (double)SA[i * ld + j];
    else if (i < d && j == n) v = (double)Sb[i];
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int c = ty; c < 32; c += 8) {
    const int64_t j = j0 + c, i = i0 + tx;
    if (i < d && j <= n) a.M[j * d + i] = tile[tx][c];
  }
}

// One Householder step of the panel, column K (a compile-time index so the
// register array P is never indexed at run time).
template <int MAXR, int NB, int NT, int K>
__device__ __forceinline__ void panel_step(double (&P)[MAXR][NB], int t, int64_t j0,
                                           double* red, double* tot, double* piv, double* Ts,
                                           double* __restrict__ tau, double* __restrict__ flags) {
  const int64_t jk = j0 + K;  // pivot row, owned by thread K (r = 0)
  // the pivot row alternates between two LDS buffers: step K + 1 may write
  // its row while a slower wave still reads this one (no barrier ends a step)
  piv += (K & 1) * NB;
  // partial sums over the rows below the pivot, x = column K there:
  // G_c = x . M[:, c] (c >= K) and Y_a = x . V[:, a] (a < K).  Rows at or
  // above the pivot contribute x = 0; rows past d hold zeros.
  double g[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) g[c] = 0.0;
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    const int64_t i = j0 + t + (int64_t)NT * r;
    const double x = i > jk ? P[r][K] : 0.0;
#pragma unroll
    for (int c = 0; c < NB; ++c) g[c] = fma(x, P[r][c], g[c]);
  }
  if (t == K) {
#pragma unroll
    for (int c = 0; c < NB; ++c) piv[c] = P[0][c];
  }
  block_reduce_multi<NB, NT>(g, red, tot);  // its barriers also publish piv
  const double alpha = piv[K];
  const double nu = sqrt(alpha * alpha + tot[K]);
  double beta = 0.0, tk = 0.0, scale = 0.0;
  if (nu != 0.0) {
    beta = alpha >= 0.0 ? -nu : nu;
    tk = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  // apply H_K = I - tau v v^T to the columns right of K:
  // w_c = v . M[:, c] = piv[c] + scale G_c, M[i, c] -= tau v_i w_c with
  // v_i = scale x_i below the pivot, 1 at the pivot, 0 above
  double w[NB];
#pragma unroll
  for (int c = K + 1; c < NB; ++c) w[c] = piv[c] + scale * tot[c];
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    const int64_t i = j0 + t + (int64_t)NT * r;
    const bool below = i > jk, at = i == jk;
    const double v = P[r][K] * scale;
    const double f = below ? tk * v : (at ? tk : 0.0);
#pragma unroll
    for (int c = K + 1; c < NB; ++c) P[r][c] = fma(-f, w[c], P[r][c]);
    P[r][K] = below ? v : (at ? beta : P[r][K]);
  }
  // T[0:K, K] = -tau_K T[0:K, 0:K] (V[:, 0:K]^T v_K), with
  // V[:, a]^T v_K = piv[a] + scale Y_a; T[K, K] = tau_K
  if (t < K) {
    // all K loads issued together (K is a compile-time bound; b < t adds zero)
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < K; ++b) {
      const double tb = Ts[b * NB + t];
      const double yb = piv[b] + scale * tot[b];
      s += b >= t ? tb * yb : 0.0;
    }
    Ts[K * NB + t] = -tk * s;
  }
  if (t == 0) {
    Ts[K * NB + K] = tk;
    tau[jk] = tk;
    if (!isfinite(nu)) flags[2] = 1.0;
  }
  // No barrier here: the next step's reduction barriers order every later
  // use of red, tot and Ts; each thread's Ts column entries are its own.
}

template <int MAXR, int NB, int NT, int K>
__device__ __forceinline__ void panel_steps(double (&P)[MAXR][NB], int t, int64_t j0, int nbw,
                                            double* red, double* tot, double* piv, double* Ts,
                                            double* __restrict__ tau, double* __restrict__ flags) {
  if constexpr (K < NB) {
    if (K < nbw) {
      panel_step<MAXR, NB, NT, K>(P, t, j0, red, tot, piv, Ts, tau, flags);
      panel_steps<MAXR, NB, NT, K + 1>(P, t, j0, nbw, red, tot, piv, Ts, tau, flags);
    }
  }
}

// Factor panel columns [j0, j0 + nbw) of M over rows [j0, d), nbw =
// min(NB, n - j0).  Thread t owns rows j0 + t + NT r, r < MAXR.  Writes R
// entries, Householder vectors (below the diagonal), tau, and T (NB x NB,
// column-major, upper).  One work item per problem; problems with n <= j0
// have nothing to do.
template <int MAXR, int NB, int NT>
__global__ __launch_bounds__(NT) void k_qr_panel(const QrArgs* __restrict__ P, Map mp,
                                                            int64_t j0) {
  __shared__ double red[NT * NB];
  __shared__ double tot[NB];
  __shared__ double piv[2 * NB];
  __shared__ double Ts[NB * NB];
  const int t = threadIdx.x;
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const QrArgs& a = P[map_find(mp, it)];
  const int64_t d = a.d;
  if (j0 >= a.n) return;
  const int nbw = (int)((a.n - j0) < NB ? (a.n - j0) : NB);
  double* __restrict__ M = a.M;
  double Pn[MAXR][NB];
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    const int64_t i = j0 + t + (int64_t)NT * r;
#pragma unroll
    for (int c = 0; c < NB; ++c) Pn[r][c] = (i < d && c < nbw) ? M[(j0 + c) * d + i] : 0.0;
  }
  for (int e = t; e < NB * NB; e += NT) Ts[e] = 0.0;
  __syncthreads();
  panel_steps<MAXR, NB, NT, 0>(Pn, t, j0, nbw, red, tot, piv, Ts, a.tau, a.scal);
  __syncthreads();  // Ts complete
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    const int64_t i = j0 + t + (int64_t)NT * r;
    if (i < d)
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nbw) M[(j0 + c) * d + i] = Pn[r][c];
  }
  for (int e = t; e < NB * NB; e += NT) a.T[e] = Ts[e];
}

// C <- (I - V T V^T)^T C = C - V (T^T (V^T C)) for the trailing columns
// [j0 + nbw, n] (Sb is the last one), rows [j0, d).  A work-group of NT
// threads owns CB columns (trail_cb).  Sweep 1: every thread accumulates its
// rows' share of W = V^T C in registers (independent loads, no barriers); W
// is reduced over the group through LDS in a fixed order and multiplied by
// T^T.  Sweep 2 applies the update from the same registers.
//
// Threads of the trailing work-group for panels of NB columns: 1024 for
// 8-column panels (half the rows per thread of 512 threads, so more loads in
// flight per work-group: 4.64 -> 4.47 ms for the 4000 x 1000 QR); 512 for
// 16-column panels (1024 threads with one column per group measured 1.54
// against 1.50 ms at 2048 x 512) and 4-column panels (1024 threads spill).
template <int NB>
constexpr int trail_threads() {
  return NB == 8 ? 1024 : 512;
}

// Two columns per work-group need 2 NB x NT doubles of LDS for the reduction.
template <int NB>
constexpr int trail_max_cb() {
  return (size_t)2 * NB * trail_threads<NB>() * sizeof(double) <= 140 * 1024 ? 2 : 1;
}

// Columns per trailing group when no tuned entry covers the problem (the
// reduction order, hence the rounding, follows it).  Since a work-group keeps
// V for all the groups it takes, one column per group is as fast as two or
// faster at every measured size (4000 x 1000: 4.04 against 4.28 ms; 3000 x
// 700: 2.46 against 2.66 ms; 2048 x 512 and 1024 x 256 equal or better),
// with one exception within 0.3 % (8192 x 600).
int trail_cb(int64_t) { return 1; }

template <int NB>
__device__ __forceinline__ double v_entry(const double* __restrict__ M, int64_t d, int64_t j0,
                                          int a, int nbw, int64_t i) {
  const int64_t ja = j0 + a;
  if (a >= nbw) return 0.0;
  return i > ja ? M[ja * d + i] : (i == ja ? 1.0 : 0.0);
}

// A problem's trailing columns at step j0 (Sb included) form
// ceil(ntr / CB) groups of CB; its nit work items take groups loc,
// loc + nit, ...  (nit is capped so that one problem's items are resident
// together: a step then runs as one round of work-groups, and V is read once
// per work-group rather than once per group of columns).  Thread t owns rows
// j0 + t + NT r, r < MAXR (d <= MAXR NT): its entries of V stay in registers
// for all of the item's columns, and those of its columns from the first
// sweep to the second.  Every column's arithmetic (and its reduction order)
// is the same whichever item takes it.
template <int MAXR, int NB, int CB, int NT>
__global__ __launch_bounds__(NT) void k_qr_trailing(const QrArgs* __restrict__ P, Map mp,
                                                    int64_t j0) {
  constexpr int NV = NB * CB;
  __shared__ double red[NV * NT];
  __shared__ double W[NV];
  __shared__ double Wt[NV];
  __shared__ double Ts[NB * NB];
  static_assert(NB * NB <= NT, "one entry of T per thread");
  const int t = threadIdx.x;
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const int pi = map_find(mp, it);
  const QrArgs& a = P[pi];
  const uint32_t loc = it - mp.off[pi];
  const uint32_t nit = mp.off[pi + 1] - mp.off[pi];
  const int64_t d = a.d, n = a.n;
  if (j0 >= n) return;
  const int nbw = (int)((n - j0) < NB ? (n - j0) : NB);
  const int64_t ntr = n + 1 - (j0 + nbw);
  const int64_t ngrp = (ntr + CB - 1) / CB;
  if ((int64_t)loc >= ngrp) return;  // uniform over the work-group
  double* __restrict__ M = a.M;
  // T once per work-group for all its column groups (the first reduction's
  // barriers publish it)
  if (t < NB * NB) Ts[t] = a.T[t];
  double v[MAXR][NB];
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    const int64_t i = j0 + t + (int64_t)NT * r;
    const bool in = i < d;
#pragma unroll
    for (int q = 0; q < NB; ++q) v[r][q] = in ? v_entry<NB>(M, d, j0, q, nbw, i) : 0.0;
  }
  // this thread's entries of the columns of group g (zero past d or n)
  auto load_cols = [&](int64_t g, double (&dst)[MAXR][CB]) {
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
      const int64_t i = j0 + t + (int64_t)NT * r;
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int64_t j = j0 + nbw + g * CB + c;
        dst[r][c] = (i < d && j <= n) ? M[j * d + i] : 0.0;
      }
    }
  };
  for (int64_t g = loc; g < ngrp; g += nit) {
    double cv[MAXR][CB];
    load_cols(g, cv);
    const int64_t jc0 = j0 + nbw + g * CB;
    int64_t jc[CB];
    bool ok[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      jc[c] = jc0 + c;
      ok[c] = jc[c] <= n;
    }
    double acc[NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) acc[e] = 0.0;
#pragma unroll
    for (int r = 0; r < MAXR; ++r)
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[q * CB + c] = fma(v[r][q], cv[r][c], acc[q * CB + c]);
    // (the previous group's reads of W and Wt ended before this reduction's
    // first barrier)
    block_reduce_multi<NV, NT>(acc, red, W);
    // W' = T^T W with T upper triangular (column-major NB x NB)
    if (t < NV) {
      const int q = t / CB, c = t % CB;
      double s = 0.0;
      for (int b2 = 0; b2 <= q && b2 < nbw; ++b2) s += Ts[q * NB + b2] * W[b2 * CB + c];
      Wt[t] = q < nbw ? s : 0.0;
    }
    __syncthreads();
    double wt[NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) wt[e] = Wt[e];
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
      const int64_t i = j0 + t + (int64_t)NT * r;
      if (i >= d) continue;
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        if (!ok[c]) continue;
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q) s = fma(v[r][q], wt[q * CB + c], s);
        M[jc[c] * d + i] = cv[r][c] - s;
      }
    }
  }
}

// R out of the factored M: Rc (column-major, ld n), Rr and the optional Rout
// (row-major) and invd = 1 / diag, by 32 x 32 tiles transposed through LDS
// (a work item is one tile; tiles below the diagonal write zeros).
__global__ void k_qr_extract(const QrArgs* __restrict__ P, Map mp) {
  __shared__ double tile[32][33];
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  const int pi = map_find(mp, it);
  const QrArgs& a = P[pi];
  const uint32_t loc = it - mp.off[pi];
  const int64_t d = a.d, n = a.n;
  const double* __restrict__ M = a.M;
  const uint32_t tiles = (uint32_t)((n + 31) / 32);
  const int64_t i0 = (int64_t)(loc % tiles) * 32, j0 = (int64_t)(loc / tiles) * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  for (int c = ty; c < 32; c += 8) {
    const int64_t j = j0 + c, i = i0 + tx;
    double v = 0.0;
    if (i < n && j < n) {
      if (i <= j) v = M[j * d + i];
      a.R[j * n + i] = v;
    }
    tile[c][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + r, j = j0 + tx;
    if (i < n && j < n) {
      const double v = tile[tx][r];
      a.Rr[i * n + j] = v;
      if (a.Rout) a.Rout[i * n + j] = v;
    }
  }
  if (i0 == j0 && ty == 0 && i0 + tx < n) a.invd[i0 + tx] = 1.0 / M[(i0 + tx) * d + i0 + tx];
}

// rho, rank and finiteness checks, and x0 = R^{-1} c (R and invd from
// k_qr_extract).  One work item (1024 threads) per problem.
__device__ __forceinline__ void qr_finish_item(const QrArgs& a, double* sh) {
  const int64_t d = a.d, n = a.n;
  const double* __restrict__ M = a.M;
  double* x = sh;            // n
  double* blk = sh + n;      // 64 x 64
  double* red = blk + 4096;  // 16
  const int t = threadIdx.x, nt = blockDim.x;
  double s = 0.0;
  for (int64_t i = n + t; i < d; i += nt) {
    const double v = M[n * d + i];
    s += v * v;
  }
  const double rho = sqrt(block_sum(s, red));
  double mx = 0.0;
  bool bad = false;
  for (int64_t i = t; i < n; i += nt) {
    const double r = M[i * d + i];
    mx = fmax(mx, fabs(r));
    if (!isfinite(r)) bad = true;
  }
  const double maxdiag = block_max(mx, red);
  const double thr = 10.0 * (double)n * 1.1102230246251565e-16 * maxdiag;
  double small = 0.0;
  for (int64_t i = t; i < n; i += nt)
    if (fabs(M[i * d + i]) <= thr) small = 1.0;
  const double rankdef = block_max(small, red);
  const double nonfin =
      block_max(bad ? 1.0 : 0.0, red) + a.scal[2] + (isfinite(rho) ? 0.0 : 1.0);
  for (int64_t i = t; i < n; i += nt) x[i] = M[n * d + i];
  __syncthreads();
  __syncthreads();
  trsv_lds<true, 1024>(a.R, n, (int)n, a.invd, x, blk);
  for (int64_t i = t; i < n; i += nt) a.x0[i] = x[i];
  if (t == 0) {
    a.scal[0] = rho;
    a.scal[1] = rankdef;
    sns_info* info = a.info;
    info->status =
        nonfin > 0.0 ? SNS_ERR_NUMERICAL : (rankdef > 0.0 ? SNS_ERR_RANK_DEFICIENT : SNS_OK);
    info->iters = 0;
    info->rel_resid_est = 0.0;
    info->sketch_resid = rho;
  }
}

__global__ __launch_bounds__(1024) void k_qr_finish(const QrArgs* __restrict__ P, Map mp) {
  extern __shared__ double sh[];
  const uint32_t it = blockIdx.x;
  if (it >= mp.off[mp.nprob]) return;
  qr_finish_item(P[map_find(mp, it)], sh);
}

int qr_cfg_builtin(int64_t d) {
  if (d <= 512) return 0;
  if (d <= 1024) return 1;
  if (d <= 2048) return 2;
  if (d <= 4096) return 3;
  return 4;
}

// Panel configuration and trailing columns of a problem: a tuning-table
// entry when one covers (d, n) and its configuration holds d, else the
// built-in rule.
void qr_shape(int64_t d, int64_t n, int* cfg, int* cb) {
  int c = 0, b = 0;
  if (tune_qr_lookup(d, n, &c, &b) && qr_cfg_capacity(c) >= d && b >= 1 &&
      b <= qr_cfg_max_cb(c)) {
    *cfg = c;
    *cb = b;
    return;
  }
  *cfg = qr_cfg_builtin(d);
  const int mcb = qr_cfg_max_cb(*cfg);
  *cb = trail_cb(n) < mcb ? trail_cb(n) : mcb;
}

template <int MAXR, int NB, int NT, int CB>
void run_panels(const QrJob::Cls& c, hipStream_t st) {
  // rows per thread of the trailing update (d <= MAXR NT, the panel's bound)
  constexpr int NTT = trail_threads<NB>();
  constexpr int TR = (MAXR * NT + NTT - 1) / NTT;
  for (int64_t j0 = 0; j0 < c.maxn; j0 += NB) {
    SNS_LAUNCH("qr_panel", (k_qr_panel<MAXR, NB, NT>), dim3(grid_for((uint32_t)c.count)),
               dim3(NT), 0, st, c.args, c.mone, j0);
    if (c.ntrail)
      SNS_LAUNCH("qr_trailing", (k_qr_trailing<TR, NB, CB, NTT>), dim3(grid_for(c.ntrail)),
                 dim3(NTT), 0, st, c.args, c.mtrail, j0);
  }
}

// Trailing work-groups of configuration (MAXR, NB, NT) with CB columns that
// the device holds at once: its CU count times the kernel's occupancy.
template <int MAXR, int NB, int NT, int CB>
int trail_resident(int dev) {
  constexpr int NTT = trail_threads<NB>();
  constexpr int TR = (MAXR * NT + NTT - 1) / NTT;
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, reinterpret_cast<const void*>(&k_qr_trailing<TR, NB, CB, NTT>), NTT, 0) !=
          hipSuccess)
    return 0;
  return cus * (per > 0 ? per : 1);
}

template <int MAXR, int NB, int NT>
int trail_resident_cb(int cb, int dev) {
  if constexpr (trail_max_cb<NB>() == 2)
    if (cb == 2) return trail_resident<MAXR, NB, NT, 2>(dev);
  return trail_resident<MAXR, NB, NT, 1>(dev);
}

// Cap on the trailing work items of one problem (one round of resident
// work-groups; 0 = no cap), per device, configuration and width, computed
// once.
uint32_t trail_items_cap(int cfg, int cb) {
  constexpr int kDevs = 64;
  static std::atomic<int> cache[kDevs][5][2];  // 0 = not yet known, -1 = none
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevs || cfg < 0 || cfg > 4 ||
      cb < 1 || cb > 2)
    return 0;
  std::atomic<int>& slot = cache[dev][cfg][cb - 1];
  int v = slot.load();
  if (v == 0) {
    switch (cfg) {
      case 0: v = trail_resident_cb<2, 16, 256>(cb, dev); break;
      case 1: v = trail_resident_cb<4, 16, 256>(cb, dev); break;
      case 2: v = trail_resident_cb<4, 16, 512>(cb, dev); break;
      case 3: v = trail_resident_cb<8, 8, 512>(cb, dev); break;
      default: v = trail_resident_cb<16, 4, 512>(cb, dev); break;
    }
    if (v <= 0) v = -1;
    slot.store(v);
  }
  return v > 0 ? (uint32_t)v : 0u;
}

template <int MAXR, int NB, int NT>
void run_panels_cb(const QrJob::Cls& c, hipStream_t st) {
  if constexpr (trail_max_cb<NB>() == 2) {
    if (c.cb == 2) {
      run_panels<MAXR, NB, NT, 2>(c, st);
      return;
    }
  }
  run_panels<MAXR, NB, NT, 1>(c, st);
}

}  // namespace

size_t qr_workspace_bytes(int64_t d, int64_t n) {
  Carve c(nullptr, 0);
  QrBufs q;
  carve_qr(c, d, n, q);
  return c.off;
}

void carve_qr(Carve& c, int64_t d, int64_t n, QrBufs& q) {
  q.M = c.take<double>((size_t)d * (n + 1));
  q.T = c.take<double>(64 * 64);
  q.tau = c.take<double>((size_t)n);
  q.R = c.take<double>((size_t)n * n);
  q.Rr = c.take<double>((size_t)n * n);
  q.invd = c.take<double>((size_t)n);
  q.xw = c.take<double>((size_t)n);
  q.scal = c.take<double>(8);
}

QrArgs qr_args(int64_t d, int64_t n, const void* SA, int64_t ld_sa, const void* Sb,
               const QrBufs& q, double* x0, double* Rout, sns_info* info) {
  QrArgs a;
  a.d = d;
  a.n = n;
  a.ld_sa = ld_sa;
  a.SA = SA;
  a.Sb = Sb;
  a.M = q.M;
  a.T = q.T;
  a.tau = q.tau;
  a.R = q.R;
  a.Rr = q.Rr;
  a.invd = q.invd;
  a.x0 = x0;
  a.Rout = Rout;
  a.scal = q.scal;
  a.info = info;
  return a;
}

namespace {

// force_cfg < 0: each problem's own shape (qr_shape); else every problem in
// configuration force_cfg with force_cb trailing columns per work-group.
QrJob build_qr_job_impl(ArgTable& t, const std::vector<QrArgs>& a, bool f64, int force_cfg,
                        int force_cb) {
  QrJob j;
  j.f64 = f64;
  j.count = (int)a.size();
  if (a.empty()) return j;
  std::vector<uint32_t> load, one, ext;
  std::vector<int> pcfg, pcb;
  for (const QrArgs& x : a) {
    load.push_back((uint32_t)(((x.d + 31) / 32) * ((x.n + 1 + 31) / 32)));
    ext.push_back((uint32_t)(((x.n + 31) / 32) * ((x.n + 31) / 32)));
    one.push_back(1u);
    j.maxn = x.n > j.maxn ? x.n : j.maxn;
    int c = force_cfg, b = force_cb;
    if (force_cfg < 0) qr_shape(x.d, x.n, &c, &b);
    if (b > qr_cfg_max_cb(c)) b = qr_cfg_max_cb(c);  // the class's kernels take at most that
    if (b < 1) b = 1;
    pcfg.push_back(c);
    pcb.push_back(b);
  }
  j.all = t.add(a.data(), a.size());
  j.mload = t.map(load, &j.nload);
  j.mextract = t.map(ext, &j.nextract);
  uint32_t tmp = 0;
  j.mone = t.map(one, &tmp);
  for (int key = 0; key < 10; ++key) {
    const int cfg = key / 2, cb = 1 + key % 2;
    std::vector<QrArgs> sub;
    std::vector<uint32_t> cone, ctr;
    int64_t maxn = 0;
    for (size_t k = 0; k < a.size(); ++k) {
      const QrArgs& x = a[k];
      if (pcfg[k] != cfg || pcb[k] != cb) continue;
      sub.push_back(x);
      cone.push_back(1u);
      const uint32_t groups = (uint32_t)((x.n + cb - 1) / cb), cap = trail_items_cap(cfg, cb);
      ctr.push_back(cap > 0 && groups > cap ? cap : groups);
      maxn = x.n > maxn ? x.n : maxn;
    }
    if (sub.empty()) continue;
    QrJob::Cls c;
    c.cfg = cfg;
    c.cb = cb;
    c.args = t.add(sub.data(), sub.size());
    c.mone = t.map(cone, &tmp);
    c.mtrail = t.map(ctr, &c.ntrail);
    c.count = (int)sub.size();
    c.maxn = maxn;
    j.cls.push_back(c);
  }
  return j;
}

}  // namespace

QrJob build_qr_job(ArgTable& t, const std::vector<QrArgs>& a, bool f64) {
  return build_qr_job_impl(t, a, f64, -1, 0);
}

QrJob build_qr_job_forced(ArgTable& t, const std::vector<QrArgs>& a, bool f64, int cfg, int cb) {
  return build_qr_job_impl(t, a, f64, cfg, cb);
}

int qr_cfg_max_cb(int cfg) {
  switch (cfg) {
    case 0: case 1: case 2: return trail_max_cb<16>();
    case 3: return trail_max_cb<8>();
    case 4: return trail_max_cb<4>();
    default: return 0;
  }
}

int64_t qr_cfg_capacity(int cfg) {
  switch (cfg) {
    case 0: return 2 * 256;
    case 1: return 4 * 256;
    case 2: return 4 * 512;
    case 3: return 8 * 512;
    case 4: return 16 * 512;
    default: return 0;
  }
}

sns_status launch_qr_job(const QrJob& j, hipStream_t st) {
  if (j.count == 0) return SNS_OK;
  region_begin("qr", st);
  if (j.f64)
    SNS_LAUNCH("qr_load", k_qr_load<double>, dim3(grid_for(j.nload)), dim3(32, 8), 0, st, j.all,
               j.mload);
  else
    SNS_LAUNCH("qr_load", k_qr_load<float>, dim3(grid_for(j.nload)), dim3(32, 8), 0, st, j.all,
               j.mload);
  for (const QrJob::Cls& c : j.cls) {
    switch (c.cfg) {
      // panel configurations: rows per thread, panel width, threads (d <= NT * MAXR)
      case 0: run_panels_cb<2, 16, 256>(c, st); break;
      case 1: run_panels_cb<4, 16, 256>(c, st); break;
      case 2: run_panels_cb<4, 16, 512>(c, st); break;
      case 3: run_panels_cb<8, 8, 512>(c, st); break;
      default: run_panels_cb<16, 4, 512>(c, st); break;
    }
  }
  SNS_LAUNCH("qr_extract", k_qr_extract, dim3(grid_for(j.nextract)), dim3(32, 8), 0, st, j.all,
             j.mextract);
  const size_t lds = ((size_t)j.maxn + 4096 + 16) * sizeof(double);
  SNS_LAUNCH("qr_finish", k_qr_finish, dim3(grid_for((uint32_t)j.count)), dim3(1024), lds, st,
             j.all, j.mone);
  region_end(st);
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace sns
