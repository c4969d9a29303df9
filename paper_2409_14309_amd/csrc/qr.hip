// Householder QR of the augmented sketch [SA | Sb] (d x (n+1)) in fp64 and
// the triangular solve R x0 = c, c = (Q^T Sb)[:n]: step 3 of sketch-and-solve.
//
// Layout: the working copy M is column-major with leading dimension d.
// Blocked right-looking algorithm: for each panel of nb columns,
//   k_qr_panel    one work-group of 512 threads holds the panel rows in
//                 registers and factors it column by column.  Each column
//                 needs one work-group reduction, which yields the norm, the
//                 products of the column with the remaining panel columns
//                 (for the rank-1 update) and with the earlier Householder
//                 vectors (for the compact-WY factor T).
//   k_qr_trailing applies (I - V T V^T)^T to the trailing columns, Sb
//                 included; each work-group owns 8 columns.
// Reflector convention (LAPACK): beta = -sign(alpha) ||x|| (sign(0) = +1),
// tau = (beta - alpha) / beta, v = x / (alpha - beta) with v[0] = 1.
#include "common.hpp"
#include "kernels.hpp"
#include "linalg.hpp"

namespace sns {

namespace {

constexpr int kPanelThreads = 512;

// M[j * d + i] = SA[i * ld + j] (j < n), M[n * d + i] = Sb[i], via 32x32 tiles.
template <typename T>
__global__ void k_qr_load(int64_t d, int64_t n, const T* __restrict__ SA, int64_t ld,
                          const T* __restrict__ Sb, double* __restrict__ M) {
  __shared__ double tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
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
    if (i < d && j <= n) M[j * d + i] = tile[tx][c];
  }
}

// One Householder step of the panel, column K (a compile-time index so the
// register array P is never indexed at run time).
template <int MAXR, int NB, int K>
__device__ __forceinline__ void panel_step(double (&P)[MAXR][NB], int t, int64_t j0, int64_t d,
                                           double* red, double* tot, double* piv, double* Ts,
                                           double* __restrict__ tau, double* __restrict__ flags) {
  const int64_t jk = j0 + K;  // pivot row, owned by thread K (r = 0)
  // partial sums over the rows below the pivot, x = column K there:
  // G_c = x . M[:, c] (c >= K) and Y_a = x . V[:, a] (a < K).  Rows at or
  // above the pivot contribute x = 0; rows past d hold zeros.
  double g[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) g[c] = 0.0;
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    const int64_t i = j0 + t + (int64_t)kPanelThreads * r;
    const double x = i > jk ? P[r][K] : 0.0;
#pragma unroll
    for (int c = 0; c < NB; ++c) g[c] = fma(x, P[r][c], g[c]);
  }
  if (t == K) {
#pragma unroll
    for (int c = 0; c < NB; ++c) piv[c] = P[0][c];
  }
  block_reduce_multi<NB, kPanelThreads>(g, red, tot);  // its barriers also publish piv
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
    const int64_t i = j0 + t + (int64_t)kPanelThreads * r;
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
    double s = 0.0;
    for (int b = t; b < K; ++b) s += Ts[b * NB + t] * (piv[b] + scale * tot[b]);
    Ts[K * NB + t] = -tk * s;
  }
  if (t == 0) {
    Ts[K * NB + K] = tk;
    tau[jk] = tk;
    if (!isfinite(nu)) flags[2] = 1.0;
  }
  __syncthreads();
}

template <int MAXR, int NB, int K>
__device__ __forceinline__ void panel_steps(double (&P)[MAXR][NB], int t, int64_t j0, int64_t d,
                                            int nbw, double* red, double* tot, double* piv,
                                            double* Ts, double* __restrict__ tau,
                                            double* __restrict__ flags) {
  if constexpr (K < NB) {
    if (K < nbw) {
      panel_step<MAXR, NB, K>(P, t, j0, d, red, tot, piv, Ts, tau, flags);
      panel_steps<MAXR, NB, K + 1>(P, t, j0, d, nbw, red, tot, piv, Ts, tau, flags);
    }
  }
}

// Factor panel columns [j0, j0 + nbw) of M over rows [j0, d).  Thread t owns
// rows j0 + t + 512 r, r < MAXR.  Writes R entries, Householder vectors
// (below the diagonal), tau, and T (NB x NB, column-major, upper).
template <int MAXR, int NB>
__global__ __launch_bounds__(kPanelThreads) void k_qr_panel(int64_t d, int64_t j0, int nbw,
                                                            double* __restrict__ M,
                                                            double* __restrict__ tau,
                                                            double* __restrict__ Tg,
                                                            double* __restrict__ flags) {
  __shared__ double red[kPanelThreads * NB];
  __shared__ double tot[NB];
  __shared__ double piv[NB];
  __shared__ double Ts[NB * NB];
  const int t = threadIdx.x;
  double P[MAXR][NB];
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    const int64_t i = j0 + t + (int64_t)kPanelThreads * r;
#pragma unroll
    for (int c = 0; c < NB; ++c) P[r][c] = (i < d && c < nbw) ? M[(j0 + c) * d + i] : 0.0;
  }
  for (int e = t; e < NB * NB; e += kPanelThreads) Ts[e] = 0.0;
  __syncthreads();
  panel_steps<MAXR, NB, 0>(P, t, j0, d, nbw, red, tot, piv, Ts, tau, flags);
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    const int64_t i = j0 + t + (int64_t)kPanelThreads * r;
    if (i < d)
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nbw) M[(j0 + c) * d + i] = P[r][c];
  }
  for (int e = t; e < NB * NB; e += kPanelThreads) Tg[e] = Ts[e];
}

// C <- (I - V T V^T)^T C = C - V (T^T (V^T C)) for the trailing columns
// [j0 + nbw, n] (Sb is the last one), rows [j0, d).  A work-group owns CB
// columns.  Sweep 1: every thread accumulates its rows' share of W = V^T C in
// registers (independent loads, no barriers); W is reduced over the group
// through LDS in a fixed order and multiplied by T^T.  Sweep 2 re-reads V and
// C and applies the update.
constexpr int kTrailThreads = 256;
constexpr int kTrailCB = 4;

template <int NB>
__device__ __forceinline__ double v_entry(const double* __restrict__ M, int64_t d, int64_t j0,
                                          int a, int nbw, int64_t i) {
  const int64_t ja = j0 + a;
  if (a >= nbw) return 0.0;
  return i > ja ? M[ja * d + i] : (i == ja ? 1.0 : 0.0);
}

template <int NB>
__global__ __launch_bounds__(kTrailThreads) void k_qr_trailing(int64_t d, int64_t n, int64_t j0,
                                                               int nbw, double* __restrict__ M,
                                                               const double* __restrict__ Tg) {
  constexpr int CB = kTrailCB, NT = kTrailThreads, NV = NB * CB;
  __shared__ double red[NV * NT];
  __shared__ double W[NV];
  __shared__ double Wt[NV];
  const int t = threadIdx.x;
  const int64_t jc0 = j0 + nbw + (int64_t)blockIdx.x * CB;
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
  for (int64_t i = j0 + t; i < d; i += NT) {
    double v[NB], cv[CB];
#pragma unroll
    for (int a = 0; a < NB; ++a) v[a] = v_entry<NB>(M, d, j0, a, nbw, i);
#pragma unroll
    for (int c = 0; c < CB; ++c) cv[c] = ok[c] ? M[jc[c] * d + i] : 0.0;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int c = 0; c < CB; ++c) acc[a * CB + c] = fma(v[a], cv[c], acc[a * CB + c]);
  }
  block_reduce_multi<NV, NT>(acc, red, W);
  // W' = T^T W with T upper triangular (column-major NB x NB)
  if (t < NV) {
    const int a = t / CB, c = t % CB;
    double s = 0.0;
    for (int b2 = 0; b2 <= a && b2 < nbw; ++b2) s += Tg[a * NB + b2] * W[b2 * CB + c];
    Wt[t] = a < nbw ? s : 0.0;
  }
  __syncthreads();
  double wt[NV];
#pragma unroll
  for (int e = 0; e < NV; ++e) wt[e] = Wt[e];
  for (int64_t i = j0 + t; i < d; i += NT) {
    double v[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) v[a] = v_entry<NB>(M, d, j0, a, nbw, i);
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      if (!ok[c]) continue;
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < NB; ++a) s = fma(v[a], wt[a * CB + c], s);
      M[jc[c] * d + i] -= s;
    }
  }
}

// rho, R (column-major copy and optional row-major output), rank and
// finiteness checks, and x0 = R^{-1} c.  One work-group.
__global__ __launch_bounds__(1024) void k_qr_finish(int64_t d, int64_t n,
                                                    const double* __restrict__ M,
                                                    double* __restrict__ Rc,
                                                    double* __restrict__ Rr,
                                                    double* __restrict__ invd,
                                                    double* __restrict__ Rout,
                                                    double* __restrict__ x0,
                                                    double* __restrict__ flags,
                                                    sns_info* __restrict__ info) {
  extern __shared__ double sh[];
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
  for (int64_t e = t; e < n * n; e += nt) {
    const int64_t j = e / n, i = e % n;  // Rc[j * n + i] = R[i, j]
    const double v = i <= j ? M[j * d + i] : 0.0;
    Rc[e] = v;
    Rr[i * n + j] = v;
    if (Rout) Rout[i * n + j] = v;
  }
  for (int64_t i = t; i < n; i += nt) invd[i] = 1.0 / M[i * d + i];
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
  const double nonfin = block_max(bad ? 1.0 : 0.0, red) + flags[2] + (isfinite(rho) ? 0.0 : 1.0);
  for (int64_t i = t; i < n; i += nt) x[i] = M[n * d + i];
  __syncthreads();
  __syncthreads();
  trsv_lds<true, 1024>(Rc, n, (int)n, invd, x, blk);
  for (int64_t i = t; i < n; i += nt) x0[i] = x[i];
  if (t == 0) {
    flags[0] = rho;
    flags[1] = rankdef;
    info->status = nonfin > 0.0 ? SNS_ERR_NUMERICAL : (rankdef > 0.0 ? SNS_ERR_RANK_DEFICIENT : SNS_OK);
    info->iters = 0;
    info->rel_resid_est = 0.0;
    info->sketch_resid = rho;
  }
}

__global__ void k_zero(double* p, int64_t count) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = 0.0;
}

template <int MAXR, int NB>
void run_panels(int64_t d, int64_t n, const QrBufs& q, hipStream_t st) {
  for (int64_t j0 = 0; j0 < n; j0 += NB) {
    const int nbw = (int)((n - j0) < NB ? (n - j0) : NB);
    SNS_LAUNCH("qr_panel", (k_qr_panel<MAXR, NB>), dim3(1), dim3(kPanelThreads), 0, st, d, j0, nbw,
                       q.M, q.tau, q.T, q.scal);
    const int64_t ntr = n + 1 - (j0 + nbw);
    if (ntr > 0)
      SNS_LAUNCH("qr_trailing", (k_qr_trailing<NB>), dim3((unsigned)((ntr + kTrailCB - 1) / kTrailCB)),
                 dim3(kTrailThreads), 0, st,
                         d, n, j0, nbw, q.M, q.T);
  }
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

sns_status launch_qr_solve(int64_t d, int64_t n, sns_dtype dt, const void* SA, int64_t ld_sa,
                           const void* Sb, const QrBufs& q, double* x0, double* Rout,
                           sns_info* info_dev, hipStream_t st) {
  if (d > 8192 || n > 4096) return SNS_ERR_SHAPE;
  SNS_LAUNCH("zero", k_zero, dim3(1), dim3(64), 0, st, q.scal, (int64_t)8);
  const dim3 lg((unsigned)((d + 31) / 32), (unsigned)((n + 1 + 31) / 32));
  if (dt == SNS_F64)
    SNS_LAUNCH("qr_load", k_qr_load<double>, lg, dim3(32, 8), 0, st, d, n,
                       static_cast<const double*>(SA), ld_sa, static_cast<const double*>(Sb), q.M);
  else
    SNS_LAUNCH("qr_load", k_qr_load<float>, lg, dim3(32, 8), 0, st, d, n,
                       static_cast<const float*>(SA), ld_sa, static_cast<const float*>(Sb), q.M);
  if (d <= 512) run_panels<1, 16>(d, n, q, st);
  else if (d <= 1024) run_panels<2, 16>(d, n, q, st);
  else if (d <= 2048) run_panels<4, 16>(d, n, q, st);
  else if (d <= 4096) run_panels<8, 8>(d, n, q, st);
  else run_panels<16, 4>(d, n, q, st);
  const size_t lds = ((size_t)n + 4096 + 16) * sizeof(double);
  SNS_LAUNCH("qr_finish", k_qr_finish, dim3(1), dim3(1024), lds, st, d, n, q.M, q.R, q.Rr, q.invd,
             Rout, x0, q.scal,
                     info_dev);
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace sns
