// SAA-SAS (sketch-and-apply, the second solver in the paper's solver list):
// the preconditioned matrix Y = A X with X = R^{-1} is formed once,
// explicitly, and LSQR then runs on Y itself instead of applying X on both
// sides of every pass.
//
// k_form_y: Y = A X for A (m x n, row-major, fp32 or fp64) and the upper-
// triangular X (n x n, row-major fp64, zeros below the diagonal).  Products
// and sums are fp64 (A's values are widened exactly); Y is stored in A's
// dtype with row stride ldy.  Work-group tile: 128 rows x 128 columns of Y,
// K-steps of 16 rows of X staged in LDS; a column tile starting at j0 only
// needs the rows k < j0 + 128 of X (X is upper triangular), so the product
// costs about m n^2 multiply-adds, taken on the fp64 matrix cores.
#include "common.hpp"
#include "kernels.hpp"

namespace sns {

namespace {

constexpr int kYT = 128, kYK = 16, kYThreads = 256, kYPad = 2;

template <typename T>
__global__ __launch_bounds__(kYThreads, 2) void k_form_y(const T* __restrict__ A, int64_t ld,
                                                      int64_t m, int n,
                                                      const double* __restrict__ X,
                                                      T* __restrict__ Y, int64_t ldy, int ctn) {
  __shared__ __attribute__((aligned(16))) T As[kYK][kYT + kYPad];  // A's dtype, widened when read
  __shared__ __attribute__((aligned(16))) double Xs[kYK][kYT + kYPad];
  const int t = threadIdx.x;
  // Work-groups are handed to the 8 XCDs in turn; renumber them so that the
  // column tiles of one row tile, which read the same rows of A, run on one
  // XCD and share those rows in its L2.
  const unsigned nwg = gridDim.x, h = blockIdx.x;
  const unsigned L = (nwg % 8u == 0u) ? (h % 8u) * (nwg / 8u) + h / 8u : h;
  const int cj = (int)(L % (unsigned)ctn);
  const int64_t i0 = (int64_t)(L / (unsigned)ctn) * kYT;
  const int j0 = cj * kYT;
  const int kend = j0 + kYT < n ? j0 + kYT : n;  // X[k][j] = 0 for k > j
  const int nk = (kend + kYK - 1) / kYK;

  // A loader: row ar of the tile, K-columns 8 ah .. 8 ah + 7 of the step
  const int ar = t & (kYT - 1), ah = t >> 7;
  const int64_t ai = i0 + ar;
  const T* arow = A + (ai < m ? ai : 0) * ld;
  // X loader: row xk of the step, columns 8 xq .. 8 xq + 7 of the tile
  const int xk = t >> 4, xq = t & 15;
  T ra[8];
  double rx[8];
  auto load = [&](int k0) {
    const int ka = k0 + 8 * ah;
    if (ai < m && ka + 8 <= n) {
      if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          const double2 v = *reinterpret_cast<const double2*>(arow + ka + e);
          ra[e] = (T)v.x;
          ra[e + 1] = (T)v.y;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; e += 4) {
          const float4 v = *reinterpret_cast<const float4*>(arow + ka + e);
          ra[e] = (T)v.x; ra[e + 1] = (T)v.y; ra[e + 2] = (T)v.z; ra[e + 3] = (T)v.w;
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] = (ai < m && ka + e < n) ? arow[ka + e] : T(0);
    }
    const int kx = k0 + xk;
    const double* xrow = X + (int64_t)(kx < n ? kx : 0) * n;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int j = j0 + 8 * xq + e;
      rx[e] = (kx < n && j < n) ? xrow[j] : 0.0;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < 8; ++e) As[8 * ah + e][ar] = ra[e];
#pragma unroll
    for (int e = 0; e < 8; ++e) Xs[xk][8 * xq + e] = rx[e];
  };

  // products on the matrix cores: wave (wr, wc) owns rows [64 wr, 64 wr + 64)
  // and columns [64 wc, 64 wc + 64) of the tile as 4 x 4 tiles of 16 x 16,
  // each v_mfma_f64_16x16x4f64 adding 4 K-rows: lane l supplies
  // A[16 rt + l % 16][k + l / 16] and X[k + l / 16][16 ct + l % 16].
  typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;
  const int lane = t & 63, wave = t >> 6, wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc[4][4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[rt][ct][q] = 0.0;

  load(0);
  for (int kb = 0; kb < nk; ++kb) {
    __syncthreads();  // the previous step's reads are done
    store();
    __syncthreads();
    if (kb + 1 < nk) load((kb + 1) * kYK);  // in flight during the products
#pragma unroll
    for (int k4 = 0; k4 < kYK; k4 += 4) {
      double a[4], x[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = (double)As[k4 + lk][64 * wr + 16 * r + li];
#pragma unroll
      for (int c = 0; c < 4; ++c) x[c] = Xs[k4 + lk][64 * wc + 16 * c + li];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], x[c], acc[r][c], 0, 0, 0);
    }
  }
  // accumulator element q of lane l in a 16 x 16 fp64 tile: row l / 16 + 4 q, column l % 16
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = i0 + 64 * wr + 16 * r + lk + 4 * q;
      if (i >= m) continue;
      T* yrow = Y + i * ldy;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int j = j0 + 64 * wc + 16 * c + li;
        if (j < n) yrow[j] = (T)acc[r][c][q];
      }
    }
}

}  // namespace

int64_t saa_ldy(const sns_matrix& A) {
  const int64_t per16 = A.dtype == SNS_F64 ? 2 : 4;
  return (A.n + per16 - 1) / per16 * per16;
}

sns_status launch_form_y(const SaaJob& y, hipStream_t st) {
  if (!y.Y) return SNS_OK;
  const int ctn = (y.n + kYT - 1) / kYT;
  const int64_t rtn = (y.m + kYT - 1) / kYT;
  const int64_t blocks = rtn * ctn;
  if (blocks > 0x7FFFFFFF) return SNS_ERR_SHAPE;
  if (y.f64)
    SNS_LAUNCH("form_y", k_form_y<double>, dim3((unsigned)blocks), dim3(kYThreads), 0, st,
               static_cast<const double*>(y.A), y.ld, y.m, y.n, y.X, static_cast<double*>(y.Y),
               y.ldy, ctn);
  else
    SNS_LAUNCH("form_y", k_form_y<float>, dim3((unsigned)blocks), dim3(kYThreads), 0, st,
               static_cast<const float*>(y.A), y.ld, y.m, y.n, y.X, static_cast<float*>(y.Y),
               y.ldy, ctn);
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}

}  // namespace sns
