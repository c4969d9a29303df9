// Internal launchers of libsns (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/sns.h"

namespace sns {

// Kernel timing hooks (no-ops unless timing is enabled).
void timing_begin(const char* name, hipStream_t s);
void timing_end(hipStream_t s);

#define SNS_LAUNCH(name, kernel, grid, block, lds, stream, ...)              \
  do {                                                                      \
    ::sns::timing_begin(name, stream);                                      \
    hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);      \
    ::sns::timing_end(stream);                                              \
  } while (0)

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Bump allocator over a caller-provided workspace.
struct Carve {
  char* base;
  size_t off = 0;
  size_t cap;
  Carve(void* p, size_t c) : base(static_cast<char*>(p)), cap(c) {}
  template <typename T>
  T* take(size_t count) {
    off = align_up(off);
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
  bool ok() const { return off <= cap; }
};

// ---------------------------------------------------------------- sort ----
// Stable counting sort of rows 0..m-1 by CountSketch bucket.  Produces
// perm[m] (row id with the sign in bit 31, rows ascending inside a bucket),
// bucket_ptr[d+1], and, when b is given, bperm[m] = s(i) b[i] in perm order.
struct SortPlan {
  int64_t m = 0;
  uint32_t d = 0;
  int64_t rw = 0;       // rows per wave-block
  int64_t nwb = 0;      // wave-blocks
  int waves = 1;        // waves per work-group in count/scatter
  int64_t seg = 64;     // wave-blocks per scan segment
  int64_t nseg = 0;     // scan segments
};
SortPlan make_sort_plan(int64_t m, uint32_t d);
struct SortBufs {
  uint32_t* perm;
  void* bperm;
  uint32_t* bucket_ptr;
  uint32_t* counts;
  uint32_t* segtot;
};
void carve_sort(Carve& c, const SortPlan& p, size_t b_elem_bytes, SortBufs& s);
// rows (optional, ascending): sort rows[0..m) instead of 0..m-1; b is then
// indexed by the row id.  mdev (optional): device-side key count <= p.m.
sns_status launch_bucket_sort(const SortPlan& p, uint64_t seed, const void* b, sns_dtype bt,
                              const SortBufs& s, hipStream_t st, const uint32_t* rows = nullptr,
                              const uint32_t* mdev = nullptr);

// ------------------------------------------------------------------ CSR ----
// CountSketch of a CSR matrix: SA (d x n, A's dtype) and, when b is given,
// Sb (d).  Deterministic; see csr.hip.
size_t csr_workspace_bytes(const sns_matrix& A, uint32_t d, bool acc64);
sns_status launch_csr_sketch(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b,
                             void* SA, void* Sb, bool acc64, void* ws, size_t ws_bytes,
                             hipStream_t st);
sns_status launch_hash(uint64_t seed, uint32_t d, int64_t i0, int64_t count, uint32_t* h,
                       int8_t* s, hipStream_t st);

// ---------------------------------------------------------- CountSketch ----
struct GatherPlan {
  int vec = 1, lpr = 64, ct = 64, coltiles = 1, nseg = 1;
  bool acc64 = false;
};
GatherPlan make_gather_plan(const sns_matrix& A, uint32_t d, bool acc64);
size_t gather_partial_bytes(const GatherPlan& g, const sns_matrix& A, uint32_t d);
sns_status launch_cs_gather(const GatherPlan& g, const sns_matrix& A, uint32_t d,
                            const SortBufs& s, bool with_b, void* SA, void* Sb, void* part,
                            hipStream_t st);

// ------------------------------------------------------------------- QR ----
struct QrBufs {
  double* M;      // d x (n+1) column-major working copy of [SA | Sb]
  double* T;      // nb x nb compact-WY factor of the current panel
  double* tau;    // n
  double* R;      // n x n column-major copy of R (ld n)
  double* Rr;     // n x n row-major copy of R (ld n)
  double* invd;   // n: 1 / R_jj
  double* xw;     // n: x0, then scratch
  double* scal;   // small scalars: [0] rho, [1] rank-deficient flag, [2] non-finite flag
};
size_t qr_workspace_bytes(int64_t d, int64_t n);
void carve_qr(Carve& c, int64_t d, int64_t n, QrBufs& q);
// Factor [SA | Sb] and solve R x0 = c.  Writes x0 (fp64 n) and, if Rout is
// set, R row-major.  info_dev (device sns_info) gets status and sketch_resid.
sns_status launch_qr_solve(int64_t d, int64_t n, sns_dtype dt, const void* SA, int64_t ld_sa,
                           const void* Sb, const QrBufs& q, double* x0, double* Rout,
                           sns_info* info_dev, hipStream_t st);

// ----------------------------------------------------------------- LSQR ----
struct LsqrState;  // device-resident scalars, defined in lsqr.hip
struct LsqrBufs {
  void* u;          // m, A's dtype: the unnormalised Golub-Kahan vector
  double* zpart;    // G x n partial A^T u
  double* npart;    // G partial ||u||^2
  double* zred2;    // first-level reduction of zpart
  double* nred2;    // first-level reduction of npart
  double* Xc;       // X = R^{-1}, column-major (n x n)
  double* Xr;       // X = R^{-1}, row-major (n x n)
  double* ypart;    // per-group shares of ||y||^2 in k_lsqr_xtz
  double* vecs;     // 6 n: w_pass, v, wd, dy, y, scratch
  void* state;      // LsqrState
};
struct LsqrPlan {
  int grid = 512;   // work-groups of the fused pass
  int lpr = 16;     // lanes per row
  int nch = 4;      // column chunks per lane (a chunk is 16 bytes per lane)
  int unroll = 1;   // rows per slot and step (1 or 2)
};
LsqrPlan make_lsqr_plan(const sns_matrix& A);
size_t lsqr_workspace_bytes(const sns_matrix& A, const LsqrPlan& p);
void carve_lsqr(Carve& c, const sns_matrix& A, const LsqrPlan& p, LsqrBufs& l);
// SAP-SAS refinement: LSQR on A R^{-1} from r0 = b - A x0.  R is the n x n
// column-major factor in q.R; x0 in q.xw.  Writes x (fp64 n) and updates
// info_dev (iters, rel_resid_est, status).
sns_status launch_sap_refine(const sns_matrix& A, const void* b, const LsqrPlan& p,
                             const LsqrBufs& l, const QrBufs& q, int d, int max_iters,
                             double rtol, double* x, sns_info* info_dev, hipStream_t st);

// ------------------------------------------------------------- Gaussian ----
const uint16_t* gauss_table_host();
size_t gauss_workspace_bytes(const sns_matrix& A, uint32_t d);
sns_status launch_gauss_sketch(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b,
                               void* SA, void* Sb, void* ws, hipStream_t st);

}  // namespace sns
