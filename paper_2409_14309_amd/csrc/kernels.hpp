// Internal launchers of libsns (not part of the C ABI).
//
// Every kernel of the sort, CountSketch, QR and LSQR steps is batched: it
// reads its per-problem arguments from a device-resident table, and work-group
// g takes work item g, problem p owning items [off[p], off[p+1]).  A
// single solve is a batch of one; a batch of uneven problems runs the same
// kernels with the same per-problem arithmetic, so a problem's result does
// not depend on what else is in the batch.  The host builds the argument
// tables (ArgTable) and uploads them with a kernel launch, so a launch
// sequence can be captured in a HIP graph.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/sns.h"

namespace sns {

// Kernel timing hooks (no-ops unless timing is enabled).
void timing_begin(const char* name, hipStream_t s);
void timing_end(hipStream_t s);
// The same for a phase of several launches (one region open per thread).
void region_begin(const char* name, hipStream_t s);
void region_end(hipStream_t s);

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

// ------------------------------------------------------------ batching ----
// Work-item map of a batched launch (device pointers).
struct Map {
  const uint32_t* off;  // nprob + 1 entries; off[nprob] = total items
  int nprob;
};

// Problem owning work item `item` (binary search; the value is uniform over
// the work-group, so the loads are scalar).
__device__ __forceinline__ int map_find(const Map& mp, uint32_t item) {
  int lo = 0, hi = mp.nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (mp.off[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Work-groups are handed to the 8 XCDs in turn.  Item order that gives XCD x
// the x-th contiguous eighth of the first 8 floor(n / 8) items (the rest keep
// their place), so neighbouring items share one L2.  A bijection on [0, n).
__device__ __forceinline__ uint32_t xcd_order(uint32_t h, uint32_t n) {
  const uint32_t q = n / 8u;
  return h < 8u * q ? (h % 8u) * q + h / 8u : h;
}

// Work-groups to launch for `total` items: one per item (work-groups past
// the last item return at once, so a launch may be sized for more).
inline unsigned grid_for(uint32_t total) { return total ? total : 1u; }

// Host builder of the device argument table.  Entries are appended to a host
// image whose device location is known up front (dev may be null to size
// it); upload() copies the image with kernel launches (no host memory is
// referenced after it returns).
class ArgTable {
 public:
  explicit ArgTable(void* dev = nullptr) : dev_(static_cast<char*>(dev)) {}
  template <typename T>
  T* add(const T* items, size_t count) {
    const size_t off = reserve(sizeof(T) * count);
    if (count) memcpy_bytes(off, items, sizeof(T) * count);
    return reinterpret_cast<T*>(dev_ ? dev_ + off : nullptr);
  }
  // Offsets of a map from per-problem item counts; `total` receives the sum.
  Map map(const std::vector<uint32_t>& counts, uint32_t* total);
  size_t bytes() const { return host_.size(); }
  sns_status upload(hipStream_t st) const;

 private:
  size_t reserve(size_t nbytes);
  void memcpy_bytes(size_t off, const void* src, size_t nbytes);
  std::vector<unsigned char> host_;
  char* dev_;
};
// Alignment of the entries of an argument table (bytes).
constexpr size_t kArgTableAlign = 16;

// ---------------------------------------------------------------- sort ----
// Stable counting sort of rows 0..m-1 by CountSketch bucket.  Produces
// perm[m] (row id with the sign in bit 31, rows ascending inside a bucket),
// bucket_ptr[d+1], and, when b is given, bperm[m] = s(i) b[i] in perm order.
// The counting pass keeps each key's bucket and sign (hkey, 2 bytes a key)
// for the placing pass, so every key is hashed once.
struct SortPlan {
  int64_t m = 0;        // keys: rows x zeta
  uint32_t d = 0;
  uint32_t zeta = 1;    // nonzeros per column of S (key t: row t / zeta, hash t % zeta)
  int64_t rw = 0;       // rows per wave-block
  int64_t nwb = 0;      // wave-blocks
  int64_t seg = 64;     // wave-blocks per scan segment
  int64_t nseg = 0;     // scan segments
};
SortPlan make_sort_plan(int64_t keys, uint32_t d, uint32_t zeta = 1);
// Nonzeros per column of the sketch (1 for the CountSketch).
inline uint32_t sketch_zeta(const sns_sketch& sk) {
  return sk.kind == SNS_SKETCH_SPARSE_SIGN ? (uint32_t)sk.zeta : 1u;
}
struct SortBufs {
  uint16_t* hkey;  // bucket of each key (bits 0-14) and its sign (bit 15)
  uint32_t* perm;
  void* bperm;
  uint32_t* bucket_ptr;
  uint32_t* counts;
  uint32_t* segtot;
};
void carve_sort(Carve& c, const SortPlan& p, size_t b_elem_bytes, SortBufs& s);
// One problem's sort.  rows (optional, ascending): sort rows[0..m) instead of
// 0..m-1; b is then indexed by the row id.  mdev (optional): device-side key
// count <= m.
struct SortArgs {
  uint64_t seed;
  int64_t m, rw, nwb, seg, nseg;
  uint32_t d;
  uint32_t zeta;  // > 1: key t is hash t % zeta of row t / zeta (no row list)
  const uint32_t* rows;
  const uint32_t* mdev;
  const void* b;
  uint16_t* hkey;
  uint32_t* perm;
  void* bperm;
  uint32_t* bucket_ptr;
  uint32_t* counts;
  uint32_t* segtot;
};
SortArgs sort_args(const SortPlan& p, uint64_t seed, const void* b, const SortBufs& s,
                   const uint32_t* rows = nullptr, const uint32_t* mdev = nullptr);
// A batched sort launch sequence (all problems share b's element type).
struct SortJob {
  const SortArgs* args = nullptr;
  Map mcount{}, mseg{}, mscan{};
  uint32_t ncount = 0, nseg = 0, nscan = 0;
  uint32_t maxd = 1;
  bool f64 = false;
  bool staged = false;   // place through LDS (every group's keys fit)
  int cap = 0;           // staged keys per group
  size_t place_lds = 0;  // LDS bytes of the staged placing
  int count = 0;
};
SortJob build_sort_job(ArgTable& t, const std::vector<SortArgs>& a, bool f64);
sns_status launch_sort_job(const SortJob& j, hipStream_t st);
sns_status launch_hash(uint64_t seed, uint32_t d, int64_t i0, int64_t count, uint32_t* h,
                       int8_t* s, hipStream_t st);

// ---------------------------------------------------------- CountSketch ----
struct GatherPlan {
  int vec = 1, lpr = 64, ct = 64, coltiles = 1, nseg = 1;
  bool acc64 = false;
};
GatherPlan make_gather_plan(const sns_matrix& A, uint32_t d, bool acc64, int64_t keys = -1);
size_t gather_partial_bytes(const GatherPlan& g, const sns_matrix& A, uint32_t d);
struct GatherArgs {
  const void* A;
  int64_t ld;
  int n, nseg, coltiles, red_blocks;
  uint32_t d;
  const uint32_t* perm;
  const void* bperm;  // null: no Sb
  const uint32_t* bucket_ptr;
  void* SA;
  void* Sb;
  void* partA;
  void* partB;
};
GatherArgs gather_args(const GatherPlan& g, const sns_matrix& A, uint32_t d, const SortBufs& s,
                       bool with_b, void* SA, void* Sb, void* part);
struct GatherProb {  // host-side pairing of a plan with its arguments
  GatherPlan plan;
  GatherArgs args;
  sns_dtype dtype;
};
struct GatherLaunch {
  GatherPlan plan;  // class (vec, lpr, acc64) shared by the launch
  sns_dtype dtype;
  const GatherArgs* args;
  Map map;
  uint32_t items;
  const GatherArgs* rargs;  // problems with segment partials
  Map rmap;
  uint32_t ritems;
};
std::vector<GatherLaunch> build_gather_job(ArgTable& t, const std::vector<GatherProb>& p);
sns_status launch_gather_job(const std::vector<GatherLaunch>& j, hipStream_t st);

// ------------------------------------------------------------------ CSR ----
// CountSketch of a CSR matrix: SA (d x n, A's dtype) and, when b is given,
// Sb (d).  Deterministic; see csr.hip.
size_t csr_workspace_bytes(const sns_matrix& A, uint32_t d, bool acc64);
sns_status launch_csr_sketch(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b,
                             void* SA, void* Sb, bool acc64, void* ws, size_t ws_bytes,
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
// set, R row-major.  info (device sns_info) gets status and sketch_resid.
struct QrArgs {
  int64_t d, n, ld_sa;
  const void* SA;
  const void* Sb;
  double* M;
  double* T;
  double* tau;
  double* R;
  double* Rr;
  double* invd;
  double* x0;
  double* Rout;
  double* scal;
  sns_info* info;
};
QrArgs qr_args(int64_t d, int64_t n, const void* SA, int64_t ld_sa, const void* Sb,
               const QrBufs& q, double* x0, double* Rout, sns_info* info);
struct QrJob {
  bool f64 = false;  // SA element type
  const QrArgs* all = nullptr;
  Map mload{}, mone{}, mextract{};
  uint32_t nload = 0, nextract = 0;
  int count = 0;
  int64_t maxn = 0;
  struct Cls {
    int cfg;  // panel configuration index
    int cb;   // trailing columns per work item
    const QrArgs* args;
    Map mone, mtrail;
    uint32_t ntrail;
    int count;
    int64_t maxn;
  };
  std::vector<Cls> cls;
};
QrJob build_qr_job(ArgTable& t, const std::vector<QrArgs>& a, bool f64);
sns_status launch_qr_job(const QrJob& j, hipStream_t st);

// ---------------------------------------------------------------- fused ----
// Sketch, QR and x0 of problems with d <= 256, n <= 64 and m (n + 1) <= 2^21
// (CountSketch, dense) in one persistent launch over a device queue of row chunks
// (fused.hip).  Writes what the blocked QR path writes for the refinement:
// R (column-major), 1 / diag, x0, scal and the device sns_info.
constexpr int64_t kMaxFusedElems = int64_t(1) << 21;  // m (n + 1) of a fused problem
struct FusedCtl {
  unsigned head;  // next queue item; zero in the uploaded table
  int nprob;      // problems in the table
  unsigned pad[2];
};
struct FusedArgs {
  const void* A;
  const void* b;
  int64_t ld, m;
  int n, d;
  uint64_t seed;
  int vec;             // rows of A may be read four entries at a time (16-byte aligned)
  int64_t rc;          // rows per chunk
  int nchunk, ngroup;  // chunks, and groups of chunks summed together
  double* part;        // nchunk x d (n + 1) chunk partials (nchunk > 1)
  double* gpart;       // ngroup x d (n + 1) group partials (ngroup > 1)
  double* msys;        // d x (n + 1): the summed system, handed to the QR's registers
  double* R;
  double* invd;
  double* x0;
  double* scal;
  sns_info* info;
  unsigned cnt[12];    // [0] group arrivals, [1 + g] chunk arrivals of group g; zero in the table
};
struct FusedPlan {
  int64_t rc = 0;
  int nchunk = 0, ngroup = 0, dn = 0;
};
struct FusedJob {
  bool f64 = false;
  int count = 0;
  const FusedCtl* ctl = nullptr;
  const FusedArgs* args = nullptr;
  Map map{};
  uint32_t items = 0;
};
bool fused_eligible(const sns_sketch& sk, const sns_matrix& A);
FusedPlan make_fused_plan(const sns_sketch& sk, const sns_matrix& A);
struct FusedBufs {
  double* part = nullptr;
  double* gpart = nullptr;
  double* msys = nullptr;
};
void carve_fused(Carve& c, const FusedPlan& p, FusedBufs& f);
FusedArgs fused_args(const FusedPlan& p, const sns_sketch& sk, const sns_matrix& A, const void* b,
                     const FusedBufs& f, const QrBufs& q, double* x0, sns_info* info);
FusedJob build_fused_job(ArgTable& t, const std::vector<FusedArgs>& a, bool f64);
sns_status launch_fused_job(const FusedJob& j, hipStream_t st);
// A fused table of fixed capacity for replayed graphs: control block, then
// max_probs FusedArgs, then max_probs + 1 chunk offsets.
struct FusedTableLayout {
  int max_probs = 0;
  size_t args_off = 0, off_off = 0, bytes = 0;
};
FusedTableLayout fused_table_layout(int max_probs);
// Writes the table image of the problems a into img (host memory) and its
// size in 8-byte words; false if they exceed the capacity.
bool fused_table_fill(void* img, const FusedTableLayout& L, const std::vector<FusedArgs>& a,
                      uint64_t* words);
// Captures (on st) and instantiates the graph of one set-up: a kernel copies
// the image at host_img (pinned; *host_words words, read at replay time)
// into dev_tab, then the persistent fused launch runs on dev_tab's problems.
sns_status fused_graph_create(void* dev_tab, const FusedTableLayout& L, const void* host_img,
                              const uint64_t* host_words, bool f64, hipStream_t st,
                              hipGraphExec_t* exec);

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
  int waves = 4;    // waves per work-group (4 or 8)
};
LsqrPlan make_lsqr_plan(const sns_matrix& A);
// Tuning-table lookup (tune.hip): the entry for (dtype, n, m), if any.
bool tune_lookup(sns_dtype dt, int64_t n, int64_t m, LsqrPlan* p);
// Tuned gather shape (lanes per row, segments per bucket) and blocked-QR
// shape (panel configuration, trailing columns per work-group), if the table
// has an entry for the problem.
bool tune_gather_lookup(sns_dtype dt, int64_t n, int64_t d, int64_t m, int* lpr, int* nseg);
bool tune_qr_lookup(int64_t d, int64_t n, int* cfg, int* cb);
// Gather plan with the given lanes per row and segments (clamped to what the
// problem allows).
GatherPlan gather_plan_with(const sns_matrix& A, uint32_t d, bool acc64, int64_t keys, int lpr,
                            int nseg);
// Rows a QR panel configuration holds (d <= capacity), or 0 if cfg is unknown.
int64_t qr_cfg_capacity(int cfg);
// Most trailing columns per work-group a panel configuration supports (1 or
// 2; 0 if cfg is unknown).
int qr_cfg_max_cb(int cfg);
// The QR job with every problem forced to one panel configuration and
// trailing-column count (for the tuner).
QrJob build_qr_job_forced(ArgTable& t, const std::vector<QrArgs>& a, bool f64, int cfg, int cb);
// Whether the pass is instantiated for (lpr, nch).
bool lsqr_plan_valid(int lpr, int nch);
// Time the fused pass on A with plan p: average microseconds over `reps`
// launches after one warm-up, on a state that never stops.
sns_status time_lsqr_pass(const sns_matrix& A, const LsqrPlan& p, int reps, void* ws,
                          size_t ws_bytes, hipStream_t st, double* us);
size_t tune_workspace_bytes(const sns_matrix& A);
size_t lsqr_workspace_bytes(const sns_matrix& A, const LsqrPlan& p);
void carve_lsqr(Carve& c, const sns_matrix& A, const LsqrPlan& p, LsqrBufs& l);
struct LsqrArgs {
  const void* A;
  int64_t ld, m;
  int n, grid, max_iters;
  const void* b;
  void* u;
  double* zpart;
  double* npart;
  double* zred2;
  double* nred2;
  double* Xc;
  double* Xr;
  double* ypart;
  double* vecs;
  LsqrState* st;
  const double* Rc;
  const double* invd;
  const double* x0;
  double* x;
  sns_info* info;
  double sighat, stop;
  const void* Y;  // SAA-SAS: explicit A R^{-1} (A's dtype, row stride ldy); null for SAP-SAS
  int64_t ldy;
};
// SAP-SAS refinement of one problem: LSQR on A R^{-1} from r0 = b - A x0.  R
// is the n x n column-major factor in q.R; x0 in q.xw.  Writes x (fp64 n) and
// updates info (iters, rel_resid_est, status).
LsqrArgs lsqr_args(const sns_matrix& A, const void* b, const LsqrPlan& p, const LsqrBufs& l,
                   const QrBufs& q, int d, int max_iters, double rtol, double* x,
                   sns_info* info, const void* Y = nullptr, int64_t ldy = 0);
// SAA-SAS: Y = A X (X = R^{-1}, row-major fp64) formed once after X.
struct SaaJob {
  const void* A = nullptr;
  int64_t ld = 0, m = 0;
  int n = 0;
  const double* X = nullptr;
  void* Y = nullptr;
  int64_t ldy = 0;
  bool f64 = false;
};
int64_t saa_ldy(const sns_matrix& A);
sns_status launch_form_y(const SaaJob& y, hipStream_t st);
struct LsqrProb {
  LsqrPlan plan;
  LsqrArgs args;
};
struct LsqrJob {
  bool f64 = false;
  SaaJob saa;  // single-problem SAA-SAS only
  const LsqrArgs* all = nullptr;
  Map mone{}, minv{}, mred{}, mgemv{};
  uint32_t ninv = 0, nred = 0, ngemv = 0;
  int count = 0;
  int maxn = 0;
  bool unfused = false;  // some problem has n above the fused-step limit
  struct Cls {
    LsqrPlan plan;  // lpr, nch, unroll of the class
    const LsqrArgs* args;
    Map map;
    uint32_t items;
  };
  std::vector<Cls> cls;
  // single problem: its device state and stop threshold, for host polling
  const LsqrState* state = nullptr;
  double stop = 0.0, sighat = 0.0;
};
LsqrJob build_lsqr_job(ArgTable& t, const std::vector<LsqrProb>& p, bool f64);
// Set-up (X = R^{-1}, state), as many iterations as needed (single problem:
// host polling of the stop flag; several problems: `max_iters` of them,
// finished problems skipping), the final update and the report.
sns_status launch_lsqr_setup(const LsqrJob& j, hipStream_t st);
// ring: pinned host slots (kPollSlots of them) that a single-problem job
// posts its stop state to after every iteration, tagged with `epoch`; null
// for none.
struct PollSlot;
sns_status launch_lsqr_iteration(const LsqrJob& j, hipStream_t st, PollSlot* ring = nullptr,
                                 unsigned int epoch = 0);
sns_status launch_lsqr_finish(const LsqrJob& j, hipStream_t st);
sns_status run_lsqr_single(const LsqrJob& j, int max_iters, bool adaptive, hipStream_t st);
// Number of problems of the job that have not stopped, written to *out
// (device int) on the stream.
sns_status launch_lsqr_active(const LsqrJob& j, int* out, hipStream_t st);
// out[p] (device ints) = 1 once problem p of the job has stopped.
sns_status launch_lsqr_flags(const LsqrJob& j, int* out, hipStream_t st);

// ------------------------------------------------------------- Gaussian ----
const uint16_t* gauss_table_host();
size_t gauss_workspace_bytes(const sns_matrix& A, uint32_t d);
// Hadamard sketch (SRHT): the transformed blocks B (m' x (n + 1)) and its launch.
size_t hadamard_workspace_bytes(const sns_matrix& A, uint32_t d);
sns_status launch_hadamard_sketch(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b,
                                  void* SA, void* Sb, void* ws, hipStream_t st);
sns_status launch_gauss_sketch(const sns_matrix& A, uint32_t d, uint64_t seed, const void* b,
                               void* SA, void* Sb, void* ws, hipStream_t st);

}  // namespace sns
