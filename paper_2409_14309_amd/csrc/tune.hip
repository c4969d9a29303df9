// Autotuner of the launch shapes and the tuning table the plan lookups
// consult.  sns_tune_pass times every valid candidate of the refinement pass
// (lanes per row and chunks per lane that cover n without more than doubling
// the padded width, work-group counts from 64 to 4096, one or two rows per
// step, 4 or 8 waves per work-group, 8 only for problems of at least 2^29
// entries) on the caller's matrix and reports the fastest; sns_tune_gather does
// the same for the CountSketch gather (lanes per row, segments per bucket)
// after one bucket sort, and sns_tune_qr for the blocked Householder QR
// (panel configuration, width of the trailing column groups) on a given [SA | Sb].
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "solve.hpp"

namespace sns {

namespace {

struct Table {
  std::mutex mu;
  std::vector<sns_tune_entry> rows;
  std::vector<sns_tune_gather_entry> grows;
  std::vector<sns_tune_qr_entry> qrows;
};

Table& table() {
  static Table t;
  return t;
}

bool same_key(const sns_tune_entry& a, const sns_tune_entry& b) {
  return a.dtype == b.dtype && a.n == b.n && a.m_lo == b.m_lo && a.m_hi == b.m_hi;
}

void put(Table& t, const sns_tune_entry& e) {
  for (sns_tune_entry& r : t.rows)
    if (same_key(r, e)) {
      r = e;
      return;
    }
  t.rows.push_back(e);
}

void put(Table& t, const sns_tune_gather_entry& e) {
  for (sns_tune_gather_entry& r : t.grows)
    if (r.dtype == e.dtype && r.n == e.n && r.d == e.d && r.m_lo == e.m_lo && r.m_hi == e.m_hi) {
      r = e;
      return;
    }
  t.grows.push_back(e);
}

void put(Table& t, const sns_tune_qr_entry& e) {
  for (sns_tune_qr_entry& r : t.qrows)
    if (r.d_lo == e.d_lo && r.d_hi == e.d_hi && r.n_lo == e.n_lo && r.n_hi == e.n_hi) {
      r = e;
      return;
    }
  t.qrows.push_back(e);
}

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

bool gather_entry_ok(const sns_tune_gather_entry& e) {
  return (e.dtype == SNS_F32 || e.dtype == SNS_F64) && e.n >= 1 && e.d >= 1 &&
         e.m_lo <= e.m_hi && pow2_in(e.lpr, 4, 64) && pow2_in(e.nseg, 1, 64);
}

bool qr_entry_ok(const sns_tune_qr_entry& e) {
  return e.d_lo >= 1 && e.d_lo <= e.d_hi && e.n_lo >= 1 && e.n_lo <= e.n_hi &&
         qr_cfg_capacity(e.cfg) >= e.d_hi && e.cb >= 1 && e.cb <= qr_cfg_max_cb(e.cfg);
}

// Average time of one call of `run` over `reps` calls after one warm-up,
// bracketed by events on stream st.
template <typename F>
sns_status time_calls(F&& run, int reps, hipStream_t st, double* us) {
  sns_status s = run();
  if (s != SNS_OK) return s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SNS_HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SNS_ERR_HIP;
  }
  float ms = 0.f;
  hipError_t he = hipEventRecord(e0, st);
  for (int r = 0; r < reps && he == hipSuccess && s == SNS_OK; ++r) s = run();
  if (he == hipSuccess) he = hipEventRecord(e1, st);
  if (he == hipSuccess) he = hipEventSynchronize(e1);
  if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != SNS_OK) return s;
  SNS_HIP_TRY(he);
  *us = 1000.0 * ms / reps;
  return SNS_OK;
}

constexpr size_t kTuneArgBytes = 8192;

// Workspace layout of the gather tuner: the sort's buffers, the largest
// segment partials any candidate needs, SA, Sb and an argument table.
struct GatherTuneWs {
  SortPlan sp;
  SortBufs sb{};
  void* part = nullptr;
  void* SA = nullptr;
  void* Sb = nullptr;
  char* args = nullptr;
};

void carve_gather_tune(Carve& c, const sns_matrix& A, uint32_t d, GatherTuneWs& w) {
  w.sp = make_sort_plan(A.m, d, 1);
  carve_sort(c, w.sp, elem(A), w.sb);
  GatherPlan big;
  big.acc64 = true;
  big.nseg = 64;
  w.part = c.take<char>(gather_partial_bytes(big, A, d));
  w.SA = c.take<char>((size_t)d * A.n * elem(A));
  w.Sb = c.take<char>((size_t)d * elem(A));
  w.args = c.take<char>(kTuneArgBytes);
}

sns_status check_gather_tune(const sns_matrix* A, int64_t d) {
  sns_status s = check_matrix(A);
  if (s != SNS_OK) return s;
  if (A->layout != SNS_DENSE_ROWMAJOR) return SNS_ERR_DTYPE;
  if (d < A->n || d > kMaxD || d > A->m || A->n > 4096) return SNS_ERR_SHAPE;
  return SNS_OK;
}

struct QrTuneWs {
  QrBufs q{};
  sns_info* info = nullptr;
  char* args = nullptr;
};

void carve_qr_tune(Carve& c, int64_t d, int64_t n, QrTuneWs& w) {
  carve_qr(c, d, n, w.q);
  w.info = c.take<sns_info>(1);
  w.args = c.take<char>(kTuneArgBytes);
}

}  // namespace

bool tune_gather_lookup(sns_dtype dt, int64_t n, int64_t d, int64_t m, int* lpr, int* nseg) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  for (const sns_tune_gather_entry& r : t.grows) {
    if (r.dtype != (int)dt || r.n != n || r.d != d || m < r.m_lo || m > r.m_hi) continue;
    *lpr = r.lpr;
    *nseg = r.nseg;
    return true;
  }
  return false;
}

bool tune_qr_lookup(int64_t d, int64_t n, int* cfg, int* cb) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  for (const sns_tune_qr_entry& r : t.qrows) {
    if (d < r.d_lo || d > r.d_hi || n < r.n_lo || n > r.n_hi) continue;
    *cfg = r.cfg;
    *cb = r.cb;
    return true;
  }
  return false;
}

bool tune_lookup(sns_dtype dt, int64_t n, int64_t m, LsqrPlan* p) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  for (const sns_tune_entry& r : t.rows) {
    if (r.dtype != (int)dt || r.n != n || m < r.m_lo || m > r.m_hi) continue;
    p->lpr = r.lpr;
    p->nch = r.nch;
    p->grid = r.grid;
    p->unroll = r.unroll;
    p->waves = r.waves;
    return true;
  }
  return false;
}

}  // namespace sns

using namespace sns;

extern "C" {

sns_status sns_tune_workspace_size(const sns_matrix* A, size_t* bytes) {
  sns_status s = check_matrix(A);
  if (s != SNS_OK) return s;
  if (!bytes || A->layout != SNS_DENSE_ROWMAJOR || A->n > 2048) return SNS_ERR_INVALID_ARG;
  *bytes = tune_workspace_bytes(*A);
  return SNS_OK;
}

sns_status sns_tune_pass(const sns_matrix* A, int reps, void* workspace, size_t ws_bytes,
                         sns_tune_entry* best, void* stream) {
  sns_status s = check_matrix(A);
  if (s != SNS_OK) return s;
  if (!best || !workspace || reps < 1 || A->layout != SNS_DENSE_ROWMAJOR || A->n > 2048)
    return SNS_ERR_INVALID_ARG;
  const size_t es = elem(*A);
  if (((uintptr_t)A->values % 16) != 0 || (A->ld * es) % 16 != 0) return SNS_ERR_SHAPE;
  const int vw = (int)(16 / es);
  const int lprs[5] = {4, 8, 16, 32, 64};
  const int nchs[4] = {1, 2, 4, 8};
  // 8-wave work-groups only for problems that fill the device alone (m n >=
  // 2^29): in a batch the small problems share the device, and there their
  // larger work-groups measured slower (serving mix 3086 -> 2676 solves/s)
  const int max_waves = (int64_t)A->m * A->n >= (int64_t(1) << 29) ? 8 : 4;
  sns_tune_entry b{};
  b.us = -1.0;
  for (int li = 0; li < 5; ++li)
    for (int ci = 0; ci < 4; ++ci) {
      const int lpr = lprs[li], nch = nchs[ci];
      const int64_t cover = (int64_t)lpr * nch * vw;
      if (!lsqr_plan_valid(lpr, nch) || cover < A->n) continue;
      if (cover >= 2 * A->n && cover > 16) continue;  // more than half of every row padding
      for (int grid = 64; grid <= 4096; grid *= 2) {
        if (grid > 64 && (int64_t)grid * 64 > A->m) break;  // fewer than 64 rows per group
        for (int unroll = 1; unroll <= 2; ++unroll)
          for (int waves = 4; waves <= max_waves; waves += 4) {
            LsqrPlan p;
            p.lpr = lpr;
            p.nch = nch;
            p.grid = grid;
            p.unroll = unroll;
            p.waves = waves;
            double us = 0.0;
            s = time_lsqr_pass(*A, p, reps, workspace, ws_bytes, (hipStream_t)stream, &us);
            if (s != SNS_OK) return s;
            if (b.us < 0.0 || us < b.us) {
              b.lpr = lpr;
              b.nch = nch;
              b.grid = grid;
              b.unroll = unroll;
              b.waves = waves;
              b.us = us;
            }
          }
      }
    }
  if (b.us < 0.0) return SNS_ERR_SHAPE;
  b.dtype = (int)A->dtype;
  b.n = (int)A->n;
  b.m_lo = b.m_hi = A->m;
  *best = b;
  return SNS_OK;
}

sns_status sns_tune_gather_workspace_size(const sns_matrix* A, int64_t d, size_t* bytes) {
  sns_status s = check_gather_tune(A, d);
  if (s != SNS_OK) return s;
  if (!bytes) return SNS_ERR_INVALID_ARG;
  Carve c(nullptr, 0);
  GatherTuneWs w;
  carve_gather_tune(c, *A, (uint32_t)d, w);
  *bytes = c.off;
  return SNS_OK;
}

sns_status sns_tune_gather(const sns_matrix* A, const void* b, int64_t d, uint64_t seed, int reps,
                           void* workspace, size_t ws_bytes, sns_tune_gather_entry* best,
                           void* stream) {
  sns_status s = check_gather_tune(A, d);
  if (s != SNS_OK) return s;
  if (!best || !workspace || !b || reps < 1) return SNS_ERR_INVALID_ARG;
  const hipStream_t st = (hipStream_t)stream;
  Carve c(workspace, ws_bytes);
  GatherTuneWs w;
  carve_gather_tune(c, *A, (uint32_t)d, w);
  if (!c.ok()) return SNS_ERR_OUT_OF_MEMORY;
  {  // the bucket sort once: every candidate gathers the same permutation
    ArgTable t(w.args);
    const SortJob j = build_sort_job(t, std::vector<SortArgs>{sort_args(w.sp, seed, b, w.sb)},
                                     A->dtype == SNS_F64);
    if (t.bytes() > kTuneArgBytes) return SNS_ERR_OUT_OF_MEMORY;
    s = t.upload(st);
    if (s == SNS_OK) s = launch_sort_job(j, st);
    if (s != SNS_OK) return s;
  }
  const bool acc64 = default_opts().accum_fp64 != 0;
  const int64_t maxseg = A->m / (d * 256);
  sns_tune_gather_entry bst{};
  bst.us = -1.0;
  for (int lpr = 4; lpr <= 64; lpr *= 2) {
    const GatherPlan probe = gather_plan_with(*A, (uint32_t)d, acc64, A->m, lpr, 1);
    if (lpr > 4 && probe.ct >= 2 * A->n) break;  // more than half of the tile padding
    for (int nseg = 1; nseg <= 64; nseg *= 2) {
      if (nseg > 1 && nseg > maxseg) break;
      const GatherPlan gp = gather_plan_with(*A, (uint32_t)d, acc64, A->m, lpr, nseg);
      ArgTable t(w.args);
      GatherProb g;
      g.plan = gp;
      g.args = gather_args(gp, *A, (uint32_t)d, w.sb, true, w.SA, w.Sb, w.part);
      g.dtype = A->dtype;
      const std::vector<GatherLaunch> j = build_gather_job(t, std::vector<GatherProb>{g});
      if (t.bytes() > kTuneArgBytes) return SNS_ERR_OUT_OF_MEMORY;
      s = t.upload(st);
      if (s != SNS_OK) return s;
      double us = 0.0;
      s = time_calls([&]() { return launch_gather_job(j, st); }, reps, st, &us);
      if (s != SNS_OK) return s;
      if (bst.us < 0.0 || us < bst.us) {
        bst.lpr = lpr;
        bst.nseg = gp.nseg;
        bst.us = us;
      }
    }
  }
  bst.dtype = (int)A->dtype;
  bst.n = (int)A->n;
  bst.d = (int)d;
  bst.m_lo = bst.m_hi = A->m;
  *best = bst;
  return SNS_OK;
}

sns_status sns_tune_qr_workspace_size(int64_t d, int64_t n, size_t* bytes) {
  if (!bytes) return SNS_ERR_INVALID_ARG;
  if (n < 1 || d < n || d > kMaxQrD || n > 4096) return SNS_ERR_SHAPE;
  Carve c(nullptr, 0);
  QrTuneWs w;
  carve_qr_tune(c, d, n, w);
  *bytes = c.off;
  return SNS_OK;
}

sns_status sns_tune_qr(int dtype, int64_t d, int64_t n, const void* SA, const void* Sb, int reps,
                       void* workspace, size_t ws_bytes, sns_tune_qr_entry* best, void* stream) {
  if (dtype != SNS_F32 && dtype != SNS_F64) return SNS_ERR_DTYPE;
  if (!SA || !Sb || !best || !workspace || reps < 1) return SNS_ERR_INVALID_ARG;
  if (n < 1 || d < n || d > kMaxQrD || n > 4096) return SNS_ERR_SHAPE;
  const hipStream_t st = (hipStream_t)stream;
  Carve c(workspace, ws_bytes);
  QrTuneWs w;
  carve_qr_tune(c, d, n, w);
  if (!c.ok()) return SNS_ERR_OUT_OF_MEMORY;
  const std::vector<QrArgs> qa{qr_args(d, n, SA, n, Sb, w.q, w.q.xw, nullptr, w.info)};
  sns_tune_qr_entry bst{};
  bst.us = -1.0;
  for (int cfg = 0; cfg < 5; ++cfg) {
    if (qr_cfg_capacity(cfg) < d) continue;
    for (int cb = 1; cb <= qr_cfg_max_cb(cfg); ++cb) {
      ArgTable t(w.args);
      const QrJob j = build_qr_job_forced(t, qa, dtype == SNS_F64, cfg, cb);
      if (t.bytes() > kTuneArgBytes) return SNS_ERR_OUT_OF_MEMORY;
      sns_status s = t.upload(st);
      if (s != SNS_OK) return s;
      double us = 0.0;
      s = time_calls([&]() { return launch_qr_job(j, st); }, reps, st, &us);
      if (s != SNS_OK) return s;
      if (bst.us < 0.0 || us < bst.us) {
        bst.cfg = cfg;
        bst.cb = cb;
        bst.us = us;
      }
    }
  }
  bst.d_lo = bst.d_hi = (int)d;
  bst.n_lo = bst.n_hi = (int)n;
  *best = bst;
  return SNS_OK;
}

sns_status sns_tune_gather_set(const sns_tune_gather_entry* e) {
  if (!e || !gather_entry_ok(*e)) return SNS_ERR_INVALID_ARG;
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  put(t, *e);
  return SNS_OK;
}

sns_status sns_tune_qr_set(const sns_tune_qr_entry* e) {
  if (!e || !qr_entry_ok(*e)) return SNS_ERR_INVALID_ARG;
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  put(t, *e);
  return SNS_OK;
}

sns_status sns_tune_set(const sns_tune_entry* e) {
  if (!e || e->n < 1 || e->m_lo > e->m_hi || !lsqr_plan_valid(e->lpr, e->nch) || e->grid < 1 ||
      e->grid > 65535 || (e->unroll != 1 && e->unroll != 2) ||
      (e->dtype != SNS_F32 && e->dtype != SNS_F64) ||
      (e->waves != 0 && e->waves != 4 && e->waves != 8))
    return SNS_ERR_INVALID_ARG;
  sns_tune_entry c = *e;
  if (c.waves == 0) c.waves = 4;
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  put(t, c);
  return SNS_OK;
}

sns_status sns_tune_clear(void) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  t.rows.clear();
  t.grows.clear();
  t.qrows.clear();
  return SNS_OK;
}

sns_status sns_tune_load(const char* path) {
  if (!path) return SNS_ERR_INVALID_ARG;
  FILE* f = fopen(path, "r");
  if (!f) return SNS_ERR_INVALID_ARG;
  char line[512];
  std::vector<sns_tune_entry> rows;
  std::vector<sns_tune_gather_entry> grows;
  std::vector<sns_tune_qr_entry> qrows;
  bool ok = true;
  while (ok && fgets(line, sizeof(line), f)) {
    const char* p = line;
    while (*p == ' ' || *p == '\t') ++p;
    if (*p == '#' || *p == '\n' || *p == '\0') continue;
    long long lo = 0, hi = 0;
    if (*p == 'G') {  // G dtype n d m_lo m_hi lpr nseg us
      sns_tune_gather_entry e{};
      ok = sscanf(p + 1, "%d %d %d %lld %lld %d %d %lf", &e.dtype, &e.n, &e.d, &lo, &hi, &e.lpr,
                  &e.nseg, &e.us) == 8;
      e.m_lo = lo;
      e.m_hi = hi;
      ok = ok && gather_entry_ok(e);
      if (ok) grows.push_back(e);
    } else if (*p == 'Q') {  // Q d_lo d_hi n_lo n_hi cfg cb us
      sns_tune_qr_entry e{};
      ok = sscanf(p + 1, "%d %d %d %d %d %d %lf", &e.d_lo, &e.d_hi, &e.n_lo, &e.n_hi, &e.cfg,
                  &e.cb, &e.us) == 7 && qr_entry_ok(e);
      if (ok) qrows.push_back(e);
    } else {  // dtype n m_lo m_hi lpr nch grid unroll us [waves] (refinement pass)
      sns_tune_entry e{};
      e.waves = 4;
      const int got = sscanf(p, "%d %d %lld %lld %d %d %d %d %lf %d", &e.dtype, &e.n, &lo, &hi,
                             &e.lpr, &e.nch, &e.grid, &e.unroll, &e.us, &e.waves);
      ok = got == 9 || got == 10;
      e.m_lo = lo;
      e.m_hi = hi;
      ok = ok && e.n >= 1 && e.m_lo <= e.m_hi && lsqr_plan_valid(e.lpr, e.nch) && e.grid >= 1 &&
           e.grid <= 65535 && (e.unroll == 1 || e.unroll == 2) &&
           (e.dtype == SNS_F32 || e.dtype == SNS_F64) && (e.waves == 4 || e.waves == 8);
      if (ok) rows.push_back(e);
    }
  }
  fclose(f);
  if (!ok) return SNS_ERR_INVALID_ARG;  // nothing loaded from a malformed file
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  for (const sns_tune_entry& e : rows) put(t, e);
  for (const sns_tune_gather_entry& e : grows) put(t, e);
  for (const sns_tune_qr_entry& e : qrows) put(t, e);
  return SNS_OK;
}

sns_status sns_tune_save(const char* path) {
  if (!path) return SNS_ERR_INVALID_ARG;
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  FILE* f = fopen(path, "w");
  if (!f) return SNS_ERR_INVALID_ARG;
  fprintf(f, "# dtype n m_lo m_hi lpr nch grid unroll us waves\n");
  for (const sns_tune_entry& e : t.rows)
    fprintf(f, "%d %d %lld %lld %d %d %d %d %.3f %d\n", e.dtype, e.n, (long long)e.m_lo,
            (long long)e.m_hi, e.lpr, e.nch, e.grid, e.unroll, e.us, e.waves);
  if (!t.grows.empty()) fprintf(f, "# G dtype n d m_lo m_hi lpr nseg us\n");
  for (const sns_tune_gather_entry& e : t.grows)
    fprintf(f, "G %d %d %d %lld %lld %d %d %.3f\n", e.dtype, e.n, e.d, (long long)e.m_lo,
            (long long)e.m_hi, e.lpr, e.nseg, e.us);
  if (!t.qrows.empty()) fprintf(f, "# Q d_lo d_hi n_lo n_hi cfg cb us\n");
  for (const sns_tune_qr_entry& e : t.qrows)
    fprintf(f, "Q %d %d %d %d %d %d %.3f\n", e.d_lo, e.d_hi, e.n_lo, e.n_hi, e.cfg, e.cb, e.us);
  fclose(f);
  return SNS_OK;
}

}  // extern "C"
