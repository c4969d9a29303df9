// Autotuner of the refinement pass's launch shape and the tuning table the
// plan lookup consults.  sns_tune_pass times every valid candidate (lanes per
// row and chunks per lane that cover n without more than doubling the padded
// width, work-group counts from 64 to 4096, one or two rows per step) on the
// caller's matrix and reports the fastest.
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

}  // namespace

bool tune_lookup(sns_dtype dt, int64_t n, int64_t m, LsqrPlan* p) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  for (const sns_tune_entry& r : t.rows) {
    if (r.dtype != (int)dt || r.n != n || m < r.m_lo || m > r.m_hi) continue;
    p->lpr = r.lpr;
    p->nch = r.nch;
    p->grid = r.grid;
    p->unroll = r.unroll;
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
        for (int unroll = 1; unroll <= 2; ++unroll) {
          LsqrPlan p;
          p.lpr = lpr;
          p.nch = nch;
          p.grid = grid;
          p.unroll = unroll;
          double us = 0.0;
          s = time_lsqr_pass(*A, p, reps, workspace, ws_bytes, (hipStream_t)stream, &us);
          if (s != SNS_OK) return s;
          if (b.us < 0.0 || us < b.us) {
            b.lpr = lpr;
            b.nch = nch;
            b.grid = grid;
            b.unroll = unroll;
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

sns_status sns_tune_set(const sns_tune_entry* e) {
  if (!e || e->n < 1 || e->m_lo > e->m_hi || !lsqr_plan_valid(e->lpr, e->nch) || e->grid < 1 ||
      e->grid > 65535 || (e->unroll != 1 && e->unroll != 2) ||
      (e->dtype != SNS_F32 && e->dtype != SNS_F64))
    return SNS_ERR_INVALID_ARG;
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  put(t, *e);
  return SNS_OK;
}

sns_status sns_tune_clear(void) {
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  t.rows.clear();
  return SNS_OK;
}

sns_status sns_tune_load(const char* path) {
  if (!path) return SNS_ERR_INVALID_ARG;
  FILE* f = fopen(path, "r");
  if (!f) return SNS_ERR_INVALID_ARG;
  char line[512];
  std::vector<sns_tune_entry> rows;
  bool ok = true;
  while (fgets(line, sizeof(line), f)) {
    const char* p = line;
    while (*p == ' ' || *p == '\t') ++p;
    if (*p == '#' || *p == '\n' || *p == '\0') continue;
    sns_tune_entry e{};
    long long lo = 0, hi = 0;
    if (sscanf(p, "%d %d %lld %lld %d %d %d %d %lf", &e.dtype, &e.n, &lo, &hi, &e.lpr, &e.nch,
               &e.grid, &e.unroll, &e.us) != 9) {
      ok = false;
      break;
    }
    e.m_lo = lo;
    e.m_hi = hi;
    if (e.n < 1 || e.m_lo > e.m_hi || !lsqr_plan_valid(e.lpr, e.nch) || e.grid < 1 ||
        e.grid > 65535 || (e.unroll != 1 && e.unroll != 2) ||
        (e.dtype != SNS_F32 && e.dtype != SNS_F64)) {
      ok = false;
      break;
    }
    rows.push_back(e);
  }
  fclose(f);
  if (!ok) return SNS_ERR_INVALID_ARG;  // nothing loaded from a malformed file
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  for (const sns_tune_entry& e : rows) put(t, e);
  return SNS_OK;
}

sns_status sns_tune_save(const char* path) {
  if (!path) return SNS_ERR_INVALID_ARG;
  Table& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  FILE* f = fopen(path, "w");
  if (!f) return SNS_ERR_INVALID_ARG;
  fprintf(f, "# dtype n m_lo m_hi lpr nch grid unroll us\n");
  for (const sns_tune_entry& e : t.rows)
    fprintf(f, "%d %d %lld %lld %d %d %d %d %.3f\n", e.dtype, e.n, (long long)e.m_lo,
            (long long)e.m_hi, e.lpr, e.nch, e.grid, e.unroll, e.us);
  fclose(f);
  return SNS_OK;
}

}  // extern "C"
