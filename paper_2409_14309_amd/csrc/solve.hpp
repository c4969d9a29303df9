// Host-side pieces shared by the C ABI (api.hip) and the server
// (serve.hip): limits, argument checks, the workspace layout of one problem
// and the launch sequences built from it (solve.hip).
#pragma once

#include <vector>

#include "kernels.hpp"

namespace sns {

constexpr int64_t kMaxRows = (int64_t(1) << 31) - 1;  // row ids fit 31 bits
constexpr int64_t kMaxD = 16384;      // CountSketch bucket sort (LDS histograms)
constexpr int64_t kMaxQrD = 8192;     // register-resident QR panels
constexpr int64_t kMaxCsrN = 4096;    // CSR sketch: one output row per wave in LDS
constexpr int64_t kMaxHadRows = int64_t(1) << 26;  // SRHT: work buffers of m' = 2^L padded rows

sns_status check_matrix(const sns_matrix* A);
sns_status check_sketch(const sns_sketch* sk, const sns_matrix* A);
sns_status check_solve(const sns_sketch& sk, const sns_matrix& A, const sns_solve_opts& o);
sns_status check_batch(const sns_problem* P, int count);
sns_solve_opts default_opts();
inline size_t elem(const sns_matrix& A) { return A.dtype == SNS_F64 ? 8 : 4; }

// Workspace of the dense CountSketch step (sort + partials).
struct SketchWs {
  SortPlan sp;
  GatherPlan gp;
  SortBufs sb{};
  void* part = nullptr;
};

void carve_sketch(Carve& c, const sns_sketch& sk, const sns_matrix& A, bool with_b, bool acc64,
                  SketchWs& w);

// The launch sequences of one call, built into one argument table.
struct Jobs {
  SortJob sort;
  std::vector<GatherLaunch> gather;
  QrJob qr;
  FusedJob fused;  // sketch + QR of the small problems, one persistent launch
  LsqrJob lsqr;
};

void add_sketch_jobs(ArgTable& t, Jobs& J, const sns_sketch& sk, const sns_matrix& A,
                     const void* b, void* SA, void* Sb, const SketchWs& w);
sns_status run_sketch_jobs(const Jobs& J, hipStream_t st);

// Argument-table bytes of a builder: a dry run against a table without a
// device location (only sizes matter, so null pointers are fine).
template <typename F>
size_t table_bytes(F&& build) {
  ArgTable t(nullptr);
  Jobs J;
  build(t, J);
  return t.bytes();
}

struct LstsqWs {
  bool fused = false;  // sketch and QR in the persistent fused launch
  FusedPlan fp;
  FusedBufs fb;
  SketchWs sw;
  void* gauss = nullptr;  // Gaussian sketch partials or the Hadamard sketch's blocks
  void* csr = nullptr;    // CSR sketch workspace
  size_t csr_bytes = 0;
  void* SA = nullptr;
  void* Sb = nullptr;
  QrBufs q{};
  LsqrPlan lp;
  LsqrBufs l{};
  void* Y = nullptr;  // SAA-SAS: A R^{-1}, m rows of stride ldy in A's dtype
  int64_t ldy = 0;
  sns_info* info = nullptr;
  char* args = nullptr;
};

// Buffers of one problem (no argument table).
void carve_lstsq_bufs(Carve& c, const sns_sketch& sk, const sns_matrix& A,
                      const sns_solve_opts& o, LstsqWs& w);
void build_lstsq_jobs(ArgTable& t, Jobs& J, const sns_sketch& sk, const sns_matrix& A,
                      const void* b, double* x, const sns_solve_opts& o, const LstsqWs& w);
// Full workspace layout of sns_lstsq: buffers, then the argument table.
void carve_lstsq(Carve& c, const sns_sketch& sk, const sns_matrix& A, const sns_solve_opts& o,
                 LstsqWs& w);

// ------------------------------------------------------------- batches ----
// Per-problem buffers of a batch; the argument table and the shared scalars
// follow them.
struct BatchWs {
  std::vector<LstsqWs> w;
  sns_info* infos = nullptr;  // count entries, contiguous
  int* active = nullptr;      // problems still refining
  char* args = nullptr;
};

void build_batch_jobs(ArgTable& t, Jobs& J, const sns_problem* P, int count, const BatchWs& B,
                      bool real);
void carve_batch(Carve& c, const sns_problem* P, int count, BatchWs& B);
// Refinement of a batch: setup, chunks of iterations until no problem is
// left running (read back between chunks), final update and report.
sns_status run_batch_lsqr(const LsqrJob& j, int max_iters, int* active_dev, bool use_graph,
                          hipStream_t st);

}  // namespace sns
