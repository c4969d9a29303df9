// Per-kernel timing: when enabled, every launch of the library (or of the
// kernels named by sns_timing_select) is bracketed by two HIP events recorded
// on the launch stream.  Durations are read back on demand
// (sns_timing_summary) and summed per kernel name.  Enabled by
// sns_timing_enable(1) or by the environment variable SNS_TRACE=1, which also
// prints the summary to stderr when the process exits.  Each bracketed launch
// costs a few microseconds of device time for the two event records, so a
// caller timing a whole solve selects only the kernels it reports.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace sns {

namespace {

struct Rec {
  const char* name;
  hipEvent_t a, b;
};

struct Registry {
  std::mutex mu;
  bool on = false;
  bool env_checked = false;
  std::vector<hipEvent_t> pool;  // free events
  std::vector<Rec> recs;
  std::map<std::string, std::pair<double, long long>> done;  // name -> (ms, launches)
  std::vector<std::string> only;  // kernels to time; empty: all
};

Registry& reg() {
  static Registry r;
  return r;
}

thread_local Rec* t_open = nullptr;
thread_local Rec t_pending;

hipEvent_t take_event(Registry& r) {
  if (!r.pool.empty()) {
    hipEvent_t e = r.pool.back();
    r.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Fold finished records into the per-name totals (waits for them).
void collect(Registry& r) {
  for (Rec& x : r.recs) {
    float ms = 0.f;
    if (hipEventSynchronize(x.b) == hipSuccess && hipEventElapsedTime(&ms, x.a, x.b) == hipSuccess) {
      auto& slot = r.done[x.name];
      slot.first += ms;
      slot.second += 1;
    }
    r.pool.push_back(x.a);
    r.pool.push_back(x.b);
  }
  r.recs.clear();
}

void print_at_exit() {
  char buf[8192];
  sns_timing_summary(buf, sizeof(buf));
  fputs(buf, stderr);
}

void check_env(Registry& r) {
  if (r.env_checked) return;
  r.env_checked = true;
  const char* v = getenv("SNS_TRACE");
  if (v && v[0] == '1') {
    r.on = true;
    atexit(print_at_exit);
  }
}

}  // namespace

void report_hip_error(hipError_t e, const char* what, const char* file, int line) {
  static const bool on = [] {
    const char* v = getenv("SNS_DEBUG");
    return v && v[0] == '1';
  }();
  if (on) fprintf(stderr, "libsns: %s failed: %s (%s:%d)\n", what, hipGetErrorString(e), file, line);
}

void timing_begin(const char* name, hipStream_t s) {
  Registry& r = reg();
  std::lock_guard<std::mutex> g(r.mu);
  check_env(r);
  if (!r.on) return;
  if (!r.only.empty()) {
    bool hit = false;
    for (const std::string& k : r.only) hit = hit || k == name;
    if (!hit) return;
  }
  // launches being captured into a graph are not timed
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
  t_pending.name = name;
  t_pending.a = take_event(r);
  t_pending.b = take_event(r);
  if (!t_pending.a || !t_pending.b) return;
  (void)hipEventRecord(t_pending.a, s);
  t_open = &t_pending;
}

void timing_end(hipStream_t s) {
  if (!t_open) return;
  Registry& r = reg();
  std::lock_guard<std::mutex> g(r.mu);
  (void)hipEventRecord(t_open->b, s);
  r.recs.push_back(*t_open);
  t_open = nullptr;
  if (r.recs.size() > 4096) collect(r);
}

}  // namespace sns

extern "C" {

void sns_timing_enable(int on) {
  sns::Registry& r = sns::reg();
  std::lock_guard<std::mutex> g(r.mu);
  sns::check_env(r);
  r.on = on != 0;
}

void sns_timing_select(const char* names) {
  sns::Registry& r = sns::reg();
  std::lock_guard<std::mutex> g(r.mu);
  r.only.clear();
  if (!names) return;
  std::string cur;
  for (const char* c = names;; ++c) {
    if (*c == ',' || *c == '\0') {
      if (!cur.empty()) r.only.push_back(cur);
      cur.clear();
      if (*c == '\0') break;
    } else {
      cur += *c;
    }
  }
}

void sns_timing_reset(void) {
  sns::Registry& r = sns::reg();
  std::lock_guard<std::mutex> g(r.mu);
  sns::collect(r);
  r.done.clear();
}

int sns_timing_summary(char* buf, size_t len) {
  sns::Registry& r = sns::reg();
  std::lock_guard<std::mutex> g(r.mu);
  sns::collect(r);
  std::string out = "# kernel launches total_ms avg_us\n";
  char line[256];
  for (auto& kv : r.done) {
    snprintf(line, sizeof(line), "%s %lld %.6f %.3f\n", kv.first.c_str(), kv.second.second,
             kv.second.first, 1000.0 * kv.second.first / (double)(kv.second.second ? kv.second.second : 1));
    out += line;
  }
  if (buf && len) {
    strncpy(buf, out.c_str(), len - 1);
    buf[len - 1] = '\0';
  }
  return (int)out.size();
}

}  // extern "C"

// ------------------------------------------------------- bandwidth probe ----
// The practical ceiling of the HBM-bound kernels: one streaming read of a
// device buffer, grid-stride over 16-byte vectors with U loads in flight per
// thread, plain or nontemporal.  The sum is stored only when it equals a
// value no finite input of this size reaches, so the loads stay live without
// a store per work-group.
namespace sns {
namespace {

template <int U, bool NT>
__global__ void k_read_probe(const float* __restrict__ a, size_t nvec, float* __restrict__ out) {
  typedef float F4 __attribute__((ext_vector_type(4)));
  const F4* __restrict__ p = reinterpret_cast<const F4*>(a);
  F4 acc = {0.f, 0.f, 0.f, 0.f};
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < nvec; i += U * stride) {
    F4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = NT ? __builtin_nontemporal_load(p + i + u * stride) : p[i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u];
  }
  for (; i < nvec; i += stride) acc += NT ? __builtin_nontemporal_load(p + i) : p[i];
  const float s = (acc.x + acc.y) + (acc.z + acc.w);
  if (s == -3.0e38f) out[blockIdx.x] = s;
}

template <int U, bool NT>
void launch_read_probe(const float* a, size_t nvec, int groups, int threads, float* out,
                       hipStream_t st) {
  SNS_LAUNCH("read_probe", (k_read_probe<U, NT>), dim3(groups), dim3(threads), 0, st, a, nvec, out);
}

}  // namespace
}  // namespace sns

extern "C" sns_status sns_read_probe(const void* buf, size_t bytes, int groups, int threads,
                                     int unroll, int nontemporal, float* out, void* stream) {
  if (!buf || !out) return SNS_ERR_INVALID_ARG;
  if (groups < 1 || groups > 65536 || (threads != 256 && threads != 512 && threads != 1024) ||
      (unroll != 1 && unroll != 4))
    return SNS_ERR_INVALID_ARG;
  if (bytes % 16 != 0 || reinterpret_cast<uintptr_t>(buf) % 16 != 0) return SNS_ERR_SHAPE;
  if (bytes == 0) return SNS_OK;
  const float* a = static_cast<const float*>(buf);
  const size_t nvec = bytes / 16;
  hipStream_t st = (hipStream_t)stream;
  if (unroll == 4) {
    if (nontemporal) sns::launch_read_probe<4, true>(a, nvec, groups, threads, out, st);
    else sns::launch_read_probe<4, false>(a, nvec, groups, threads, out, st);
  } else {
    if (nontemporal) sns::launch_read_probe<1, true>(a, nvec, groups, threads, out, st);
    else sns::launch_read_probe<1, false>(a, nvec, groups, threads, out, st);
  }
  SNS_HIP_TRY(hipGetLastError());
  return SNS_OK;
}
