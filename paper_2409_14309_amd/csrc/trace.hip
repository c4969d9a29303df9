// Per-kernel timing: when enabled, every launch of the library (or of the
// kernels named by sns_timing_select) is bracketed by two HIP events recorded
// on the launch stream.  Durations are read back on demand
// (sns_timing_summary) and summed per kernel name.  Enabled by
// sns_timing_enable(1) or by the environment variable SNS_TRACE=1, which also
// prints the summary to stderr when the process exits.  Each bracketed launch
// costs a few microseconds of device time for the two event records, so a
// caller timing a whole solve selects only the kernels it reports.  A region
// (region_begin / region_end around a phase of several launches, e.g. the
// whole QR) is timed the same way under its own name.
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
// a region (a phase of several launches) is timed in a slot of its own, so a
// kernel inside it can be timed too
thread_local Rec* t_region_open = nullptr;
thread_local Rec t_region;

bool selected(const Registry& r, const char* name) {
  if (r.only.empty()) return true;
  for (const std::string& k : r.only)
    if (k == name) return true;
  return false;
}

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
  if (!r.on || !selected(r, name)) return;
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

void region_begin(const char* name, hipStream_t s) {
  Registry& r = reg();
  std::lock_guard<std::mutex> g(r.mu);
  check_env(r);
  if (!r.on || !selected(r, name)) return;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
  t_region.name = name;
  t_region.a = take_event(r);
  t_region.b = take_event(r);
  if (!t_region.a || !t_region.b) return;
  (void)hipEventRecord(t_region.a, s);
  t_region_open = &t_region;
}

void region_end(hipStream_t s) {
  if (!t_region_open) return;
  Registry& r = reg();
  std::lock_guard<std::mutex> g(r.mu);
  (void)hipEventRecord(t_region_open->b, s);
  r.recs.push_back(*t_region_open);
  t_region_open = nullptr;
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
