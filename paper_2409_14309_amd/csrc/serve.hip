// Continuous-batching server for least-squares requests.
//
// A scheduler thread owns one HIP stream and runs rounds:
//   1. admit waiting requests in arrival order while a slot is free and the
//      request's workspace fits in the pool (first-fit allocator over the
//      caller's device memory);
//   2. set the admitted requests up on a second stream, so that the set-up
//      overlaps the iterations of step 3: the small ones (d <= 256, n <= 64,
//      m (n + 1) <= 2^21)
//      in the persistent fused sketch + QR launch, replayed from a captured
//      HIP graph whose first kernel copies this round's problem table from
//      pinned memory (two graphs, tables and images used in turn, each
//      rewritten only after its previous replay has finished); the others in
//      one batched launch per kernel (CountSketch sort and gather, blocked
//      QR); then, for refined requests, X = R^{-1} and the LSQR state.  The
//      requests join the batch in the next round, once the iteration stream
//      has waited for their set-up;
//   3. advance every refining request by `chunk_iters` LSQR iterations, again
//      one batched launch per kernel over all of them, and read back which
//      ones have stopped;
//   4. retire those (final update x = x0 + X dy and report) together with the
//      plain requests admitted this round, copy their sns_info to the host,
//      free their memory and wake any waiter.
// Requests keep their state in their own workspace, so a request that joins
// at round k simply enters the batch at its own iteration 0.  Each request's
// arithmetic depends only on its own data and plan, never on the batch.
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "solve.hpp"

namespace {

using sns::ArgTable;
using sns::Carve;

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;
constexpr size_t kTableBytesPerSlot = 4096;  // argument-table room per admitted request

// First-fit allocator over [0, cap) with coalescing of free ranges.
class PoolAlloc {
 public:
  explicit PoolAlloc(size_t cap = 0) { if (cap) free_[0] = cap; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = sns::align_up(bytes, kAlign);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = sns::align_up(bytes, kAlign);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

struct Req {
  uint64_t ticket = 0;
  sns_problem p{};
  size_t bytes = 0, off = 0;
  sns::LstsqWs w;
  sns_info* info_dev = nullptr;
  sns::LsqrProb lp{};
  bool done = false;
  sns_info info{};
  Clock::time_point t_submit, t_done;
};

// Workspace bytes of one request inside the pool.
size_t request_bytes(const sns_problem& p) {
  Carve c(nullptr, 0);
  sns::LstsqWs w;
  sns::carve_lstsq_bufs(c, p.sketch, p.A, p.opts, w);
  c.take<sns_info>(1);
  return c.off;
}

}  // namespace

struct sns_server {
  sns_serve_config cfg{};
  int device = 0;
  hipStream_t stream = nullptr;   // iterations, finishing, results
  hipStream_t stream2 = nullptr;  // set-up of admitted requests
  hipEvent_t ev = nullptr;
  hipEvent_t ev_setup = nullptr;  // the last set-up launched on stream2
  char* pool = nullptr;  // request area (after the reserved part)
  size_t usable = 0;     // bytes of the request area
  // reserved at the start of the pool
  char* tab_setup = nullptr;
  char* tab_iter = nullptr;
  char* tab_fin = nullptr;
  size_t tab_bytes = 0;
  int* flags_dev = nullptr;
  // set-up of the small requests: the fused sketch + QR launch replayed from
  // one of two graphs, each with its own device table and pinned image
  sns::FusedTableLayout ftl;
  char* ftab[2] = {nullptr, nullptr};
  void* fimg[2] = {nullptr, nullptr};
  uint64_t* fwords[2] = {nullptr, nullptr};
  hipGraphExec_t fexec[2] = {nullptr, nullptr};
  hipEvent_t fev[2] = {nullptr, nullptr};
  int fbuf = 0;
  // pinned host mirrors
  int* flags_host = nullptr;
  sns_info* infos_host = nullptr;
  PoolAlloc alloc;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, Req*> reqs;  // every request not yet collected
  int admitted = 0;

  // statistics (under mu)
  uint64_t submitted = 0, completed = 0, rounds = 0;
  std::vector<double> lat_ms;
  bool have_first = false;
  Clock::time_point t_first, t_last;
  size_t peak_pool = 0;
  int peak_slots = 0;

  std::thread worker;

  void run();
  sns_status round(std::vector<Req*>& fresh, std::vector<Req*>& pending,
                   std::vector<Req*>& refining);
  sns_status init_fused();
  void release_fused();
  void complete(std::vector<Req*>& fin, sns_status err);
};

namespace {

// One round's jobs for the freshly admitted requests.
void build_setup(ArgTable& t, sns::Jobs& J, const std::vector<Req*>& fresh, bool f64,
                 std::vector<sns::FusedArgs>& fa) {
  std::vector<sns::SortArgs> sa;
  std::vector<sns::GatherProb> ga;
  std::vector<sns::QrArgs> qa;
  std::vector<sns::LsqrProb> la;
  fa.clear();
  for (Req* r : fresh) {
    const sns_problem& q = r->p;
    const sns::LstsqWs& w = r->w;
    if (w.fused) {
      fa.push_back(sns::fused_args(w.fp, q.sketch, q.A, q.b, w.fb, w.q, w.q.xw,
                                   r->info_dev));
    } else {
      sa.push_back(sns::sort_args(w.sw.sp, q.sketch.seed, q.b, w.sw.sb));
      sns::GatherProb g;
      g.plan = w.sw.gp;
      g.args = sns::gather_args(w.sw.gp, q.A, (uint32_t)q.sketch.d, w.sw.sb, true, w.SA, w.Sb,
                                w.sw.part);
      g.dtype = q.A.dtype;
      ga.push_back(g);
      qa.push_back(sns::qr_args(q.sketch.d, q.A.n, w.SA, q.A.n, w.Sb, w.q, w.q.xw, nullptr,
                                r->info_dev));
    }
    if (q.opts.refine) la.push_back(r->lp);
  }
  J.sort = sns::build_sort_job(t, sa, f64);
  J.gather = sns::build_gather_job(t, ga);
  J.qr = sns::build_qr_job(t, qa, f64);
  J.lsqr = sns::build_lsqr_job(t, la, f64);
}

sns::LsqrJob build_lsqr(ArgTable& t, const std::vector<Req*>& rs, bool f64) {
  std::vector<sns::LsqrProb> la;
  for (Req* r : rs) la.push_back(r->lp);
  return sns::build_lsqr_job(t, la, f64);
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - (double)i;
  return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

}  // namespace

// Mark requests finished (their info already copied to infos_host in order)
// and release their memory.
void sns_server::complete(std::vector<Req*>& fin, sns_status err) {
  const auto now = Clock::now();
  std::lock_guard<std::mutex> g(mu);
  for (size_t k = 0; k < fin.size(); ++k) {
    Req* r = fin[k];
    if (err == SNS_OK) {
      r->info = infos_host[k];
    } else {
      r->info = sns_info{};
      r->info.status = err;
    }
    r->done = true;
    r->t_done = now;
    alloc.release(r->off, r->bytes);
    --admitted;
    ++completed;
    lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
    t_last = now;
  }
  fin.clear();
  cv_done.notify_all();
  cv_work.notify_all();
}

// Pinned images, events and the two set-up graphs of the fused launch.
sns_status sns_server::init_fused() {
  for (int i = 0; i < 2; ++i) {
    SNS_HIP_TRY(hipHostMalloc(&fimg[i], ftl.bytes, hipHostMallocDefault));
    SNS_HIP_TRY(hipHostMalloc((void**)&fwords[i], sizeof(uint64_t), hipHostMallocDefault));
    *fwords[i] = 0;
    SNS_HIP_TRY(hipEventCreateWithFlags(&fev[i], hipEventDisableTiming));
    sns_status s = sns::fused_graph_create(ftab[i], ftl, fimg[i], fwords[i],
                                           cfg.dtype == SNS_F64, stream2, &fexec[i]);
    if (s != SNS_OK) return s;
  }
  return SNS_OK;
}

void sns_server::release_fused() {
  for (int i = 0; i < 2; ++i) {
    if (fexec[i]) (void)hipGraphExecDestroy(fexec[i]);
    if (fev[i]) (void)hipEventDestroy(fev[i]);
    if (fimg[i]) (void)hipHostFree(fimg[i]);
    if (fwords[i]) (void)hipHostFree(fwords[i]);
    fexec[i] = nullptr;
    fev[i] = nullptr;
    fimg[i] = nullptr;
    fwords[i] = nullptr;
  }
}

sns_status sns_server::round(std::vector<Req*>& fresh, std::vector<Req*>& pending,
                             std::vector<Req*>& refining) {
  const bool f64 = cfg.dtype == SNS_F64;
  hipStream_t st = stream;
  sns_status s = SNS_OK;
  std::vector<Req*> fin;
  // -- requests set up during the previous round join (the iteration stream
  //    waits for their set-up); plain ones are finished
  if (!pending.empty()) {
    SNS_HIP_TRY(hipStreamWaitEvent(st, ev_setup, 0));
    for (Req* r : pending) {
      if (r->p.opts.refine) {
        refining.push_back(r);
      } else {
        SNS_HIP_TRY(hipMemcpyAsync(r->p.x, r->w.q.xw, sizeof(double) * r->p.A.n,
                                   hipMemcpyDeviceToDevice, st));
        fin.push_back(r);
      }
    }
    pending.clear();
  }
  // -- set-up of the admitted requests on the second stream
  if (!fresh.empty()) {
    hipStream_t s2 = stream2;
    ArgTable t(tab_setup);
    sns::Jobs J;
    std::vector<sns::FusedArgs> fa;
    build_setup(t, J, fresh, f64, fa);
    if (t.bytes() > tab_bytes) return SNS_ERR_OUT_OF_MEMORY;
    if (!fa.empty()) {
      // the image of this buffer is free once its previous replay has run
      const int bi = fbuf;
      fbuf ^= 1;
      SNS_HIP_TRY(hipEventSynchronize(fev[bi]));
      if (!sns::fused_table_fill(fimg[bi], ftl, fa, fwords[bi])) return SNS_ERR_OUT_OF_MEMORY;
      sns::region_begin("fused", s2);
      SNS_HIP_TRY(hipGraphLaunch(fexec[bi], s2));
      sns::region_end(s2);
      SNS_HIP_TRY(hipEventRecord(fev[bi], s2));
    }
    if ((s = t.upload(s2)) != SNS_OK) return s;
    if ((s = sns::run_sketch_jobs(J, s2)) != SNS_OK) return s;
    if ((s = sns::launch_qr_job(J.qr, s2)) != SNS_OK) return s;
    if ((s = sns::launch_lsqr_setup(J.lsqr, s2)) != SNS_OK) return s;
    SNS_HIP_TRY(hipEventRecord(ev_setup, s2));
    pending.swap(fresh);
    fresh.clear();
  }
  // -- one chunk of iterations for every refining request
  if (!refining.empty()) {
    ArgTable t(tab_iter);
    const sns::LsqrJob j = build_lsqr(t, refining, f64);
    if (t.bytes() > tab_bytes) return SNS_ERR_OUT_OF_MEMORY;
    if ((s = t.upload(st)) != SNS_OK) return s;
    for (int k = 0; k < cfg.chunk_iters; ++k)
      if ((s = sns::launch_lsqr_iteration(j, st)) != SNS_OK) return s;
    if ((s = sns::launch_lsqr_flags(j, flags_dev, st)) != SNS_OK) return s;
    SNS_HIP_TRY(hipMemcpyAsync(flags_host, flags_dev, sizeof(int) * refining.size(),
                               hipMemcpyDeviceToHost, st));
    SNS_HIP_TRY(hipEventRecord(ev, st));
    SNS_HIP_TRY(hipEventSynchronize(ev));
    std::vector<Req*> keep, stopped;
    for (size_t k = 0; k < refining.size(); ++k)
      (flags_host[k] ? stopped : keep).push_back(refining[k]);
    refining.swap(keep);
    if (!stopped.empty()) {
      ArgTable tf(tab_fin);
      const sns::LsqrJob jf = build_lsqr(tf, stopped, f64);
      if (tf.bytes() > tab_bytes) return SNS_ERR_OUT_OF_MEMORY;
      if ((s = tf.upload(st)) != SNS_OK) return s;
      if ((s = sns::launch_lsqr_finish(jf, st)) != SNS_OK) return s;
      fin.insert(fin.end(), stopped.begin(), stopped.end());
    }
  }
  // -- results of the finished requests
  if (!fin.empty()) {
    for (size_t k = 0; k < fin.size(); ++k)
      SNS_HIP_TRY(hipMemcpyAsync(&infos_host[k], fin[k]->info_dev, sizeof(sns_info),
                                 hipMemcpyDeviceToHost, st));
    SNS_HIP_TRY(hipEventRecord(ev, st));
    SNS_HIP_TRY(hipEventSynchronize(ev));
    complete(fin, SNS_OK);
  }
  return SNS_OK;
}

void sns_server::run() {
  (void)hipSetDevice(device);
  std::vector<Req*> refining, pending;
  for (;;) {
    std::vector<Req*> fresh;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] {
        return stop || !queue.empty() || !refining.empty() || !pending.empty();
      });
      if (stop && queue.empty() && refining.empty() && pending.empty()) break;
      // admission in arrival order by slot and by workspace footprint
      while (!queue.empty() && admitted < cfg.max_slots) {
        Req* r = queue.front();
        size_t off = 0;
        if (!alloc.alloc(r->bytes, &off)) break;
        r->off = off;
        queue.pop_front();
        fresh.push_back(r);
        ++admitted;
      }
      peak_slots = std::max(peak_slots, admitted);
      peak_pool = std::max(peak_pool, alloc.used());
      ++rounds;
    }
    for (Req* r : fresh) {
      Carve c(pool + r->off, r->bytes);
      sns::carve_lstsq_bufs(c, r->p.sketch, r->p.A, r->p.opts, r->w);
      r->info_dev = c.take<sns_info>(1);
      if (r->p.opts.refine) {
        r->lp.plan = r->w.lp;
        r->lp.args = sns::lsqr_args(r->p.A, r->p.b, r->w.lp, r->w.l, r->w.q,
                                    (int)r->p.sketch.d, r->p.opts.max_iters, r->p.opts.rtol,
                                    r->p.x, r->info_dev);
      }
    }
    if (fresh.empty() && refining.empty() && pending.empty()) {
      // nothing admissible now (the head waits for memory held by nobody
      // cannot happen: requests larger than the pool are refused at submit)
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait_for(lk, std::chrono::milliseconds(1));
      continue;
    }
    std::vector<Req*> all_inflight = refining;
    all_inflight.insert(all_inflight.end(), pending.begin(), pending.end());
    all_inflight.insert(all_inflight.end(), fresh.begin(), fresh.end());
    const sns_status s = round(fresh, pending, refining);
    if (s != SNS_OK) {
      // fail everything in flight and keep serving the queue
      (void)hipStreamSynchronize(stream2);
      (void)hipStreamSynchronize(stream);
      std::vector<Req*> fin;
      for (Req* r : all_inflight)
        if (!r->done) fin.push_back(r);
      refining.clear();
      pending.clear();
      complete(fin, s);
    }
  }
}

extern "C" {

sns_status sns_serve_create(const sns_serve_config* cfg, sns_server** out) {
  if (!cfg || !out || !cfg->pool) return SNS_ERR_INVALID_ARG;
  if (cfg->max_slots < 1 || cfg->max_slots > 4096 || cfg->queue_capacity < 1 ||
      cfg->chunk_iters < 1 || (cfg->dtype != SNS_F32 && cfg->dtype != SNS_F64))
    return SNS_ERR_INVALID_ARG;
  sns_server* s = new sns_server();
  s->cfg = *cfg;
  s->pool = static_cast<char*>(cfg->pool);
  // reserved tables and flags at the start of the pool
  s->tab_bytes = (size_t)cfg->max_slots * kTableBytesPerSlot + 16384;
  Carve c(cfg->pool, cfg->pool_bytes);
  s->tab_setup = c.take<char>(s->tab_bytes);
  s->tab_iter = c.take<char>(s->tab_bytes);
  s->tab_fin = c.take<char>(s->tab_bytes);
  s->flags_dev = c.take<int>((size_t)cfg->max_slots);
  s->ftl = sns::fused_table_layout(cfg->max_slots);
  for (int i = 0; i < 2; ++i) s->ftab[i] = c.take<char>(s->ftl.bytes);
  c.off = sns::align_up(c.off);
  if (!c.ok() || c.off >= cfg->pool_bytes) {
    delete s;
    return SNS_ERR_OUT_OF_MEMORY;
  }
  const size_t reserved = c.off;
  s->pool += reserved;
  s->usable = cfg->pool_bytes - reserved;
  s->alloc = PoolAlloc(s->usable);
  if (hipGetDevice(&s->device) != hipSuccess ||
      hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->stream2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev_setup, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void**)&s->flags_host, sizeof(int) * cfg->max_slots, hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&s->infos_host, sizeof(sns_info) * cfg->max_slots,
                    hipHostMallocDefault) != hipSuccess) {
    if (s->flags_host) (void)hipHostFree(s->flags_host);
    if (s->infos_host) (void)hipHostFree(s->infos_host);
    if (s->ev_setup) (void)hipEventDestroy(s->ev_setup);
    if (s->ev) (void)hipEventDestroy(s->ev);
    if (s->stream2) (void)hipStreamDestroy(s->stream2);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return SNS_ERR_HIP;
  }
  if (s->init_fused() != SNS_OK) {
    s->release_fused();
    (void)hipHostFree(s->flags_host);
    (void)hipHostFree(s->infos_host);
    (void)hipEventDestroy(s->ev_setup);
    (void)hipEventDestroy(s->ev);
    (void)hipStreamDestroy(s->stream2);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return SNS_ERR_HIP;
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return SNS_OK;
}

sns_status sns_serve_submit(sns_server* srv, const sns_problem* req, uint64_t* ticket) {
  if (!srv || !req || !ticket) return SNS_ERR_INVALID_ARG;
  sns_status s = sns::check_batch(req, 1);
  if (s != SNS_OK) return s;
  if (req->A.dtype != srv->cfg.dtype) return SNS_ERR_DTYPE;
  if (!req->b || !req->x) return SNS_ERR_INVALID_ARG;
  Req* r = new Req();
  r->p = *req;
  r->bytes = sns::align_up(request_bytes(*req), kAlign);
  if (r->bytes > srv->usable) {  // could never be admitted
    delete r;
    return SNS_ERR_OUT_OF_MEMORY;
  }
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if ((int)srv->queue.size() >= srv->cfg.queue_capacity) {
      delete r;
      return SNS_ERR_QUEUE_FULL;
    }
    r->ticket = srv->next_ticket++;
    r->t_submit = Clock::now();
    if (!srv->have_first) {
      srv->have_first = true;
      srv->t_first = r->t_submit;
    }
    ++srv->submitted;
    srv->queue.push_back(r);
    srv->reqs[r->ticket] = r;
    *ticket = r->ticket;
  }
  srv->cv_work.notify_all();
  return SNS_OK;
}

static sns_status collect(sns_server* srv, uint64_t ticket, sns_info* out, bool wait) {
  if (!srv) return SNS_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return SNS_ERR_INVALID_ARG;
  Req* r = it->second;
  if (wait) srv->cv_done.wait(lk, [&] { return r->done; });
  if (!r->done) return SNS_ERR_NOT_READY;
  if (out) *out = r->info;
  srv->reqs.erase(it);
  delete r;
  return SNS_OK;
}

sns_status sns_serve_poll(sns_server* srv, uint64_t ticket, sns_info* out) {
  return collect(srv, ticket, out, false);
}

sns_status sns_serve_wait(sns_server* srv, uint64_t ticket, sns_info* out) {
  return collect(srv, ticket, out, true);
}

sns_status sns_serve_stats_get(sns_server* srv, sns_serve_stats* out) {
  if (!srv || !out) return SNS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(srv->mu);
  sns_serve_stats s{};
  s.submitted = srv->submitted;
  s.completed = srv->completed;
  s.p50_ms = percentile(srv->lat_ms, 0.50);
  s.p99_ms = percentile(srv->lat_ms, 0.99);
  double sum = 0.0;
  for (double v : srv->lat_ms) sum += v;
  s.mean_ms = srv->lat_ms.empty() ? 0.0 : sum / (double)srv->lat_ms.size();
  s.span_s = srv->completed ? std::chrono::duration<double>(srv->t_last - srv->t_first).count()
                            : 0.0;
  s.peak_pool_bytes = srv->peak_pool;
  s.peak_slots = srv->peak_slots;
  s.rounds = srv->rounds;
  *out = s;
  return SNS_OK;
}

sns_status sns_serve_destroy(sns_server* srv) {
  if (!srv) return SNS_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  for (auto& kv : srv->reqs) delete kv.second;
  srv->reqs.clear();
  (void)hipStreamSynchronize(srv->stream2);
  (void)hipStreamSynchronize(srv->stream);
  srv->release_fused();
  (void)hipHostFree(srv->flags_host);
  (void)hipHostFree(srv->infos_host);
  (void)hipEventDestroy(srv->ev_setup);
  (void)hipEventDestroy(srv->ev);
  (void)hipStreamDestroy(srv->stream2);
  (void)hipStreamDestroy(srv->stream);
  delete srv;
  return SNS_OK;
}

}  // extern "C"
