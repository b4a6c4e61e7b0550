// nls_serve.cpp -- the request server behind the nls_server_* entry points.
//
// Clients queue host-memory requests; one scheduler thread per server
//   * reaps finished launches (event query), copies their results from the
//     pinned mirror into the callers' arrays and releases their arena space;
//   * admits the longest first-come-first-served prefix of the queue whose
//     launches fit the device arena (requests with the same kernel and
//     settings admitted together share one launch), stages their inputs in
//     the pinned mirror and enqueues, on the least-loaded stream: one
//     host-to-device copy of the inputs, the work-counter reset, the
//     persistent solver launch and one device-to-host copy of the outputs,
//     then an event.
// Launches whose inputs or results take more than a few MiB of host copies
// hand those copies, split by systems, to a small pool of copy threads, so
// that one large request does not hold up the reaping and admission of the
// others while its megabytes move; the launch is enqueued once its inputs
// are staged, and completed once its results are in the callers' arrays.
// Everything the device touches lives in the arena (allocated once at
// creation), so admission and completion never call hipMalloc or hipFree.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <list>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "nls.h"
#include "nls_launch.h"
#include "nls_runtime.h"
#include "nls_serve_core.hpp"

using namespace nls;
using namespace nls::rt;
using namespace nls::serve;

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  uint64_t id = 0;
  nls_batch b{};          // the caller's descriptor; its arrays stay caller-owned
  nls_alg_options opts{};
  nls_results r{};
  int fam = 0, n = 1, alg = 0, P = 0;
  int64_t M = 0;
  std::string key;
  double t_submit = 0.0, t_admit = 0.0;
};

enum Phase { PH_STAGING, PH_DEVICE, PH_SCATTER };

struct InFlight {
  PlannedLaunch plan;
  std::vector<Req> reqs;  // in the order of plan.reqs
  hipEvent_t ev = nullptr;
  int stream = 0;
  int counter = 0;
  int32_t status = NLS_OK;
  Phase phase = PH_DEVICE;
  // copy jobs of the current phase not yet finished (copy threads decrement)
  std::shared_ptr<std::atomic<int>> pending = std::make_shared<std::atomic<int>>(0);
};

// host copies of a launch above this size go to the copy threads, in jobs of
// about kCopyJobBytes each (NLS_SERVE_INLINE_COPY_BYTES and
// NLS_SERVE_COPY_JOB_BYTES, read at creation, override them)
constexpr size_t kInlineCopyBytes = size_t(4) << 20;
constexpr size_t kCopyJobBytes = size_t(16) << 20;
constexpr int kCopyThreads = 4;

}  // namespace

struct nls_server {
  int device = 0;
  int nstreams = 4;
  int max_inflight = 256;
  int max_admit = 256;
  double slice_work = 0.0;  // no slicing unless NLS_SERVE_SLICE_WORK > 0
  size_t inline_copy_bytes = kInlineCopyBytes;
  size_t copy_job_bytes = kCopyJobBytes;
  std::vector<hipStream_t> streams;
  std::vector<double> load;  // estimated outstanding work per stream
  char* dev = nullptr;       // device arena
  char* host = nullptr;      // pinned host mirror (same offsets)
  Arena arena;
  int64_t* counters = nullptr;
  std::vector<int> free_counters;
  std::vector<hipEvent_t> free_events;
  Clock::time_point t0;
  std::list<InFlight> inflight;  // scheduler thread only
  std::thread th;

  // copy threads and their job queue, under cmu
  std::vector<std::thread> copiers;
  std::mutex cmu;
  std::condition_variable ccv;
  std::deque<std::function<void()>> cjobs;
  bool cstop = false;

  // shared with client threads, under mu
  std::mutex mu;
  std::condition_variable cv_work;
  std::condition_variable cv_done;
  std::deque<Req> queue;
  std::deque<nls_request_info> done;
  bool stop = false;
  uint64_t next_id = 1;
  int64_t outstanding = 0;  // submitted, not yet in `done`
  nls_server_stats st{};

  double now_ms() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }
};

namespace {

int sfail(int code, const std::string& m) {
  set_thread_error(m);
  return code;
}

// bytes of the per-request merge key: requests with equal keys run the same
// kernel with the same settings and may share a launch
std::string merge_key(const Req& q) {
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append((const char*)p, n); };
  const int32_t v[5] = {q.fam, q.n, q.alg, (int32_t)q.b.precision, q.b.maxiters};
  put(v, sizeof v);
  put(&q.b.abstol, sizeof q.b.abstol);
  put(&q.opts, sizeof q.opts);
  return k;
}

// copy systems [i0, i1) of a request's inputs into the pinned mirror of its
// launch region
void stage_inputs(nls_server* s, const InFlight& L, const Req& q, int64_t first, int64_t i0, int64_t i1) {
  char* base = s->host + L.plan.offset;
  double* P = (double*)(base + L.plan.layout.params) + first * q.P;
  double* U = (double*)(base + L.plan.layout.u0) + first * q.n;
  if (q.P > 0) {
    if (!q.b.p_offset) std::memcpy(P + i0 * q.P, q.b.params + i0 * q.P, sizeof(double) * (i1 - i0) * q.P);
    else
      for (int64_t i = i0; i < i1; ++i) std::memcpy(P + i * q.P, q.b.params + q.b.p_offset[i], sizeof(double) * q.P);
  }
  if (!q.b.u_offset) std::memcpy(U + i0 * q.n, q.b.u0 + i0 * q.n, sizeof(double) * (i1 - i0) * q.n);
  else
    for (int64_t i = i0; i < i1; ++i) std::memcpy(U + i * q.n, q.b.u0 + q.b.u_offset[i], sizeof(double) * q.n);
}

// copy systems [i0, i1) of a request's outputs from the pinned mirror into
// the caller's arrays
void scatter_results(nls_server* s, const InFlight& L, const Req& q, int64_t first, int64_t i0, int64_t i1) {
  const char* base = s->host + L.plan.offset;
  const Region& g = L.plan.layout;
  const double* u = (const double*)(base + g.u) + first * q.n;
  const int64_t k = i1 - i0;
  if (!q.b.u_offset) std::memcpy(q.r.u + i0 * q.n, u + i0 * q.n, sizeof(double) * k * q.n);
  else
    for (int64_t i = i0; i < i1; ++i) std::memcpy(q.r.u + q.b.u_offset[i], u + i * q.n, sizeof(double) * q.n);
  first += i0;
  std::memcpy(q.r.fnorm_inf + i0, (const double*)(base + g.fnorm) + first, sizeof(double) * k);
  std::memcpy(q.r.iters + i0, (const int32_t*)(base + g.iters) + first, sizeof(int32_t) * k);
  std::memcpy(q.r.retcode + i0, (const int32_t*)(base + g.retcode) + first, sizeof(int32_t) * k);
  if (q.r.nfev) std::memcpy(q.r.nfev + i0, (const int32_t*)(base + g.nfev) + first, sizeof(int32_t) * k);
  if (q.r.njev) std::memcpy(q.r.njev + i0, (const int32_t*)(base + g.njev) + first, sizeof(int32_t) * k);
}

size_t input_bytes_per_system(const Req& q) { return sizeof(double) * (size_t)(q.P + q.n); }
size_t result_bytes_per_system(const Req& q) { return sizeof(double) * (size_t)(q.n + 1) + 4 * sizeof(int32_t); }

// run copy(L, q, first, i0, i1) over every request of launch L: inline when
// the launch's bytes are few, else as jobs of the copy threads (L.pending
// counts them down; the scheduler polls it).  Returns true if done inline.
template <typename Copy>
bool run_copies(nls_server* s, InFlight& L, size_t (*bytes_per_system)(const Req&), Copy copy) {
  size_t total = 0;
  for (const Req& q : L.reqs) total += bytes_per_system(q) * (size_t)q.M;
  if (total <= s->inline_copy_bytes || s->copiers.empty()) {
    for (size_t j = 0; j < L.reqs.size(); ++j) copy(s, L, L.reqs[j], L.plan.first[j], int64_t(0), L.reqs[j].M);
    return true;
  }
  std::vector<std::function<void()>> jobs;
  for (size_t j = 0; j < L.reqs.size(); ++j) {
    const Req& q = L.reqs[j];
    const int64_t first = L.plan.first[j];
    for (const auto& rg : copy_ranges(q.M, bytes_per_system(q), s->copy_job_bytes)) {
      const int64_t i0 = rg.first, i1 = rg.second;
      InFlight* lp = &L;
      const Req* qp = &q;
      jobs.push_back([s, lp, qp, first, i0, i1, copy] {
        copy(s, *lp, *qp, first, i0, i1);
        if (lp->pending->fetch_sub(1) == 1) {
          // the last job of the phase: wake the scheduler
          std::lock_guard<std::mutex> lk(s->mu);
          s->cv_work.notify_all();
        }
      });
    }
  }
  L.pending->store((int)jobs.size());
  {
    std::lock_guard<std::mutex> lk(s->cmu);
    for (auto& f : jobs) s->cjobs.push_back(std::move(f));
  }
  s->ccv.notify_all();
  return false;
}

void copier(nls_server* s) {
  while (true) {
    std::function<void()> job;
    {
      std::unique_lock<std::mutex> lk(s->cmu);
      s->ccv.wait(lk, [&] { return s->cstop || !s->cjobs.empty(); });
      if (s->cjobs.empty()) return;  // stopping, nothing left
      job = std::move(s->cjobs.front());
      s->cjobs.pop_front();
    }
    job();
  }
}

// enqueue one launch: inputs in, counter reset, solve, outputs out, event
int32_t enqueue(nls_server* s, InFlight& L) {
  const Req& q0 = L.reqs.front();
  const Region& g = L.plan.layout;
  hipStream_t st = s->streams[L.stream];
  char* d = s->dev + L.plan.offset;
  char* h = s->host + L.plan.offset;
  hipError_t e = hipMemcpyAsync(d, h, g.in_bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return NLS_E_DEVICE;
  const Mapping mp = fixed_mapping(q0.n);
  const bool chain = q0.alg == ALG_POLY;
  // (the chain's later stages need the whole launch in one Newton stage)
  const int64_t step = chain ? std::max<int64_t>(L.plan.m, 1) : slice_systems(q0.n, s->slice_work);
  for (int64_t s0 = 0; s0 < L.plan.m; s0 += step) {
    // one slice: systems s0 .. s0 + cnt - 1 of the launch (its own counter
    // reset; slices on one stream run one after the other)
    const int64_t cnt = std::min<int64_t>(step, L.plan.m - s0);
    if (launch_zero_counters(s->counters + L.counter, 1, st) != 0) return NLS_E_DEVICE;
    KArgs a{};
    a.params = (const double*)(d + g.params) + s0 * q0.P;
    a.u0 = (const double*)(d + g.u0) + s0 * q0.n;
    a.u_out = (double*)(d + g.u) + s0 * q0.n;
    a.fnorm = (double*)(d + g.fnorm) + s0;
    a.iters = (int32_t*)(d + g.iters) + s0;
    a.retcode = (int32_t*)(d + g.retcode) + s0;
    a.nfev = (int32_t*)(d + g.nfev) + s0;
    a.njev = (int32_t*)(d + g.njev) + s0;
    a.counter = s->counters + L.counter;
    a.count = cnt;
    a.P = q0.P;
    a.n = q0.n;
    a.maxiters = q0.b.maxiters;
    a.abstol = q0.b.abstol;
    a.o = to_kopts(q0.opts);
    if (s->streams.size() > 1 && launch_work(L.plan.m, q0.n) > kExpressWork) a.grid_pct = kLargeGridPct;
    if (launch(mp.key_n, mp.lane, q0.fam, chain ? ALG_NEWTON : q0.alg, q0.b.precision, a, st) != 0)
      return NLS_E_DEVICE;
    if (chain) {
      ChainScratch sc{(int32_t*)(d + g.sel1),   (int32_t*)(d + g.sel2),    (int64_t*)(d + g.cnt),
                      (double*)(d + g.u_t),     (double*)(d + g.fnorm_t),  (int32_t*)(d + g.iters_t),
                      (int32_t*)(d + g.retcode_t), (int32_t*)(d + g.nfev_t), (int32_t*)(d + g.njev_t)};
      if (run_chain(a, mp.lane, mp.key_n, q0.fam, q0.b.precision, sc, st) != 0) return NLS_E_DEVICE;
    }
  }
  e = hipMemcpyAsync(h + g.out_off, d + g.out_off, g.out_bytes, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return NLS_E_DEVICE;
  if (hipEventRecord(L.ev, st) != hipSuccess) return NLS_E_DEVICE;
  return NLS_OK;
}

// release a launch whose results are in the callers' arrays (or that failed)
// and report its requests
void complete(nls_server* s, InFlight& L) {
  const double t = s->now_ms();
  s->arena.release(L.plan.offset, L.plan.layout.total);
  s->free_counters.push_back(L.counter);
  if (L.ev) s->free_events.push_back(L.ev);
  s->load[L.stream] -= L.plan.cost;
  std::lock_guard<std::mutex> lk(s->mu);
  for (const Req& q : L.reqs) {
    nls_request_info info{};
    info.id = q.id;
    info.status = L.status;
    info.merged = (int32_t)L.reqs.size();
    info.systems = q.M;
    info.t_submit_ms = q.t_submit;
    info.t_admit_ms = q.t_admit;
    info.t_done_ms = t;
    s->done.push_back(info);
    s->outstanding -= 1;
    s->st.completed += 1;
  }
  s->st.inflight_launches -= 1;
  s->st.resident_bytes = s->arena.used();
  s->cv_done.notify_all();
}

// a launch failed to enqueue: wait for what was enqueued for it, then report
void fail_launch(nls_server* s, InFlight& L) {
  hipStreamSynchronize(s->streams[L.stream]);
  complete(s, L);
}

// move launch L on when its current phase has ended; true when L is done
bool advance(nls_server* s, InFlight& L) {
  if (L.phase == PH_STAGING) {
    if (L.pending->load() != 0) return false;
    L.status = enqueue(s, L);
    if (L.status != NLS_OK) {
      fail_launch(s, L);
      return true;
    }
    L.phase = PH_DEVICE;
  }
  if (L.phase == PH_DEVICE) {
    const hipError_t e = hipEventQuery(L.ev);
    if (e == hipErrorNotReady) return false;
    if (e != hipSuccess) L.status = NLS_E_DEVICE;
    if (L.status != NLS_OK || run_copies(s, L, result_bytes_per_system, scatter_results)) {
      complete(s, L);
      return true;
    }
    L.phase = PH_SCATTER;
    return false;
  }
  if (L.pending->load() != 0) return false;
  complete(s, L);
  return true;
}

bool reap(nls_server* s) {
  bool any = false;
  for (auto it = s->inflight.begin(); it != s->inflight.end();) {
    const Phase ph = it->phase;
    if (advance(s, *it)) {
      it = s->inflight.erase(it);
      any = true;
      continue;
    }
    any = any || it->phase != ph;
    ++it;
  }
  return any;
}

bool admit(nls_server* s) {
  const size_t slots = (size_t)s->max_inflight - s->inflight.size();
  if (slots == 0) return false;
  std::vector<QueuedReq> view;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    const size_t k = std::min(s->queue.size(), (size_t)s->max_admit);
    view.reserve(k);
    for (size_t i = 0; i < k; ++i) {
      const Req& q = s->queue[i];
      view.push_back(QueuedReq{q.id, q.key, q.M, q.P, q.n, launch_work(q.M, q.n), q.alg == ALG_POLY});
    }
  }
  if (view.empty()) return false;
  std::vector<PlannedLaunch> plan = plan_admission(view, s->arena, (size_t)s->max_admit, slots);
  if (plan.empty()) return false;
  size_t taken = 0;
  for (auto& L : plan) taken += L.reqs.size();
  std::vector<Req> reqs;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (size_t i = 0; i < taken; ++i) {
      reqs.push_back(std::move(s->queue.front()));
      s->queue.pop_front();
    }
    s->st.queued = (int64_t)s->queue.size();
  }
  const double t_admit = s->now_ms();  // one scheduling step: one stamp
  for (auto& P : plan) {
    InFlight L;
    L.plan = P;
    for (size_t j : P.reqs) L.reqs.push_back(std::move(reqs[j]));
    L.stream = pick_stream(s->load, P.cost);
    s->load[L.stream] += P.cost;
    L.counter = s->free_counters.back();
    s->free_counters.pop_back();
    if (!s->free_events.empty()) {
      L.ev = s->free_events.back();
      s->free_events.pop_back();
    } else if (hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) != hipSuccess) {
      L.ev = nullptr;
    }
    for (Req& q : L.reqs) q.t_admit = t_admit;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->st.launches += 1;
      s->st.inflight_launches += 1;
      s->st.resident_bytes = s->arena.used();
      s->st.peak_resident_bytes = std::max(s->st.peak_resident_bytes, s->st.resident_bytes);
    }
    if (!L.ev) {
      L.status = NLS_E_DEVICE;
      complete(s, L);
      continue;
    }
    // (the list node stays put while copy jobs refer to it)
    s->inflight.push_back(std::move(L));
    InFlight& R = s->inflight.back();
    if (!run_copies(s, R, input_bytes_per_system, stage_inputs)) {
      R.phase = PH_STAGING;
      continue;
    }
    R.status = enqueue(s, R);
    if (R.status != NLS_OK) {
      fail_launch(s, R);
      s->inflight.pop_back();
    }
  }
  return true;
}

void run(nls_server* s) {
  hipSetDevice(s->device);
  while (true) {
    bool progressed = reap(s);
    progressed = admit(s) || progressed;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop && s->queue.empty() && s->inflight.empty()) break;
    if (progressed) continue;
    if (s->inflight.empty()) {
      // idle: sleep until a request arrives (or the server stops)
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
    } else {
      // work on the device: poll its events, waking early on a submission
      s->cv_work.wait_for(lk, std::chrono::microseconds(50));
    }
  }
}

void free_server(nls_server* s) {
  {
    std::lock_guard<std::mutex> lk(s->cmu);
    s->cstop = true;
  }
  s->ccv.notify_all();
  for (auto& t : s->copiers)
    if (t.joinable()) t.join();
  hipSetDevice(s->device);
  for (auto st : s->streams)
    if (st) hipStreamSynchronize(st);
  for (auto ev : s->free_events) hipEventDestroy(ev);
  for (auto st : s->streams)
    if (st) hipStreamDestroy(st);
  if (s->counters) hipFree(s->counters);
  if (s->dev) hipFree(s->dev);
  if (s->host) hipHostFree(s->host);
  delete s;
}

}  // namespace

extern "C" {

int nls_server_create(const nls_server_desc* d, nls_server** out) {
  if (!d || !out) return sfail(NLS_E_INVALID, "nls_server_create: NULL argument");
  const int streams = d->streams ? d->streams : 4;
  const int max_inflight = d->max_inflight ? d->max_inflight : 256;
  const int max_admit = d->max_admit ? d->max_admit : 256;
  if (streams < 1 || streams > 16) return sfail(NLS_E_INVALID, "nls_server_create: streams outside 1..16");
  if (max_inflight < 1 || max_inflight > 4096)
    return sfail(NLS_E_INVALID, "nls_server_create: max_inflight outside 1..4096");
  if (max_admit < 1) return sfail(NLS_E_INVALID, "nls_server_create: max_admit must be >= 1");
  if (d->mem_budget_bytes < Arena::kAlign) return sfail(NLS_E_INVALID, "nls_server_create: mem_budget_bytes too small");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return sfail(NLS_E_DEVICE, std::string("hipGetDeviceCount: ") + hipGetErrorString(e));
  if (d->device < 0 || d->device >= ndev) return sfail(NLS_E_INVALID, "nls_server_create: bad device ordinal");
  if ((e = hipSetDevice(d->device)) != hipSuccess) return sfail(NLS_E_DEVICE, hipGetErrorString(e));
  nls_server* s = new nls_server();
  s->device = d->device;
  s->nstreams = streams;
  s->max_inflight = max_inflight;
  s->max_admit = max_admit;
  if (const char* w = std::getenv("NLS_SERVE_SLICE_WORK")) {
    const double v = std::atof(w);
    if (v > 0) s->slice_work = v;
  }
  if (const char* w = std::getenv("NLS_SERVE_INLINE_COPY_BYTES")) {
    const long long v = std::atoll(w);
    if (v >= 0) s->inline_copy_bytes = (size_t)v;
  }
  if (const char* w = std::getenv("NLS_SERVE_COPY_JOB_BYTES")) {
    const long long v = std::atoll(w);
    if (v > 0) s->copy_job_bytes = (size_t)v;
  }
  s->arena.reset(d->mem_budget_bytes);
  s->st.budget_bytes = s->arena.capacity();
  s->t0 = Clock::now();
  s->load.assign(streams, 0.0);
  s->streams.assign(streams, nullptr);
  for (int j = 0; j < streams && e == hipSuccess; ++j) e = hipStreamCreateWithFlags(&s->streams[j], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc((void**)&s->counters, sizeof(int64_t) * max_inflight);
  if (e == hipSuccess) e = hipMalloc((void**)&s->dev, s->arena.capacity());
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->host, s->arena.capacity(), hipHostMallocDefault);
  if (e != hipSuccess) {
    const std::string m = std::string("nls_server_create: ") + hipGetErrorString(e);
    free_server(s);
    return sfail(e == hipErrorOutOfMemory ? NLS_E_NOMEM : NLS_E_DEVICE, m);
  }
  for (int i = max_inflight - 1; i >= 0; --i) s->free_counters.push_back(i);
  try {
    for (int j = 0; j < kCopyThreads; ++j) s->copiers.emplace_back(copier, s);
    s->th = std::thread(run, s);
  } catch (const std::exception& x) {
    // (no scheduler thread yet: free_server stops and joins the copy threads)
    const std::string m = std::string("nls_server_create: cannot start threads: ") + x.what();
    free_server(s);
    return sfail(NLS_E_DEVICE, m);
  }
  *out = s;
  return NLS_OK;
}

int nls_server_submit(nls_server* s, const nls_batch* b, const nls_results* r, uint64_t* id) {
  if (!s || !id) return sfail(NLS_E_INVALID, "nls_server_submit: NULL argument");
  int64_t bad = -1;
  std::string m = validate(b, &bad);
  if (m.empty()) m = check_results(r, b->count);
  if (!m.empty()) return sfail(NLS_E_INVALID, m);
  if (b->mem_kind != NLS_MEM_HOST) return sfail(NLS_E_INVALID, "server requests are host-memory batches");
  Req q;
  q.b = *b;
  q.M = b->count;
  if (r) q.r = *r;
  fill_defaults(&q.opts);
  if (b->opts) q.opts = *b->opts;
  q.b.opts = nullptr;
  q.fam = b->family ? (q.M ? b->family[0] : 0) : b->family_all;
  q.n = b->n ? (q.M ? b->n[0] : 1) : b->n_all;
  q.alg = b->alg ? (q.M ? b->alg[0] : 0) : b->alg_all;
  for (int64_t i = 0; i < q.M; ++i) {
    if ((b->family && b->family[i] != q.fam) || (b->n && b->n[i] != q.n) || (b->alg && b->alg[i] != q.alg))
      return sfail(NLS_E_INVALID, "server requests have one family, size and algorithm");
  }
  q.P = nparams_of(q.fam, q.n);
  q.key = merge_key(q);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return sfail(NLS_E_INVALID, "server is shutting down");
  if (region_layout(q.M, q.P, q.n, q.alg == ALG_POLY).total > s->arena.capacity())
    return sfail(NLS_E_NOMEM, "request needs more device memory than the server's budget");
  q.id = s->next_id++;
  q.t_submit = s->now_ms();
  *id = q.id;
  if (q.M == 0) {
    nls_request_info info{};
    info.id = q.id;
    info.status = NLS_OK;
    info.merged = 1;
    info.t_submit_ms = info.t_admit_ms = info.t_done_ms = q.t_submit;
    s->done.push_back(info);
    s->st.completed += 1;
    s->cv_done.notify_all();
    return NLS_OK;
  }
  s->queue.push_back(std::move(q));
  s->outstanding += 1;
  s->st.queued = (int64_t)s->queue.size();
  s->cv_work.notify_one();
  return NLS_OK;
}

int nls_server_poll(nls_server* s, int32_t wait_ms, nls_request_info* out, int32_t max_out, int32_t* n_out) {
  if (!s || !n_out || (max_out > 0 && !out) || max_out < 0) return sfail(NLS_E_INVALID, "nls_server_poll: bad argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [&] { return !s->done.empty() || s->outstanding == 0; };
  if (wait_ms < 0) s->cv_done.wait(lk, ready);
  else if (wait_ms > 0) s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
  int32_t k = 0;
  while (k < max_out && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n_out = k;
  return NLS_OK;
}

int nls_server_stats_get(nls_server* s, nls_server_stats* st) {
  if (!s || !st) return sfail(NLS_E_INVALID, "nls_server_stats_get: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *st = s->st;
  return NLS_OK;
}

int nls_server_destroy(nls_server* s) {
  if (!s) return NLS_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  free_server(s);
  return NLS_OK;
}

}  // extern "C"
