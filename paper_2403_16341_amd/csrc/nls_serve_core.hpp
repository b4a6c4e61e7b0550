// nls_serve_core.hpp -- the device-independent parts of the request server:
// the arena that places resident requests inside the device-memory budget,
// the layout of one launch's region in it, and the admission planner that
// turns the head of the request queue into launches.  Plain C++ (offsets and
// sizes only), so the policy runs and is tested without a device.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <iterator>
#include <map>
#include <string>
#include <utility>
#include <vector>

namespace nls {
namespace serve {

// First-fit allocator over [0, capacity) in 256-byte granules.  Free extents
// are kept by offset and merged with their neighbours on release.
class Arena {
 public:
  static constexpr uint64_t kAlign = 256;
  explicit Arena(uint64_t capacity = 0) { reset(capacity); }
  void reset(uint64_t capacity) {
    cap_ = capacity / kAlign * kAlign;
    used_ = 0;
    free_.clear();
    if (cap_) free_[0] = cap_;
  }
  static uint64_t round(uint64_t n) { return (std::max<uint64_t>(n, 1) + kAlign - 1) / kAlign * kAlign; }
  // place n bytes; false if no free extent is large enough
  bool alloc(uint64_t n, uint64_t* off) {
    n = round(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const uint64_t rest = it->second - n, at = it->first + n;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += n;
      return true;
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    n = round(n);
    used_ -= n;
    uint64_t start = off, len = n;
    auto next = free_.lower_bound(off);
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + n == next->first) {
      len += next->second;
      free_.erase(next);
    }
    free_[start] = len;
  }
  uint64_t capacity() const { return cap_; }
  uint64_t used() const { return used_; }
  size_t extents() const { return free_.size(); }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  uint64_t cap_ = 0, used_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

// Byte layout of one launch's region: the inputs (parameters, then starting
// points) and, after them, the outputs in one contiguous span so that each
// direction is a single copy.  A launch of the fallback chain adds the
// chain's device scratch after the outputs (never copied).
struct Region {
  uint64_t params, u0, in_bytes;  // inputs: [0, in_bytes)
  uint64_t u, fnorm, iters, retcode, nfev, njev;
  uint64_t out_off, out_bytes;    // outputs: [out_off, out_off + out_bytes)
  // chain scratch (0 when absent): two system lists, four counts, and
  // scratch outputs laid out like the outputs
  uint64_t sel1, sel2, cnt, u_t, fnorm_t, iters_t, retcode_t, nfev_t, njev_t;
  uint64_t total;
};

inline uint64_t align16(uint64_t x) { return (x + 15) / 16 * 16; }

inline Region region_layout(int64_t m, int P, int n, bool chain = false) {
  Region r{};
  uint64_t o = 0;
  r.params = o;
  o = align16(o + 8ull * m * P);
  r.u0 = o;
  o = align16(o + 8ull * m * n);
  r.in_bytes = o;
  r.out_off = o;
  r.u = o;
  o = align16(o + 8ull * m * n);
  r.fnorm = o;
  o = align16(o + 8ull * m);
  r.iters = o;
  o = align16(o + 4ull * m);
  r.retcode = o;
  o = align16(o + 4ull * m);
  r.nfev = o;
  o = align16(o + 4ull * m);
  r.njev = o;
  o = align16(o + 4ull * m);
  r.out_bytes = o - r.out_off;
  if (chain) {
    const uint64_t sizes[9] = {4ull * m, 4ull * m, 32, 8ull * m * n, 8ull * m, 4ull * m, 4ull * m, 4ull * m, 4ull * m};
    uint64_t* at[9] = {&r.sel1, &r.sel2, &r.cnt, &r.u_t, &r.fnorm_t, &r.iters_t, &r.retcode_t, &r.nfev_t, &r.njev_t};
    for (int k = 0; k < 9; ++k) {
      *at[k] = o;
      o = align16(o + sizes[k]);
    }
  }
  r.total = o;
  return r;
}

// A queued request as the planner sees it.  Requests with equal keys (same
// kernel, tolerances and options) may share one launch.
struct QueuedReq {
  uint64_t id;
  std::string key;
  int64_t m;  // systems
  int P, n;
  double cost;         // estimated work, for stream balancing
  bool chain = false;  // the fallback chain (its region carries scratch)
};

struct PlannedLaunch {
  std::string key;
  std::vector<size_t> reqs;      // positions in the queue, in arrival order
  std::vector<int64_t> first;    // first system of each request inside the launch
  int64_t m = 0;
  int P = 0, n = 0;
  bool chain = false;
  double cost = 0.0;
  Region layout{};
  uint64_t offset = 0;           // placement in the arena
};

// Admission: the longest prefix of the queue (first come, first served; at
// most max_reqs requests and max_launches new launches) whose launches can
// all be placed in the arena at once.  Requests of the prefix with equal keys
// are merged into one launch.  The head request blocks the rest when it does
// not fit, so large requests are never starved.  The launches are placed in
// the arena on return; an empty result means nothing fits until memory is
// released.
inline std::vector<PlannedLaunch> plan_admission(const std::vector<QueuedReq>& q, Arena& arena,
                                                 size_t max_reqs, size_t max_launches) {
  std::vector<PlannedLaunch> best;
  std::vector<PlannedLaunch> cur;
  std::map<std::string, size_t> at;
  const size_t limit = std::min(q.size(), max_reqs);
  for (size_t i = 0; i < limit; ++i) {
    const QueuedReq& r = q[i];
    auto it = at.find(r.key);
    if (it == at.end()) {
      if (cur.size() >= max_launches) break;
      PlannedLaunch L;
      L.key = r.key;
      L.P = r.P;
      L.n = r.n;
      L.chain = r.chain;
      at[r.key] = cur.size();
      cur.push_back(L);
      it = at.find(r.key);
    }
    PlannedLaunch& L = cur[it->second];
    L.reqs.push_back(i);
    L.first.push_back(L.m);
    L.m += r.m;
    L.cost += r.cost;
    L.layout = region_layout(L.m, L.P, L.n, L.chain);
    // can every launch of the prefix be placed at once?  (largest first on a
    // copy of the arena; the same order is used for the real placement)
    std::vector<size_t> ord(cur.size());
    for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](size_t a, size_t b) { return cur[a].layout.total > cur[b].layout.total; });
    Arena trial = arena;
    bool fits = true;
    for (size_t k : ord) {
      uint64_t off;
      if (!trial.alloc(cur[k].layout.total, &off)) { fits = false; break; }
      cur[k].offset = off;
    }
    if (!fits) break;
    best = cur;
  }
  // commit the placement of the accepted prefix
  std::vector<size_t> ord(best.size());
  for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
  std::stable_sort(ord.begin(), ord.end(),
                   [&](size_t a, size_t b) { return best[a].layout.total > best[b].layout.total; });
  for (size_t k : ord) {
    uint64_t off = 0;
    arena.alloc(best[k].layout.total, &off);
    best[k].offset = off;
  }
  return best;
}

// Slicing: a launch whose work (systems x n^3) exceeds a bound may run as
// several persistent launches in a row on its stream; between two of them the
// device's dispatcher hands freed compute units to other streams' launches.
// Off by default: each slice ends with its slowest system, which costs more
// throughput than the latency it saves (measured on the serving workload).
constexpr int64_t kNoSlice = int64_t(1) << 60;  // more systems than any launch

// Systems per slice for size n under the bound slice_work (<= 0: no slicing):
// a multiple of 64, at least 64.
inline int64_t slice_systems(int n, double slice_work) {
  if (!(slice_work > 0)) return kNoSlice;
  const double n3 = (double)n * n * n;
  const double m = slice_work / n3;
  if (m >= (double)kNoSlice) return kNoSlice;
  const int64_t k = (int64_t)m / 64 * 64;
  return k < 64 ? 64 : k;
}

inline double launch_work(int64_t m, int n) { return (double)m * n * n * n; }

// Host copy jobs of a request of m systems at bytes_per_system each: ranges
// [i0, i1) that cover 0 .. m - 1 in order, each of at most job_bytes (at least
// one system per range).
inline std::vector<std::pair<int64_t, int64_t>> copy_ranges(int64_t m, size_t bytes_per_system, size_t job_bytes) {
  std::vector<std::pair<int64_t, int64_t>> r;
  const int64_t step = std::max<int64_t>(1, (int64_t)(job_bytes / (bytes_per_system ? bytes_per_system : 1)));
  for (int64_t i0 = 0; i0 < m; i0 += step) r.emplace_back(i0, std::min<int64_t>(m, i0 + step));
  return r;
}

// Launches up to this much work (systems x n^3; e.g. 16k systems at n = 16,
// 256 at n = 64) may use stream 0; larger ones never do.
constexpr double kExpressWork = 67108864.0;  // 2^26

// Larger launches run on at most this share of the device's resident
// wavefronts (percent): a persistent grid sized for the whole device would
// hold every compute unit until its last system ends, so an express launch
// queued meanwhile on stream 0 could not start.
constexpr int kLargeGridPct = 75;

// Stream for a launch: the least-loaded one (ties: lowest index).  With more
// than one stream, stream 0 is kept for small launches, so a small request
// never waits behind a large one in stream order.
inline int pick_stream(const std::vector<double>& load, double work, double express_work = kExpressWork) {
  const size_t first = (load.size() > 1 && work > express_work) ? 1 : 0;
  return (int)(std::min_element(load.begin() + first, load.end()) - load.begin());
}

}  // namespace serve
}  // namespace nls
