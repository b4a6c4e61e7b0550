// Host-only checks of the request server's allocator, region layout and
// admission planner (no device).  Built and run by tests/test_serve_core.py;
// prints "OK" and exits 0, or names the failed check and exits 1.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "nls_serve_core.hpp"

using namespace nls::serve;

static int failures = 0;
#define CHECK(c, ...)                                   \
  do {                                                  \
    if (!(c)) {                                         \
      std::printf("FAIL %s:%d: ", __FILE__, __LINE__);  \
      std::printf(__VA_ARGS__);                         \
      std::printf("\n");                                \
      if (++failures > 20) std::exit(1);                \
    }                                                   \
  } while (0)

// Occupancy model of the arena, one flag per 256-byte granule.
struct Model {
  std::vector<char> used;
  explicit Model(uint64_t cap) : used(cap / Arena::kAlign, 0) {}
  bool mark(uint64_t off, uint64_t n, char v) {
    const uint64_t a = off / Arena::kAlign, b = (off + Arena::round(n)) / Arena::kAlign;
    if (off % Arena::kAlign || b > used.size()) return false;
    for (uint64_t g = a; g < b; ++g) {
      if (used[g] == v) return false;  // double allocation or double free
      used[g] = v;
    }
    return true;
  }
  uint64_t count() const {
    uint64_t c = 0;
    for (char x : used) c += x;
    return c * Arena::kAlign;
  }
  // the largest run of free granules
  uint64_t largest_free() const {
    uint64_t best = 0, run = 0;
    for (char x : used) {
      run = x ? 0 : run + 1;
      best = std::max(best, run);
    }
    return best * Arena::kAlign;
  }
};

static void check_arena() {
  std::mt19937_64 rng(7);
  for (int trial = 0; trial < 20; ++trial) {
    const uint64_t cap = (1 + rng() % 64) * 4096 + (rng() % 255);  // not a multiple of 256
    Arena a(cap);
    CHECK(a.capacity() == cap / 256 * 256, "capacity rounding");
    Model m(a.capacity());
    std::vector<std::pair<uint64_t, uint64_t>> live;
    for (int step = 0; step < 2000; ++step) {
      if (live.empty() || rng() % 3) {
        const uint64_t n = 1 + rng() % (a.capacity() / 4 + 1);
        uint64_t off = 0;
        const bool ok = a.alloc(n, &off);
        // first fit succeeds exactly when some free run is long enough
        CHECK(ok == (m.largest_free() >= Arena::round(n)), "alloc success vs free runs (n=%llu)",
              (unsigned long long)n);
        if (ok) {
          CHECK(m.mark(off, n, 1), "overlapping allocation at %llu", (unsigned long long)off);
          live.push_back({off, n});
        }
      } else {
        const size_t k = rng() % live.size();
        a.release(live[k].first, live[k].second);
        CHECK(m.mark(live[k].first, live[k].second, 0), "bad release");
        live.erase(live.begin() + k);
      }
      CHECK(a.used() == m.count(), "used() = %llu, model %llu", (unsigned long long)a.used(),
            (unsigned long long)m.count());
      CHECK(a.largest_free() == m.largest_free(), "largest free extent");
    }
    for (auto& x : live) a.release(x.first, x.second);
    CHECK(a.used() == 0 && a.extents() == 1 && a.largest_free() == a.capacity(), "full coalescing");
  }
}

static void check_layout() {
  for (int64_t m : {1, 3, 64, 1000}) {
    for (int n : {1, 2, 7, 8, 64}) {
      for (int P : {0, 3, n * n + n, n * n + n + 1}) {
        const Region r = region_layout(m, P, n);
        CHECK(r.params == 0 && r.u0 >= 8ull * m * P && r.in_bytes >= r.u0 + 8ull * m * n, "input spans");
        CHECK(r.out_off == r.in_bytes && r.u == r.out_off, "outputs follow inputs");
        CHECK(r.fnorm >= r.u + 8ull * m * n && r.iters >= r.fnorm + 8ull * m, "u, fnorm");
        CHECK(r.retcode >= r.iters + 4ull * m && r.nfev >= r.retcode + 4ull * m && r.njev >= r.nfev + 4ull * m,
              "counts");
        CHECK(r.out_off + r.out_bytes == r.total && r.total >= r.njev + 4ull * m, "total");
        for (uint64_t x : {r.u0, r.u, r.fnorm, r.iters, r.retcode, r.nfev, r.njev, r.total})
          CHECK(x % 16 == 0, "16-byte alignment");
      }
    }
  }
}

static std::vector<QueuedReq> random_queue(std::mt19937_64& rng, int len, int keys, int64_t maxm) {
  std::vector<QueuedReq> q;
  for (int i = 0; i < len; ++i) {
    const int k = (int)(rng() % keys);
    const int n = 2 + k % 7;
    q.push_back(QueuedReq{(uint64_t)i + 1, "k" + std::to_string(k), 1 + (int64_t)(rng() % maxm), n * n + n, n,
                          1.0});
  }
  return q;
}

static void check_chain_layout() {
  for (int64_t m : {1, 7, 64, 1000}) {
    for (int n : {1, 8, 24, 64}) {
      const int P = n * n + n + 1;
      const Region a = region_layout(m, P, n), c = region_layout(m, P, n, true);
      CHECK(a.sel1 == 0 && a.total == a.out_off + a.out_bytes, "no scratch without the chain");
      CHECK(c.out_off == a.out_off && c.out_bytes == a.out_bytes && c.u == a.u && c.njev == a.njev,
            "the chain keeps the input/output layout");
      const uint64_t lo[9] = {c.sel1, c.sel2, c.cnt, c.u_t, c.fnorm_t, c.iters_t, c.retcode_t, c.nfev_t, c.njev_t};
      const uint64_t sz[9] = {4ull * m, 4ull * m, 32, 8ull * m * n, 8ull * m, 4ull * m, 4ull * m, 4ull * m, 4ull * m};
      uint64_t prev = c.out_off + c.out_bytes;
      for (int k = 0; k < 9; ++k) {
        CHECK(lo[k] >= prev && lo[k] % 16 == 0, "chain span %d after the previous, aligned", k);
        prev = lo[k] + sz[k];
      }
      CHECK(c.total >= prev, "chain scratch inside the region");
    }
  }
  // the planner sizes chain launches with their scratch
  Arena arena(1 << 20);
  std::vector<QueuedReq> q = {QueuedReq{1, "chain", 10, 73, 8, 1.0, true}};
  auto plan = plan_admission(q, arena, 8, 8);
  CHECK(plan.size() == 1 && plan[0].chain && plan[0].layout.total == region_layout(10, 73, 8, true).total,
        "chain launch planned with scratch");
}

static void check_planner() {
  std::mt19937_64 rng(11);
  for (int trial = 0; trial < 400; ++trial) {
    const uint64_t cap = (1 + rng() % 32) * 65536;
    Arena a(cap);
    Model m(a.capacity());
    // some memory already held by earlier launches
    std::vector<std::pair<uint64_t, uint64_t>> held;
    for (int i = 0; i < (int)(rng() % 6); ++i) {
      uint64_t off, n = 1 + rng() % (cap / 8);
      if (a.alloc(n, &off)) {
        m.mark(off, n, 1);
        held.push_back({off, n});
      }
    }
    const Arena before = a;
    const uint64_t used0 = a.used();
    auto q = random_queue(rng, 1 + (int)(rng() % 40), 1 + (int)(rng() % 6), 1 + (int64_t)(rng() % 600));
    const size_t max_reqs = 1 + rng() % 50, max_launches = 1 + rng() % 8;
    auto plan = plan_admission(q, a, max_reqs, max_launches);
    // the admitted requests are a prefix of the queue, each exactly once, and
    // each launch holds requests of one key with consecutive system ranges
    std::set<size_t> seen;
    uint64_t placed = 0;
    for (auto& L : plan) {
      CHECK(!L.reqs.empty() && L.reqs.size() == L.first.size(), "launch members");
      int64_t acc = 0;
      for (size_t j = 0; j < L.reqs.size(); ++j) {
        const QueuedReq& r = q[L.reqs[j]];
        CHECK(r.key == L.key && r.n == L.n && r.P == L.P, "merged requests share the key");
        CHECK(L.first[j] == acc, "first system of a member");
        CHECK(j == 0 || L.reqs[j] > L.reqs[j - 1], "members in arrival order");
        acc += r.m;
        CHECK(seen.insert(L.reqs[j]).second, "request admitted twice");
      }
      CHECK(acc == L.m, "launch size");
      const Region g = region_layout(L.m, L.P, L.n);
      CHECK(g.total == L.layout.total, "launch layout");
      CHECK(m.mark(L.offset, L.layout.total, 1), "placement overlaps held memory or another launch");
      placed += Arena::round(L.layout.total);
    }
    const size_t k = seen.size();
    CHECK(k == 0 || *seen.rbegin() == k - 1, "admitted set is not a prefix");
    CHECK(k <= max_reqs && plan.size() <= max_launches, "limits");
    CHECK(a.used() == used0 + placed, "arena accounting");
    // maximality: the next request could not have been admitted too
    if (k < q.size() && k < max_reqs) {
      std::vector<QueuedReq> q2(q.begin(), q.begin() + k + 1);
      Arena b = before;
      auto p2 = plan_admission(q2, b, k + 1, max_launches);
      size_t k2 = 0;
      for (auto& L : p2) k2 += L.reqs.size();
      CHECK(k2 == k, "prefix not maximal (%zu admitted, %zu possible)", k, k2);
    }
    // head-of-line blocking: nothing is admitted when the head does not fit
    if (k == 0) {
      const Region g = region_layout(q[0].m, q[0].P, q[0].n);
      CHECK(Arena::round(g.total) > before.largest_free() || max_launches == 0, "head fits but was refused");
    }
  }
}

// Event-driven simulation of the scheduler with a fake clock: arrivals with
// random gaps, a launch finishes after a time proportional to its systems,
// completed launches release their memory.  Checks that the budget is never
// exceeded, requests are admitted in arrival order and every request
// completes exactly once.
static void check_simulation() {
  std::mt19937_64 rng(5);
  for (int trial = 0; trial < 30; ++trial) {
    const uint64_t cap = 4 * 1048576;
    Arena a(cap);
    auto all = random_queue(rng, 300, 8, 3000);
    std::vector<double> arrive(all.size());
    double t = 0;
    for (auto& x : arrive) x = (t += (rng() % 1000) * 1e-3);
    struct Run { double end; uint64_t off, bytes; std::vector<uint64_t> ids; };
    std::vector<Run> running;
    std::vector<QueuedReq> queue;
    std::vector<uint64_t> admitted_order, completed;
    size_t next = 0;
    double now = 0;
    while (completed.size() < all.size()) {
      // next event: an arrival or a completion
      double t_arr = next < all.size() ? arrive[next] : 1e300;
      double t_end = 1e300;
      for (auto& r : running) t_end = std::min(t_end, r.end);
      now = std::min(t_arr, t_end);
      if (t_arr <= t_end) {
        queue.push_back(all[next++]);
      } else {
        for (size_t i = 0; i < running.size();) {
          if (running[i].end <= now) {
            a.release(running[i].off, running[i].bytes);
            for (auto id : running[i].ids) completed.push_back(id);
            running.erase(running.begin() + i);
          } else {
            ++i;
          }
        }
      }
      auto plan = plan_admission(queue, a, 64, 16 - std::min<size_t>(16, running.size()));
      size_t taken = 0;
      for (auto& L : plan) {
        Run r{now + 1e-4 * L.m, L.offset, L.layout.total, {}};
        for (size_t j : L.reqs) r.ids.push_back(queue[j].id);
        taken += L.reqs.size();
        running.push_back(r);
      }
      for (size_t i = 0; i < taken; ++i) admitted_order.push_back(queue[i].id);
      queue.erase(queue.begin(), queue.begin() + taken);
      CHECK(a.used() <= a.capacity(), "budget exceeded");
      if (running.empty() && !queue.empty()) CHECK(false, "stalled with an empty device");
    }
    for (size_t i = 0; i < admitted_order.size(); ++i) CHECK(admitted_order[i] == i + 1, "admission order");
    std::set<uint64_t> c(completed.begin(), completed.end());
    CHECK(c.size() == all.size() && completed.size() == all.size(), "each request completes once");
    CHECK(a.used() == 0, "memory released");
  }
}

static void check_slices_and_streams() {
  for (double w : {67108864.0, 1e6, 1e9, 1e20}) {
    int64_t prev = INT64_MAX;
    for (int n = 1; n <= 64; ++n) {
      const int64_t m = slice_systems(n, w);
      CHECK(m >= 64 && m % 64 == 0, "slice of %lld systems at n=%d", (long long)m, n);
      CHECK(m == 64 || launch_work(m, n) <= w, "slice work above the bound at n=%d", n);
      CHECK(m == 64 || w > 1e12 || launch_work(m + 64, n) > w, "slice not maximal at n=%d", n);
      CHECK(m <= prev, "slices grow with n");
      prev = m;
    }
  }
  CHECK(slice_systems(16, 67108864.0) == 16384 && slice_systems(64, 67108864.0) == 256, "slices at 2^26");
  CHECK(slice_systems(8, 0.0) == kNoSlice && slice_systems(64, -1.0) == kNoSlice, "slicing off");
  // stream 0 takes only small launches
  std::vector<double> load = {0.0, 5.0, 3.0, 3.0};
  CHECK(pick_stream(load, 10.0) == 0, "small work goes to the idle express stream");
  CHECK(pick_stream(load, kExpressWork * 2) == 2, "large work skips stream 0 (ties: lowest index)");
  load[0] = 9.0;
  CHECK(pick_stream(load, 10.0) == 2, "small work goes to the least-loaded stream");
  std::vector<double> one = {7.0};
  CHECK(pick_stream(one, kExpressWork * 2) == 0, "a single stream takes everything");
}

// copy jobs: ordered ranges that partition the systems, each within the
// job size unless a single system exceeds it
static void check_copy_ranges() {
  for (int64_t m : {int64_t(0), int64_t(1), int64_t(7), int64_t(1000), int64_t(65536)}) {
    for (size_t bps : {size_t(1), size_t(24), size_t(2304), size_t(33288)}) {
      for (size_t job : {size_t(1), size_t(3000), size_t(16) << 20}) {
        const auto r = copy_ranges(m, bps, job);
        int64_t at = 0;
        for (const auto& x : r) {
          CHECK(x.first == at && x.second > x.first, "m=%lld: ranges in order, non-empty", (long long)m);
          CHECK((size_t)(x.second - x.first) * bps <= job || x.second - x.first == 1, "range within the job size");
          at = x.second;
        }
        CHECK(at == m, "m=%lld bps=%zu job=%zu: ranges cover every system", (long long)m, bps, job);
      }
    }
  }
}

int main() {
  check_copy_ranges();
  check_chain_layout();
  check_slices_and_streams();
  check_arena();
  check_layout();
  check_planner();
  check_simulation();
  if (failures) return 1;
  std::printf("OK\n");
  return 0;
}
