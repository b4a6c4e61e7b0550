// nls_host.cpp -- host runtime behind the C ABI of include/nls.h.
//
// Validation, bucketing of mixed batches by kernel mapping, device staging of
// host payloads, launches on the context's stream, and tickets (an event per
// batch plus the device memory to release when it completes).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "nls.h"
#include "nls_launch.h"
#include "nls_runtime.h"
#include "nls_types.h"

using namespace nls;

namespace nls {
namespace rt {
thread_local std::string g_tls_error = "";
void set_thread_error(const std::string& m) { g_tls_error = m; }
const char* thread_error() { return g_tls_error.c_str(); }
}  // namespace rt
}  // namespace nls

using namespace nls::rt;

namespace {

struct Ticket {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
  std::vector<void*> device_allocs;
  int64_t systems = 0;
  int32_t status = NLS_OK;
  uint64_t bytes = 0;  // device bytes the ticket holds until released
};

}  // namespace

struct nls_context {
  int device = 0;
  uint32_t flags = 0;
  uint64_t budget = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::mutex mu;
  std::string last_error;
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, Ticket> tickets;
  uint64_t held_bytes = 0;  // device bytes held by outstanding tickets
  // dynamic work counters, one per launch of a call; calls on one stream run
  // in order, so every call may reuse them (zeroed at its start)
  int64_t* counters = nullptr;
  int ncounters = 0;
  // parallel branches of a captured multi-kernel launch
  static constexpr int kBranches = 4;
  hipStream_t branch[kBranches] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kBranches] = {};
  // the last captured graph and the launch list it was made from
  hipGraphExec_t graph_exec = nullptr;
  std::string graph_sig;
  // autotuned mapping per (n, family, algorithm, precision): 1 = lane, 2 = group
  std::map<int, int> tuned;
  std::string tune_cache_path;
  int forced = 0;  // NLS_MAPPING: 1 = lane, 2 = group for every n <= 8 system
  // plan of a mixed batch (bucketed system order, offsets, sizes): a grow-only
  // device buffer and its pinned host mirror, reused by every call (so a call
  // neither allocates nor waits, and a replayed graph sees the same
  // pointers); plan_ev marks the end of the last copy out of the mirror
  char* plan_dev = nullptr;
  char* plan_host = nullptr;
  size_t plan_cap = 0;
  hipEvent_t plan_ev = nullptr;
  bool plan_ev_pending = false;
};

namespace {

int fail(nls_context* c, int code, const std::string& msg) {
  if (c) c->last_error = msg;
  set_thread_error(msg);
  return code;
}

int hip_fail(nls_context* c, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(c, NLS_E_DEVICE, m);
}

}  // namespace

namespace nls {
namespace rt {

int group_bucket(int n) { return ((n + 7) / 8) * 8 < 16 ? 16 : ((n + 7) / 8) * 8; }

int nparams_of(int family, int n) {
  if (n < 1 || n > NLS_NMAX) return -1;
  switch (family) {
    case NLS_FAMILY_CUBIC: return n * n + n;
    case NLS_FAMILY_TANH: return n * n + n + 1;
    case NLS_FAMILY_ROSENBROCK: return n >= 2 ? 0 : -1;
    case NLS_FAMILY_PAPER_EXAMPLE: return n == 2 ? 3 : -1;
  }
  return -1;
}

// A family/size pair the kernels implement (Rosenbrock has group kernels up
// to n = 16 only).
bool supported(int family, int n) {
  if (nparams_of(family, n) < 0) return false;
  if (family == NLS_FAMILY_ROSENBROCK && n > 16) return false;
  return true;
}

// One family, size and algorithm for every system, packed back to back (the
// layout the single-launch path takes).
bool uniform_batch(const nls_batch* b, int* fam0, int* n0, int* alg0) {
  const int64_t M = b->count;
  *fam0 = b->family ? (M ? b->family[0] : 0) : b->family_all;
  *n0 = b->n ? (M ? b->n[0] : 1) : b->n_all;
  *alg0 = b->alg ? (M ? b->alg[0] : 0) : b->alg_all;
  if (!b->family && !b->n && !b->alg && !b->p_offset && !b->u_offset) return true;
  const int P0 = nparams_of(*fam0, *n0);
  for (int64_t s = 0; s < M; ++s) {
    const int fam = b->family ? b->family[s] : b->family_all;
    const int n = b->n ? b->n[s] : b->n_all;
    const int alg = b->alg ? b->alg[s] : b->alg_all;
    if (fam != *fam0 || n != *n0 || alg != *alg0) return false;
    if (b->p_offset && b->p_offset[s] != s * (int64_t)P0) return false;
    if (b->u_offset && b->u_offset[s] != s * (int64_t)*n0) return false;
  }
  return true;
}


void fill_defaults(nls_alg_options* o) {
  o->armijo_c = 1e-4;
  o->armijo_rho = 0.5;
  o->armijo_max_halvings = 10;
  o->reserved0 = 0;
  o->tr_delta0 = 1.0;
  o->tr_delta_max = 1e8;
  o->tr_eta1 = 1e-4;
  o->tr_eta2 = 0.75;
  o->tr_expand = 2.0;
  o->tr_shrink = 0.25;
  o->tr_collapse = 1e-14;
}

std::string check_options(const nls_alg_options& o) {
  auto ok = [](double x) { return std::isfinite(x); };
  if (!(ok(o.armijo_c) && o.armijo_c > 0 && o.armijo_c < 0.5)) return "armijo_c must be in (0, 0.5)";
  if (!(ok(o.armijo_rho) && o.armijo_rho > 0 && o.armijo_rho < 1)) return "armijo_rho must be in (0, 1)";
  if (o.armijo_max_halvings < 0 || o.armijo_max_halvings > 1000) return "armijo_max_halvings must be in [0, 1000]";
  if (!(ok(o.tr_delta0) && o.tr_delta0 > 0)) return "tr_delta0 must be > 0";
  if (!(o.tr_delta_max >= o.tr_delta0)) return "tr_delta_max must be >= tr_delta0";
  if (!(ok(o.tr_eta1) && ok(o.tr_eta2) && o.tr_eta1 >= 0 && o.tr_eta1 < o.tr_eta2 && o.tr_eta2 <= 1))
    return "need 0 <= tr_eta1 < tr_eta2 <= 1";
  if (!(ok(o.tr_expand) && o.tr_expand >= 1)) return "tr_expand must be >= 1";
  if (!(ok(o.tr_shrink) && o.tr_shrink > 0 && o.tr_shrink < 1)) return "tr_shrink must be in (0, 1)";
  if (!(ok(o.tr_collapse) && o.tr_collapse >= 0)) return "tr_collapse must be >= 0";
  return "";
}

// Validation shared by nls_validate and nls_solve_batch.  Returns "" if ok.
std::string validate(const nls_batch* b, int64_t* first_bad) {
  if (first_bad) *first_bad = -1;
  if (!b) return "batch is NULL";
  if (b->count < 0) return "count must be >= 0";
  if (b->count > (int64_t)INT32_MAX) return "count exceeds 2^31 - 1";
  if (b->precision != NLS_PREC_FP64 && b->precision != NLS_PREC_FP32_INNER) return "unknown precision";
  if (b->mem_kind != NLS_MEM_HOST && b->mem_kind != NLS_MEM_DEVICE) return "unknown mem_kind";
  if (!(b->abstol >= 0.0)) return "abstol must be >= 0 (and not NaN)";
  if (b->maxiters < 0) return "maxiters must be >= 0";
  if (b->opts) {
    std::string m = check_options(*b->opts);
    if (!m.empty()) return m;
  }
  const int64_t M = b->count;
  if (M == 0) return "";
  // every system described by the scalar fields and packed back to back:
  // one check covers the whole batch
  const bool scalar = !b->family && !b->n && !b->alg && !b->p_offset && !b->u_offset;
  const int64_t checked = scalar ? 1 : M;
  int64_t ptotal = 0, utotal = 0;
  for (int64_t s = 0; s < checked; ++s) {
    const int fam = b->family ? b->family[s] : b->family_all;
    const int n = b->n ? b->n[s] : b->n_all;
    const int alg = b->alg ? b->alg[s] : b->alg_all;
    char buf[160];
    if (n < 1 || n > NLS_NMAX) {
      if (first_bad) *first_bad = s;
      std::snprintf(buf, sizeof buf, "system %lld: n = %d outside [1, 64]", (long long)s, n);
      return buf;
    }
    if (fam < 0 || fam >= FAM_COUNT || !supported(fam, n)) {
      if (first_bad) *first_bad = s;
      std::snprintf(buf, sizeof buf, "system %lld: family %d is not defined at n = %d", (long long)s, fam, n);
      return buf;
    }
    if (alg < 0 || alg >= ALG_KEYS) {
      if (first_bad) *first_bad = s;
      std::snprintf(buf, sizeof buf, "system %lld: unknown algorithm %d", (long long)s, alg);
      return buf;
    }
    const int P = nparams_of(fam, n);
    if (b->p_offset) {
      if (b->p_offset[s + 1] - b->p_offset[s] < P || b->p_offset[s] < 0) {
        if (first_bad) *first_bad = s;
        std::snprintf(buf, sizeof buf, "system %lld: p_offset span %lld < %d parameters", (long long)s,
                      (long long)(b->p_offset[s + 1] - b->p_offset[s]), P);
        return buf;
      }
    }
    if (b->u_offset) {
      if (b->u_offset[s] < 0 || b->u_offset[s + 1] - b->u_offset[s] < n) {
        if (first_bad) *first_bad = s;
        std::snprintf(buf, sizeof buf, "system %lld: u_offset span shorter than n = %d", (long long)s, n);
        return buf;
      }
    }
    ptotal += P;
    utotal += n;
  }
  (void)utotal;
  if (!b->u0) return "u0 is NULL";
  if (ptotal > 0 && !b->params) return "params is NULL";
  return "";
}

std::string check_results(const nls_results* r, int64_t M) {
  if (M == 0) return "";
  if (!r) return "results is NULL";
  if (!r->u || !r->fnorm_inf || !r->iters || !r->retcode) return "a required result array is NULL";
  return "";
}

KOpts to_kopts(const nls_alg_options& o) {
  KOpts k;
  k.armijo_c = o.armijo_c;
  k.armijo_rho = o.armijo_rho;
  k.armijo_max_halvings = o.armijo_max_halvings;
  k.pad = 0;
  k.tr_delta0 = o.tr_delta0;
  k.tr_delta_max = o.tr_delta_max;
  k.tr_eta1 = o.tr_eta1;
  k.tr_eta2 = o.tr_eta2;
  k.tr_expand = o.tr_expand;
  k.tr_shrink = o.tr_shrink;
  k.tr_collapse = o.tr_collapse;
  return k;
}

int launch(int n_or_nb, bool lane, int fam, int alg, int prec, const KArgs& a, hipStream_t st) {
  if (lane) return prec == PREC_FP64 ? launch_lane_f64(n_or_nb, fam, alg, a, st)
                                     : launch_lane_f32(n_or_nb, fam, alg, a, st);
  return launch_group(prec, n_or_nb, fam, alg, a, st);
}

Mapping fixed_mapping(int n) {
  if (n > 8) return Mapping{false, group_bucket(n), hipSuccess};
  return Mapping{true, n, hipSuccess};
}

int run_chain(const KArgs& a, bool lane, int key_n, int fam, int prec, const ChainScratch& sc, hipStream_t st) {
  if (a.count <= 0) return 0;
  // cnt[stage] = systems handed to the stage, cnt[2 + stage] = its work counter
  if (int z = launch_zero_counters(sc.cnt, 4, st); z < 0) return z;
  for (int stage = 0; stage < 2; ++stage) {
    const int alg = stage == 0 ? ALG_ARMIJO : ALG_DOGLEG;
    int32_t* const out = stage == 0 ? sc.sel1 : sc.sel2;
    const int32_t* in = stage == 0 ? a.sys : sc.sel1;
    const int64_t* in_count = stage == 0 ? nullptr : sc.cnt;
    if (int z = launch_poly_select(in, in_count, a.count, a.retcode, out, sc.cnt + stage, st); z < 0) return z;
    KArgs b = a;
    b.sys = out;
    b.count_dev = sc.cnt + stage;
    b.counter = sc.cnt + 2 + stage;
    b.u_out = sc.u_t;
    b.fnorm = sc.fnorm_t;
    b.iters = sc.iters_t;
    b.retcode = sc.retcode_t;
    b.nfev = a.nfev ? sc.nfev_t : nullptr;
    b.njev = a.njev ? sc.njev_t : nullptr;
    if (int z = launch(key_n, lane, fam, alg, prec, b, st); z != 0) return z;
    PolyMergeArgs m{};
    m.list = out;
    m.count = sc.cnt + stage;
    m.cap = a.count;
    m.nsys = a.nsys;
    m.n = a.n;
    m.u_off = a.u_off;
    m.u = a.u_out;
    m.fnorm = a.fnorm;
    m.iters = a.iters;
    m.retcode = a.retcode;
    m.nfev = a.nfev;
    m.njev = a.njev;
    m.u_t = sc.u_t;
    m.fnorm_t = sc.fnorm_t;
    m.iters_t = sc.iters_t;
    m.retcode_t = sc.retcode_t;
    m.nfev_t = b.nfev;
    m.njev_t = b.njev;
    if (int z = launch_poly_merge(m, st); z < 0) return z;
  }
  return 0;
}

}  // namespace rt
}  // namespace nls

namespace {

// dense index of an (n, family, algorithm) combination (POLY included)
constexpr int kCombos = NLS_NMAX * FAM_COUNT * ALG_KEYS;
inline int combo_index(int n, int fam, int alg) { return ((n - 1) * FAM_COUNT + fam) * ALG_KEYS + alg; }
inline void combo_split(int ci, int* n, int* fam, int* alg) {
  *alg = ci % ALG_KEYS;
  *fam = (ci / ALG_KEYS) % FAM_COUNT;
  *n = ci / (ALG_KEYS * FAM_COUNT) + 1;
}

struct Launch {
  KArgs a;
  bool lane;
  int key_n, fam, alg;
  double cost;  // estimated work (sum of n^3) for branch balancing
  bool poly = false;  // the Newton stage of POLY systems
};

// The Newton-stage launch of a group of POLY systems; its later stages reuse
// the launch's kernel mapping and system list.
struct PolySeg {
  KArgs a;
  bool lane;
  int key_n, fam;
};

struct DevBuf {
  std::vector<void*>* list;
  uint64_t* bytes;
  hipError_t alloc(void** p, size_t n) {
    if (n == 0) n = 8;
    hipError_t e = hipMalloc(p, n);
    if (e == hipSuccess) {
      list->push_back(*p);
      *bytes += n;
    }
    return e;
  }
};

int tune_key(int n, int fam, int alg, int prec) { return ((n * FAM_COUNT + fam) * ALG_KEYS + alg) * 2 + prec; }

void save_tuning(nls_context* c, int key, int choice) {
  if (c->tune_cache_path.empty()) return;
  if (FILE* f = std::fopen(c->tune_cache_path.c_str(), "a")) {
    std::fprintf(f, "%d %d\n", key, choice);
    std::fclose(f);
  }
}

void load_tuning(nls_context* c) {
  if (c->tune_cache_path.empty()) return;
  if (FILE* f = std::fopen(c->tune_cache_path.c_str(), "r")) {
    int k = 0, v = 0;
    while (std::fscanf(f, "%d %d", &k, &v) == 2)
      if (v >= 1 && v <= 4) c->tuned[k] = v;
    std::fclose(f);
  }
}

// NLS_GROUP_ROWS as the group kernels read it (1 = one row per lane)
static int group_rows_env() {
  const char* e = std::getenv("NLS_GROUP_ROWS");
  return e ? std::atoi(e) : 0;
}

// Whether the two-rows-per-lane group kernels exist for a combination (the
// n <= 16 bucket; dense families; Newton, Armijo, dogleg, and the chain,
// whose stages are those three).
static bool two_rows_ok(int n, int fam, int alg) {
  return n <= 16 && (fam == FAM_CUBIC || fam == FAM_TANH) && alg != ALG_POTRA;
}

// Kernel mapping for a bucket.  Without NLS_CTX_AUTOTUNE the choice is fixed:
// one system per lane for n <= 8, else one system per group (8 lanes with two
// rows each up to n = 16 where those kernels exist, else 16/32/64 lanes with
// one row each).  With it, the first batch that holds the combination times
// every mapping with a kernel for it -- one system per lane; per group of 8
// lanes with two rows each; per group of 16 lanes with one row each -- on up
// to 32,768 of its systems (results land in the output buffers and are
// overwritten by the real solve), and keeps the fastest for the life of the
// context (and in the file named by NLS_AUTOTUNE_CACHE), so the mapping never
// depends on batch composition.
Mapping choose_mapping(nls_context* c, int n, int fam, int alg, int prec, KArgs a, int64_t P, int64_t count,
                       const int32_t* sys, const int64_t* p_off) {
  const Mapping lane{true, n, hipSuccess, 0};
  const Mapping group{false, group_bucket(n), hipSuccess, 0};
  const Mapping one{false, group_bucket(n), hipSuccess, 1};
  const Mapping two{false, group_bucket(n), hipSuccess, 2};
  const bool rows2 = two_rows_ok(n, fam, alg);
  // tuned codes: 1 lane, 2 group (default rows), 3 one row per lane, 4 two rows per lane
  auto of = [&](int v) { return v == 1 ? lane : (v == 3 ? one : (v == 4 && rows2 ? two : group)); };
  if (n > 16) return group;
  const bool lane_ok = n <= 8 && !(fam == FAM_ROSENBROCK && n < 2);
  if (n <= 8 && (fam == FAM_PAPER || (fam == FAM_ROSENBROCK && n < 2))) return lane;
  if (n <= 8 && c->forced) return c->forced == 1 ? lane : group;
  if (!(c->flags & NLS_CTX_AUTOTUNE)) return n <= 8 ? lane : group;
  if (!lane_ok && !rows2) return group;
  const int key = tune_key(n, fam, alg, prec);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) return of(it->second);
  // a sample large enough to fill the device with every candidate (the
  // two-row groups hold eight systems per wavefront), so the timing reflects
  // throughput and not the parallelism of a small sample
  a.count = count < 32768 ? count : 32768;
  a.P = P;
  a.sys = sys;
  a.p_off = p_off;
  a.counter = nullptr;
  const int codes[3] = {1, 4, 3};
  float ms[3] = {0.f, 0.f, 0.f};
  hipEvent_t e0, e1;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return Mapping{true, n, e, 0};
  if ((e = hipEventCreate(&e1)) != hipSuccess) { hipEventDestroy(e0); return Mapping{true, n, e, 0}; }
  int best = -1;
  for (int cand = 0; cand < 3; ++cand) {
    if ((cand == 0 && !lane_ok) || (cand == 1 && !rows2)) continue;
    const Mapping mp = of(codes[cand]);
    KArgs t = a;
    t.n = n;
    t.rows = mp.rows;
    for (int rep = 0; rep < 2; ++rep) {  // the first run loads the code object
      hipEventRecord(e0, c->stream);
      int rc = launch(mp.key_n, mp.lane, fam, alg, prec, t, c->stream);
      hipEventRecord(e1, c->stream);
      if (rc < 0) { hipEventDestroy(e0); hipEventDestroy(e1); return Mapping{true, n, (hipError_t)(-rc), 0}; }
      if ((e = hipEventSynchronize(e1)) != hipSuccess) { hipEventDestroy(e0); hipEventDestroy(e1); return Mapping{true, n, e, 0}; }
      hipEventElapsedTime(&ms[cand], e0, e1);
    }
    if (best < 0 || ms[cand] < ms[best]) best = cand;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  c->tuned[key] = codes[best];
  save_tuning(c, key, codes[best]);
  return of(codes[best]);
}

// Run a list of persistent launches.  One launch goes straight onto the
// stream; several are captured into one graph whose branches (at most four,
// balanced by estimated work) run concurrently, and the graph is replayed
// while the launch list stays the same.  Counters are zeroed by a kernel
// inside the graph (no memset nodes).
int run_launches(nls_context* c, std::vector<Launch>& L, int prec) {
  const int nl = (int)L.size();
  if (nl == 0) return 0;
  const bool use_graph = nl > 1 && !std::getenv("NLS_NO_GRAPH");
  if (!use_graph) {
    if (int z = launch_zero_counters(c->counters, nl, c->stream); z < 0) return z;
    for (auto& x : L) {
      int rc = launch(x.key_n, x.lane, x.fam, x.alg, prec, x.a, c->stream);
      if (rc != 0) return rc;
    }
    return 0;
  }
  // signature: every launch's kernel identity and arguments
  std::string sig;
  sig.reserve(nl * (sizeof(KArgs) + 16) + 4);
  sig.append((const char*)&prec, sizeof prec);
  for (auto& x : L) {
    sig.append((const char*)&x.a, sizeof(KArgs));
    int id[4] = {x.lane ? 1 : 0, x.key_n, x.fam, x.alg};
    sig.append((const char*)id, sizeof id);
  }
  if (c->graph_exec && sig == c->graph_sig) {
    hipError_t e = hipGraphLaunch(c->graph_exec, c->stream);
    return e == hipSuccess ? 0 : -(int)e;
  }
  // branch assignment: longest work first, onto the least-loaded branch
  std::vector<int> idx(nl);
  for (int i = 0; i < nl; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return L[x].cost > L[y].cost; });
  const int nb = std::min(nl, (int)nls_context::kBranches);
  std::vector<double> load(nb, 0.0);
  std::vector<std::vector<int>> br(nb);
  for (int i : idx) {
    int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    br[j].push_back(i);
    load[j] += L[i].cost;
  }
  hipError_t e;
  hipGraph_t g = nullptr;
  if ((e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed)) != hipSuccess) return -(int)e;
  int rc = launch_zero_counters(c->counters, nl, c->stream);
  if (rc == 0 && (e = hipEventRecord(c->fork_ev, c->stream)) != hipSuccess) rc = -(int)e;
  for (int j = 0; j < nb && rc == 0; ++j) {
    if ((e = hipStreamWaitEvent(c->branch[j], c->fork_ev, 0)) != hipSuccess) { rc = -(int)e; break; }
    for (int i : br[j]) {
      rc = launch(L[i].key_n, L[i].lane, L[i].fam, L[i].alg, prec, L[i].a, c->branch[j]);
      if (rc != 0) break;
    }
    if (rc == 0 && (e = hipEventRecord(c->join_ev[j], c->branch[j])) != hipSuccess) rc = -(int)e;
    if (rc == 0 && (e = hipStreamWaitEvent(c->stream, c->join_ev[j], 0)) != hipSuccess) rc = -(int)e;
  }
  e = hipStreamEndCapture(c->stream, &g);
  if (rc != 0) { if (g) hipGraphDestroy(g); return rc; }
  if (e != hipSuccess) return -(int)e;
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) return -(int)e;
  if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
  c->graph_exec = ex;
  c->graph_sig.swap(sig);
  e = hipGraphLaunch(c->graph_exec, c->stream);
  return e == hipSuccess ? 0 : -(int)e;
}

// The fallback chain of Sec. 3.2 for POLY systems, once the Newton stage has
// written the results: per segment (one Newton-stage launch), run_chain
// gathers the systems it left unsolved on the device, solves them again from
// u0 with Newton + Armijo into scratch outputs, folds the attempt into the
// results, and gives those still unsolved the dogleg stage.  Every step is a
// kernel on the context's stream and the host never reads a count.
int run_poly(nls_context* c, const std::vector<PolySeg>& segs, int prec, DevBuf& db, int64_t M, int64_t utotal) {
  const int ns = (int)segs.size();
  if (ns == 0) return 0;
  int64_t lists = 0;
  for (auto& g : segs) lists += g.a.count;
  const KArgs& r = segs[0].a;  // every segment writes the same result arrays
  void *sel1, *sel2, *cnt, *ut, *fnt, *itt, *rct, *nft = nullptr, *njt = nullptr;
  hipError_t e;
  if ((e = db.alloc(&sel1, lists * 4)) != hipSuccess) return -(int)e;
  if ((e = db.alloc(&sel2, lists * 4)) != hipSuccess) return -(int)e;
  if ((e = db.alloc(&cnt, (size_t)ns * 4 * 8)) != hipSuccess) return -(int)e;
  if ((e = db.alloc(&ut, utotal * 8)) != hipSuccess) return -(int)e;
  if ((e = db.alloc(&fnt, M * 8)) != hipSuccess) return -(int)e;
  if ((e = db.alloc(&itt, M * 4)) != hipSuccess) return -(int)e;
  if ((e = db.alloc(&rct, M * 4)) != hipSuccess) return -(int)e;
  if (r.nfev && (e = db.alloc(&nft, M * 4)) != hipSuccess) return -(int)e;
  if (r.njev && (e = db.alloc(&njt, M * 4)) != hipSuccess) return -(int)e;
  // segments hold disjoint systems, so they share the scratch outputs
  int64_t at = 0;
  for (int k = 0; k < ns; ++k) {
    ChainScratch sc{(int32_t*)sel1 + at, (int32_t*)sel2 + at, (int64_t*)cnt + 4 * k, (double*)ut,
                    (double*)fnt, (int32_t*)itt, (int32_t*)rct, (int32_t*)nft, (int32_t*)njt};
    const int z = run_chain(segs[k].a, segs[k].lane, segs[k].key_n, segs[k].fam, prec, sc, c->stream);
    if (z != 0) return z;
    at += segs[k].a.count;
  }
  return 0;
}

}  // namespace

extern "C" {

int nls_abi_version(void) { return NLS_ABI_VERSION; }

int nls_nparams(int family, int n) { return nparams_of(family, n); }

int nls_get_mapping(const nls_context* c, int family, int n, int alg, int precision, int32_t* lanes_per_system) {
  if (!c || !lanes_per_system) return fail(nullptr, NLS_E_INVALID, "nls_get_mapping: NULL argument");
  if (!supported(family, n) || alg < 0 || alg >= ALG_KEYS || (precision != 0 && precision != 1))
    return fail(nullptr, NLS_E_INVALID, "nls_get_mapping: bad combination");
  if (alg == ALG_POLY) alg = ALG_NEWTON;  // every stage of the chain runs on the Newton stage's mapping
  const bool rows2 = two_rows_ok(n, family, alg);
  // lanes per system of the group mapping with its default rows per lane (two
  // in both forms, unless NLS_GROUP_ROWS says)
  const int env_rows = group_rows_env();
  const int def_rows = (env_rows == 1 || env_rows == 2) ? env_rows : 2;
  const int group_l = n <= 16 ? (rows2 && def_rows == 2 ? 8 : 16) : (n <= 32 ? 32 : 64);
  if (n > 16) { *lanes_per_system = group_l; return NLS_OK; }
  if (n <= 8 && (family == FAM_PAPER || (family == FAM_ROSENBROCK && n < 2))) { *lanes_per_system = 1; return NLS_OK; }
  if (n <= 8 && c->forced) { *lanes_per_system = c->forced == 1 ? 1 : group_l; return NLS_OK; }
  if (!(c->flags & NLS_CTX_AUTOTUNE)) { *lanes_per_system = n <= 8 ? 1 : group_l; return NLS_OK; }
  if (!(n <= 8 && !(family == FAM_ROSENBROCK && n < 2)) && !rows2) { *lanes_per_system = group_l; return NLS_OK; }
  auto it = c->tuned.find(tune_key(n, family, alg, precision));
  if (it == c->tuned.end()) { *lanes_per_system = 0; return NLS_OK; }
  const int v = it->second;
  *lanes_per_system = v == 1 ? 1 : (v == 3 ? 16 : (v == 4 ? 8 : group_l));
  return NLS_OK;
}

void nls_default_options(nls_alg_options* o) {
  if (o) fill_defaults(o);
}

const char* nls_last_error(const nls_context* c) {
  if (c) return c->last_error.c_str();
  return thread_error();
}

int nls_validate(const nls_batch* b, int64_t* first_bad) {
  std::string m = validate(b, first_bad);
  if (!m.empty()) return fail(nullptr, NLS_E_INVALID, m);
  return NLS_OK;
}

int nls_create(const nls_context_desc* d, nls_context** out) {
  if (!d || !out) return fail(nullptr, NLS_E_INVALID, "nls_create: NULL argument");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
  if (d->device < 0 || d->device >= ndev) return fail(nullptr, NLS_E_INVALID, "nls_create: bad device ordinal");
  e = hipSetDevice(d->device);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
  nls_context* c = new nls_context();
  c->device = d->device;
  c->flags = d->flags;
  c->budget = d->mem_budget_bytes;
  if (d->stream) {
    c->stream = (hipStream_t)d->stream;
  } else {
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return hip_fail(nullptr, e, "hipStreamCreate");
    }
    c->own_stream = true;
  }
  c->ncounters = 512;
  e = hipMalloc((void**)&c->counters, sizeof(int64_t) * c->ncounters);
  for (int j = 0; e == hipSuccess && j < nls_context::kBranches; ++j) {
    e = hipStreamCreateWithFlags(&c->branch[j], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join_ev[j], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->plan_ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    nls_destroy(c);
    return hip_fail(nullptr, e, "nls_create");
  }
  if (const char* tc = std::getenv("NLS_AUTOTUNE_CACHE")) c->tune_cache_path = tc;
  if (const char* fm = std::getenv("NLS_MAPPING")) c->forced = std::strcmp(fm, "group") == 0 ? 2 : (std::strcmp(fm, "lane") == 0 ? 1 : 0);
  load_tuning(c);
  *out = c;
  return NLS_OK;
}

static void release_ticket(Ticket& t, nls_context* c) {
  for (void* p : t.device_allocs) hipFree(p);
  t.device_allocs.clear();
  if (t.start) hipEventDestroy(t.start);
  if (t.stop) hipEventDestroy(t.stop);
  t.start = t.stop = nullptr;
  (void)c;
}

int nls_destroy(nls_context* c) {
  if (!c) return NLS_OK;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  for (auto& kv : c->tickets) release_ticket(kv.second, c);
  c->tickets.clear();
  if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
  for (int j = 0; j < nls_context::kBranches; ++j) {
    if (c->branch[j]) hipStreamDestroy(c->branch[j]);
    if (c->join_ev[j]) hipEventDestroy(c->join_ev[j]);
  }
  if (c->fork_ev) hipEventDestroy(c->fork_ev);
  if (c->counters) hipFree(c->counters);
  if (c->plan_dev) hipFree(c->plan_dev);
  if (c->plan_host) hipHostFree(c->plan_host);
  if (c->plan_ev) hipEventDestroy(c->plan_ev);
  if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
  delete c;
  return NLS_OK;
}

int nls_solve_batch(nls_context* c, const nls_batch* b, const nls_results* r, uint64_t* ticket) {
  if (!c) return fail(nullptr, NLS_E_INVALID, "context is NULL");
  std::unique_lock<std::mutex> lk(c->mu, std::defer_lock);
  if (c->flags & NLS_CTX_THREADSAFE) lk.lock();
  if (!ticket) return fail(c, NLS_E_INVALID, "ticket is NULL");
  int64_t bad = -1;
  std::string m = validate(b, &bad);
  if (m.empty()) m = check_results(r, b->count);
  if (!m.empty()) return fail(c, NLS_E_INVALID, m);

  const int64_t M = b->count;
  const bool dev = b->mem_kind == NLS_MEM_DEVICE;
  nls_alg_options opts;
  fill_defaults(&opts);
  if (b->opts) opts = *b->opts;

  // --- plan: uniform fast path or buckets ---------------------------------
  int fam0, n0, alg0;
  const bool uniform = uniform_batch(b, &fam0, &n0, &alg0);
  const int P0 = nparams_of(fam0, n0);
  // total payload extents
  int64_t ptotal = 0, utotal = 0, npoly = 0;
  if (uniform) {
    ptotal = M * (int64_t)P0;
    utotal = M * (int64_t)n0;
    npoly = alg0 == ALG_POLY ? M : 0;
  } else {
    for (int64_t s = 0; s < M; ++s) {
      const int fam = b->family ? b->family[s] : b->family_all;
      const int n = b->n ? b->n[s] : b->n_all;
      npoly += (b->alg ? b->alg[s] : b->alg_all) == ALG_POLY;
      const int64_t pe = (b->p_offset ? b->p_offset[s] : ptotal) + nparams_of(fam, n);
      const int64_t ue = (b->u_offset ? b->u_offset[s] : utotal) + n;
      if (b->p_offset) ptotal = std::max(ptotal, pe); else ptotal = pe;
      if (b->u_offset) utotal = std::max(utotal, ue); else utotal = ue;
    }
    // the extents run to the final offsets, so gaps inside the last span are
    // staged (and, for u, returned) like every other gap
    if (b->p_offset) ptotal = std::max(ptotal, b->p_offset[M]);
    if (b->u_offset) utotal = std::max(utotal, b->u_offset[M]);
  }

  // device footprint of this call (library-owned memory only)
  uint64_t need = 0;
  if (!dev) need += (uint64_t)(ptotal + 2 * utotal + M) * 8 + (uint64_t)M * 16;
  if (!uniform) need += (uint64_t)M * (4 + 1 + 16) + 16;
  // the chain's lists, counts and scratch outputs
  if (npoly) need += (uint64_t)npoly * 8 + (uint64_t)utotal * 8 + (uint64_t)M * 24 + 4 * 8 * kCombos;
  if (c->budget && c->held_bytes + need > c->budget) {
    if (need > c->budget) return fail(c, NLS_E_NOMEM, "batch needs more device memory than the budget");
    return fail(c, NLS_E_NOMEM, "budget exhausted by outstanding tickets; query them first");
  }

  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");

  Ticket t;
  t.systems = M;
  uint64_t held = 0;
  DevBuf db{&t.device_allocs, &held};
  auto bail = [&](hipError_t err, const char* what) {
    hipStreamSynchronize(c->stream);
    release_ticket(t, c);
    return hip_fail(c, err, what);
  };
  if ((e = hipEventCreate(&t.start)) != hipSuccess) return bail(e, "hipEventCreate");
  if ((e = hipEventCreate(&t.stop)) != hipSuccess) return bail(e, "hipEventCreate");
  if ((e = hipEventRecord(t.start, c->stream)) != hipSuccess) return bail(e, "hipEventRecord");

  const double* d_params = b->params;
  const double* d_u0 = b->u0;
  double* d_u = r ? r->u : nullptr;
  double* d_fn = r ? r->fnorm_inf : nullptr;
  int32_t* d_it = r ? r->iters : nullptr;
  int32_t* d_rc = r ? r->retcode : nullptr;
  int32_t* d_nfev = r ? r->nfev : nullptr;
  int32_t* d_njev = r ? r->njev : nullptr;

  if (M > 0 && !dev) {
    void *pp = nullptr, *pu0 = nullptr, *pu = nullptr, *pfn = nullptr, *pit = nullptr, *prc = nullptr;
    void *pnf = nullptr, *pnj = nullptr;
    if ((e = db.alloc(&pp, ptotal * 8)) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = db.alloc(&pu0, utotal * 8)) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = db.alloc(&pu, utotal * 8)) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = db.alloc(&pfn, M * 8)) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = db.alloc(&pit, M * 4)) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = db.alloc(&prc, M * 4)) != hipSuccess) return bail(e, "hipMalloc");
    if (r->nfev && (e = db.alloc(&pnf, M * 4)) != hipSuccess) return bail(e, "hipMalloc");
    if (r->njev && (e = db.alloc(&pnj, M * 4)) != hipSuccess) return bail(e, "hipMalloc");
    if (ptotal && (e = hipMemcpyAsync(pp, b->params, ptotal * 8, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    if ((e = hipMemcpyAsync(pu0, b->u0, utotal * 8, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    // u keeps the caller's layout: start from u0 so that gaps between systems survive
    if ((e = hipMemcpyAsync(pu, b->u0, utotal * 8, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    d_params = (const double*)pp;
    d_u0 = (const double*)pu0;
    d_u = (double*)pu;
    d_fn = (double*)pfn;
    d_it = (int32_t*)pit;
    d_rc = (int32_t*)prc;
    d_nfev = (int32_t*)pnf;
    d_njev = (int32_t*)pnj;
  }

  KArgs base{};
  base.params = d_params;
  base.u0 = d_u0;
  base.u_out = d_u;
  base.fnorm = d_fn;
  base.iters = d_it;
  base.retcode = d_rc;
  base.nfev = d_nfev;
  base.njev = d_njev;
  base.maxiters = b->maxiters;
  base.abstol = b->abstol;
  base.o = to_kopts(opts);

  if (M > 0 && uniform) {
    const int alg1 = alg0 == ALG_POLY ? ALG_NEWTON : alg0;  // the chain starts with Newton
    const Mapping mp = choose_mapping(c, n0, fam0, alg1, b->precision, base, P0, M, nullptr, nullptr);
    if (mp.error) return bail(mp.error, "autotune");
    if (int z = launch_zero_counters(c->counters, 1, c->stream); z < 0) return bail((hipError_t)(-z), "zero counters");
    KArgs a = base;
    a.count = M;
    a.P = P0;
    a.n = n0;
    a.counter = c->counters;
    a.rows = mp.rows;
    int rcode = launch(mp.key_n, mp.lane, fam0, alg1, b->precision, a, c->stream);
    if (rcode < 0) return bail((hipError_t)(-rcode), "kernel launch");
    if (rcode > 0) return fail(c, NLS_E_INVALID, "no kernel for this family/size/algorithm");
    if (alg0 == ALG_POLY) {
      std::vector<PolySeg> segs{PolySeg{a, mp.lane, mp.key_n, fam0}};
      rcode = run_poly(c, segs, b->precision, db, M, utotal);
      if (rcode < 0) return bail((hipError_t)(-rcode), "fallback chain");
      if (rcode > 0) return fail(c, NLS_E_INVALID, "no kernel for this family/size/algorithm");
    }
  } else if (M > 0) {
    // Bucket by kernel: counting sort of the systems on a dense key
    // (mapping, size bucket, family, algorithm), one persistent launch per
    // bucket, all captured in one graph with parallel branches.  The plan is
    // written into the context's pinned mirror and copied to its device
    // buffer on the stream (no allocation and no wait in the common case).
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t o_sys = 0, o_po = al(M * 4), o_uo = o_po + al((M + 1) * 8), o_n = o_uo + al((M + 1) * 8);
    const size_t plan_bytes = o_n + al(M);
    if (plan_bytes > c->plan_cap) {
      // grow (rare): earlier calls may still read the old buffers
      if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return bail(e, "hipStreamSynchronize");
      if (c->plan_dev) hipFree(c->plan_dev);
      if (c->plan_host) hipHostFree(c->plan_host);
      c->plan_dev = c->plan_host = nullptr;
      c->plan_cap = 0;
      c->plan_ev_pending = false;
      const size_t cap = plan_bytes + plan_bytes / 4;
      if ((e = hipMalloc((void**)&c->plan_dev, cap)) != hipSuccess) return bail(e, "hipMalloc");
      if ((e = hipHostMalloc((void**)&c->plan_host, cap, hipHostMallocDefault)) != hipSuccess) {
        hipFree(c->plan_dev);
        c->plan_dev = nullptr;
        return bail(e, "hipHostMalloc");
      }
      c->plan_cap = cap;
    }
    // the previous call's copy out of the mirror has finished before it is rewritten
    if (c->plan_ev_pending && (e = hipEventSynchronize(c->plan_ev)) != hipSuccess)
      return bail(e, "hipEventSynchronize");
    int32_t* order = reinterpret_cast<int32_t*>(c->plan_host + o_sys);
    int64_t* poff = reinterpret_cast<int64_t*>(c->plan_host + o_po);
    int64_t* uoff = reinterpret_cast<int64_t*>(c->plan_host + o_uo);
    uint8_t* nn = reinterpret_cast<uint8_t*>(c->plan_host + o_n);
    std::vector<uint16_t> key(M);
    int64_t pacc = 0, uacc = 0;
    for (int64_t s = 0; s < M; ++s) {
      const int fam = b->family ? b->family[s] : b->family_all;
      const int n = b->n ? b->n[s] : b->n_all;
      const int alg = b->alg ? b->alg[s] : b->alg_all;
      poff[s] = b->p_offset ? b->p_offset[s] : pacc;
      uoff[s] = b->u_offset ? b->u_offset[s] : uacc;
      pacc = poff[s] + nparams_of(fam, n);
      uacc = uoff[s] + n;
      nn[s] = (uint8_t)n;
      key[s] = (uint16_t)combo_index(n, fam, alg);
    }
    poff[M] = pacc;
    uoff[M] = uacc;
    // systems per (n, family, algorithm) combination, in input order
    std::vector<int64_t> cnt(kCombos + 1, 0);
    for (int64_t s = 0; s < M; ++s) cnt[key[s] + 1]++;
    for (int i = 0; i < kCombos; ++i) cnt[i + 1] += cnt[i];
    {
      std::vector<int64_t> at(cnt.begin(), cnt.end() - 1);
      for (int64_t s = 0; s < M; ++s) order[at[key[s]]++] = (int32_t)s;
    }
    if ((e = hipMemcpyAsync(c->plan_dev, c->plan_host, plan_bytes, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    if ((e = hipEventRecord(c->plan_ev, c->stream)) != hipSuccess) return bail(e, "hipEventRecord");
    c->plan_ev_pending = true;
    void* dsys = c->plan_dev + o_sys;
    void* dpo = c->plan_dev + o_po;
    void* duo = c->plan_dev + o_uo;
    void* dn = c->plan_dev + o_n;
    // one launch per kernel: combinations that map to the same group bucket
    // share it (their n rides along in nsys)
    std::vector<Launch> launches;
    std::map<int, size_t> by_kernel;
    for (int ci = 0; ci < kCombos; ++ci) {
      const int64_t c0 = cnt[ci], c1 = cnt[ci + 1];
      if (c1 == c0) continue;
      int n, fam, alg;
      combo_split(ci, &n, &fam, &alg);
      KArgs a = base;
      a.sys = (const int32_t*)dsys + c0;
      a.p_off = (const int64_t*)dpo;
      a.u_off = (const int64_t*)duo;
      a.nsys = (const uint8_t*)dn;
      a.count = c1 - c0;
      a.P = 0;
      const bool poly = alg == ALG_POLY;
      const int alg1 = poly ? ALG_NEWTON : alg;  // the chain starts with Newton
      const Mapping mp = choose_mapping(c, n, fam, alg1, b->precision, a, 0, c1 - c0, a.sys, a.p_off);
      if (mp.error) return bail(mp.error, "autotune");
      const int kid = (mp.lane ? 0 : 100000 * (1 + mp.rows)) + mp.key_n * 64 + fam * ALG_KEYS + alg;
      auto it = by_kernel.find(kid);
      if (it != by_kernel.end() && !mp.lane && launches[it->second].a.sys + launches[it->second].a.count == a.sys) {
        launches[it->second].a.count += a.count;  // adjacent in the sorted order
        launches[it->second].cost += (double)a.count * n * n * n;
        continue;
      }
      a.n = mp.key_n;
      a.rows = mp.rows;
      Launch L{a, mp.lane, mp.key_n, fam, alg1, (double)a.count * n * n * n, poly};
      by_kernel[kid] = launches.size();
      launches.push_back(L);
    }
    if ((int)launches.size() > c->ncounters) return fail(c, NLS_E_INVALID, "too many kernels");
    for (size_t i = 0; i < launches.size(); ++i) launches[i].a.counter = c->counters + i;
    int rcode = run_launches(c, launches, b->precision);
    if (rcode < 0) return bail((hipError_t)(-rcode), "kernel launch");
    if (rcode > 0) return fail(c, NLS_E_INVALID, "no kernel for this family/size/algorithm");
    std::vector<PolySeg> segs;
    for (auto& x : launches)
      if (x.poly) segs.push_back(PolySeg{x.a, x.lane, x.key_n, x.fam});
    rcode = run_poly(c, segs, b->precision, db, M, utotal);
    if (rcode < 0) return bail((hipError_t)(-rcode), "fallback chain");
    if (rcode > 0) return fail(c, NLS_E_INVALID, "no kernel for this family/size/algorithm");
  }

  if (M > 0 && !dev) {
    if ((e = hipMemcpyAsync(r->u, d_u, utotal * 8, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    if ((e = hipMemcpyAsync(r->fnorm_inf, d_fn, M * 8, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    if ((e = hipMemcpyAsync(r->iters, d_it, M * 4, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    if ((e = hipMemcpyAsync(r->retcode, d_rc, M * 4, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    if (r->nfev && (e = hipMemcpyAsync(r->nfev, d_nfev, M * 4, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    if (r->njev && (e = hipMemcpyAsync(r->njev, d_njev, M * 4, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
  }
  if ((e = hipEventRecord(t.stop, c->stream)) != hipSuccess) return bail(e, "hipEventRecord");
  if (!dev) {
    // host payloads: inputs were read from caller memory; make the call
    // synchronous so that the caller may reuse its buffers at once
    if ((e = hipEventSynchronize(t.stop)) != hipSuccess) return bail(e, "hipEventSynchronize");
  }
  const uint64_t id = c->next_ticket++;
  t.bytes = held;
  c->held_bytes += held;
  c->tickets.emplace(id, std::move(t));
  *ticket = id;
  return NLS_OK;
}

int nls_query(nls_context* c, uint64_t ticket, int32_t wait_ms, nls_ticket_info* info) {
  if (!c) return fail(nullptr, NLS_E_INVALID, "context is NULL");
  std::unique_lock<std::mutex> lk(c->mu, std::defer_lock);
  if (c->flags & NLS_CTX_THREADSAFE) lk.lock();
  auto it = c->tickets.find(ticket);
  if (it == c->tickets.end()) return fail(c, NLS_E_NOTFOUND, "unknown ticket");
  Ticket& t = it->second;
  hipSetDevice(c->device);
  hipError_t e = hipEventQuery(t.stop);
  if (e == hipErrorNotReady) {
    if (wait_ms == 0) return NLS_PENDING;
    if (wait_ms < 0) {
      e = hipEventSynchronize(t.stop);
    } else {
      auto until = std::chrono::steady_clock::now() + std::chrono::milliseconds(wait_ms);
      while ((e = hipEventQuery(t.stop)) == hipErrorNotReady) {
        if (std::chrono::steady_clock::now() >= until) return NLS_PENDING;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
      }
    }
  }
  int32_t status = NLS_OK;
  float ms = 0.f;
  if (e != hipSuccess) {
    status = NLS_E_DEVICE;
    c->last_error = std::string("ticket failed: ") + hipGetErrorString(e);
  } else {
    hipEventElapsedTime(&ms, t.start, t.stop);
  }
  if (info) {
    info->done = 1;
    info->status = status;
    info->gpu_ms = ms;
    info->systems = t.systems;
  }
  c->held_bytes -= std::min(c->held_bytes, t.bytes);
  release_ticket(t, c);
  c->tickets.erase(it);
  return status == NLS_OK ? NLS_OK : NLS_E_DEVICE;
}

// Sensitivities at a solution: validation, payload staging and one launch
// per (family, size bucket).
static std::string validate_sens(const nls_sens_batch* b, const nls_sens_results* r, int64_t* ptotal,
                                 int64_t* utotal) {
  *ptotal = *utotal = 0;
  if (!b) return "batch is NULL";
  if (b->count < 0) return "count must be >= 0";
  if (b->count > (int64_t)INT32_MAX) return "count exceeds 2^31 - 1";
  if (b->mode != NLS_SENS_TANGENT && b->mode != NLS_SENS_ADJOINT) return "unknown sensitivity mode";
  if (b->mem_kind != NLS_MEM_HOST && b->mem_kind != NLS_MEM_DEVICE) return "unknown mem_kind";
  const int64_t M = b->count;
  if (M == 0) return "";
  int64_t pacc = 0, uacc = 0;
  for (int64_t s = 0; s < M; ++s) {
    const int fam = b->family ? b->family[s] : b->family_all;
    const int n = b->n ? b->n[s] : b->n_all;
    char buf[160];
    if (n < 1 || n > NLS_NMAX) {
      std::snprintf(buf, sizeof buf, "system %lld: n = %d outside [1, 64]", (long long)s, n);
      return buf;
    }
    if (fam < 0 || fam >= FAM_COUNT || !supported(fam, n)) {
      std::snprintf(buf, sizeof buf, "system %lld: family %d is not defined at n = %d", (long long)s, fam, n);
      return buf;
    }
    const int P = nparams_of(fam, n);
    const int64_t po = b->p_offset ? b->p_offset[s] : pacc;
    const int64_t uo = b->u_offset ? b->u_offset[s] : uacc;
    if (b->p_offset && (po < 0 || b->p_offset[s + 1] - po < P)) {
      std::snprintf(buf, sizeof buf, "system %lld: p_offset span shorter than %d parameters", (long long)s, P);
      return buf;
    }
    if (b->u_offset && (uo < 0 || b->u_offset[s + 1] - uo < n)) {
      std::snprintf(buf, sizeof buf, "system %lld: u_offset span shorter than n = %d", (long long)s, n);
      return buf;
    }
    pacc = po + P;
    uacc = uo + n;
    *ptotal = std::max(*ptotal, pacc);
    *utotal = std::max(*utotal, uacc);
  }
  if (b->p_offset) *ptotal = std::max(*ptotal, b->p_offset[M]);
  if (b->u_offset) *utotal = std::max(*utotal, b->u_offset[M]);
  const bool tangent = b->mode == NLS_SENS_TANGENT;
  if (!b->u) return "u is NULL";
  if (*ptotal > 0 && !b->params) return "params is NULL";
  if ((tangent ? *ptotal : *utotal) > 0 && !b->seed) return "seed is NULL";
  if (!r) return "results is NULL";
  if (!r->status) return "status is NULL";
  if ((tangent ? *utotal : *ptotal) > 0 && !r->out) return "out is NULL";
  return "";
}

int nls_sensitivity_batch(nls_context* c, const nls_sens_batch* b, const nls_sens_results* r, uint64_t* ticket) {
  if (!c) return fail(nullptr, NLS_E_INVALID, "context is NULL");
  std::unique_lock<std::mutex> lk(c->mu, std::defer_lock);
  if (c->flags & NLS_CTX_THREADSAFE) lk.lock();
  if (!ticket) return fail(c, NLS_E_INVALID, "ticket is NULL");
  int64_t ptotal = 0, utotal = 0;
  const std::string m = validate_sens(b, r, &ptotal, &utotal);
  if (!m.empty()) return fail(c, NLS_E_INVALID, m);
  const int64_t M = b->count;
  const bool dev = b->mem_kind == NLS_MEM_DEVICE;
  const bool tangent = b->mode == NLS_SENS_TANGENT;
  const bool uniform = !b->family && !b->n && !b->p_offset && !b->u_offset;
  const int64_t seed_len = tangent ? ptotal : utotal, out_len = tangent ? utotal : ptotal;
  const bool want_lambda = !tangent && r->lambda;

  uint64_t need = 0;
  if (!dev) need += (uint64_t)(ptotal + utotal + seed_len + out_len + (want_lambda ? utotal : 0)) * 8 + M * 4;
  if (!uniform) need += (uint64_t)M * (4 + 1 + 16) + 16;
  if (c->budget && c->held_bytes + need > c->budget) {
    if (need > c->budget) return fail(c, NLS_E_NOMEM, "batch needs more device memory than the budget");
    return fail(c, NLS_E_NOMEM, "budget exhausted by outstanding tickets; query them first");
  }
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");

  Ticket t;
  t.systems = M;
  uint64_t held = 0;
  DevBuf db{&t.device_allocs, &held};
  auto bail = [&](hipError_t err, const char* what) {
    hipStreamSynchronize(c->stream);
    release_ticket(t, c);
    return hip_fail(c, err, what);
  };
  if ((e = hipEventCreate(&t.start)) != hipSuccess) return bail(e, "hipEventCreate");
  if ((e = hipEventCreate(&t.stop)) != hipSuccess) return bail(e, "hipEventCreate");
  if ((e = hipEventRecord(t.start, c->stream)) != hipSuccess) return bail(e, "hipEventRecord");

  SensArgs a{};
  a.params = b->params;
  a.u = b->u;
  a.seed = b->seed;
  a.out = r->out;
  a.lambda = want_lambda ? r->lambda : nullptr;
  a.status = r->status;
  if (M > 0 && !dev) {
    // stage the inputs; the outputs start from the caller's arrays so that
    // entries in offset gaps come back unchanged
    struct Stage { const void* src; void** dst; int64_t bytes; bool out; };
    void *pp = nullptr, *pu = nullptr, *ps = nullptr, *po = nullptr, *pl = nullptr, *pst = nullptr;
    const Stage st[] = {{b->params, &pp, ptotal * 8, false}, {b->u, &pu, utotal * 8, false},
                        {b->seed, &ps, seed_len * 8, false}, {r->out, &po, out_len * 8, true},
                        {want_lambda ? r->lambda : nullptr, &pl, want_lambda ? utotal * 8 : 0, true}};
    for (const Stage& x : st) {
      if (!x.src || x.bytes == 0) continue;
      if ((e = db.alloc(x.dst, x.bytes)) != hipSuccess) return bail(e, "hipMalloc");
      if ((e = hipMemcpyAsync(*x.dst, x.src, x.bytes, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
        return bail(e, "hipMemcpyAsync");
    }
    if ((e = db.alloc(&pst, M * 4)) != hipSuccess) return bail(e, "hipMalloc");
    a.params = (const double*)pp;
    a.u = (const double*)pu;
    a.seed = (const double*)ps;
    a.out = (double*)po;
    a.lambda = (double*)pl;
    a.status = (int32_t*)pst;
  }

  if (M > 0 && uniform) {
    a.count = M;
    a.n = b->n_all;
    a.P = nparams_of(b->family_all, b->n_all);
    const int rc = launch_sens(sens_bucket(b->n_all), b->family_all, b->mode, a, c->stream);
    if (rc < 0) return bail((hipError_t)(-rc), "kernel launch");
    if (rc > 0) return fail(c, NLS_E_INVALID, "no sensitivity kernel for this family/size");
  } else if (M > 0) {
    // counting sort on (family, size bucket); one launch per key
    constexpr int kKeys = FAM_COUNT * 8;
    std::vector<int64_t> poff(M + 1), uoff(M + 1);
    std::vector<uint8_t> nn(M), key(M);
    int64_t pacc = 0, uacc = 0;
    for (int64_t s = 0; s < M; ++s) {
      const int fam = b->family ? b->family[s] : b->family_all;
      const int n = b->n ? b->n[s] : b->n_all;
      poff[s] = b->p_offset ? b->p_offset[s] : pacc;
      uoff[s] = b->u_offset ? b->u_offset[s] : uacc;
      pacc = poff[s] + nparams_of(fam, n);
      uacc = uoff[s] + n;
      nn[s] = (uint8_t)n;
      key[s] = (uint8_t)(fam * 8 + sens_bucket(n) / 8 - 1);
    }
    poff[M] = pacc;
    uoff[M] = uacc;
    std::vector<int64_t> cnt(kKeys + 1, 0);
    for (int64_t s = 0; s < M; ++s) cnt[key[s] + 1]++;
    for (int i = 0; i < kKeys; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> order(M);
    {
      std::vector<int64_t> at(cnt.begin(), cnt.end() - 1);
      for (int64_t s = 0; s < M; ++s) order[at[key[s]]++] = (int32_t)s;
    }
    void *dsys = nullptr, *dpo = nullptr, *duo = nullptr, *dn = nullptr;
    if ((e = db.alloc(&dsys, M * 4)) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = db.alloc(&dpo, (M + 1) * 8)) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = db.alloc(&duo, (M + 1) * 8)) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = db.alloc(&dn, M)) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = hipMemcpyAsync(dsys, order.data(), M * 4, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    if ((e = hipMemcpyAsync(dpo, poff.data(), (M + 1) * 8, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    if ((e = hipMemcpyAsync(duo, uoff.data(), (M + 1) * 8, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    if ((e = hipMemcpyAsync(dn, nn.data(), M, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    // the host vectors die with this call: the copies complete first
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return bail(e, "hipStreamSynchronize");
    for (int k = 0; k < kKeys; ++k) {
      if (cnt[k + 1] == cnt[k]) continue;
      SensArgs x = a;
      x.sys = (const int32_t*)dsys + cnt[k];
      x.count = cnt[k + 1] - cnt[k];
      x.p_off = (const int64_t*)dpo;
      x.u_off = (const int64_t*)duo;
      x.nsys = (const uint8_t*)dn;
      x.P = 0;
      x.n = 0;
      const int rc = launch_sens((k % 8 + 1) * 8, k / 8, b->mode, x, c->stream);
      if (rc < 0) return bail((hipError_t)(-rc), "kernel launch");
      if (rc > 0) return fail(c, NLS_E_INVALID, "no sensitivity kernel for this family/size");
    }
  }

  if (M > 0 && !dev) {
    if (out_len && r->out &&
        (e = hipMemcpyAsync(r->out, a.out, out_len * 8, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
    if (want_lambda && (e = hipMemcpyAsync(r->lambda, a.lambda, utotal * 8, hipMemcpyDeviceToHost, c->stream)) !=
                           hipSuccess)
      return bail(e, "hipMemcpyAsync");
    if ((e = hipMemcpyAsync(r->status, a.status, M * 4, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
      return bail(e, "hipMemcpyAsync");
  }
  if ((e = hipEventRecord(t.stop, c->stream)) != hipSuccess) return bail(e, "hipEventRecord");
  if (!dev && (e = hipEventSynchronize(t.stop)) != hipSuccess) return bail(e, "hipEventSynchronize");
  const uint64_t id = c->next_ticket++;
  t.bytes = held;
  c->held_bytes += held;
  c->tickets.emplace(id, std::move(t));
  *ticket = id;
  return NLS_OK;
}

}  // extern "C"
