// nls_noalloc.hip -- nls_solve_batch_noalloc: the batch solve for callers
// that cannot allocate device memory (code under stream capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// The solver kernels need scratch beyond the caller's inputs and outputs: a
// work counter per persistent launch, and for the fallback chain the device
// lists of unsolved systems, their counts and the scratch outputs of the
// later stages.  Here that scratch is one file-scope device array of fixed
// size, `scratch`; each device holds its own copy for the life of the
// process.  Its device address is taken once per device with
// hipGetSymbolAddress (the array's name is a host-side stand-in in host
// code), and only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <string>

#include "nls.h"
#include "nls_launch.h"
#include "nls_runtime.h"
#include "nls_types.h"

using namespace nls;
using namespace nls::rt;

namespace {

constexpr int64_t kCounters = 64;                          // int64 work counters
constexpr int64_t kChainSystems = NLS_NOALLOC_MAX_CHAIN_SYSTEMS;
constexpr int64_t kChainUnknowns = NLS_NOALLOC_MAX_CHAIN_UNKNOWNS;

// byte offsets of the scratch regions (each 256-byte aligned)
constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t kOffCounters = 0;
constexpr size_t kOffSel1 = align256(kOffCounters + kCounters * 8);
constexpr size_t kOffSel2 = align256(kOffSel1 + kChainSystems * 4);
constexpr size_t kOffUt = align256(kOffSel2 + kChainSystems * 4);
constexpr size_t kOffFn = align256(kOffUt + kChainUnknowns * 8);
constexpr size_t kOffIt = align256(kOffFn + kChainSystems * 8);
constexpr size_t kOffRc = align256(kOffIt + kChainSystems * 4);
constexpr size_t kOffNf = align256(kOffRc + kChainSystems * 4);
constexpr size_t kOffNj = align256(kOffNf + kChainSystems * 4);
constexpr size_t kScratchBytes = align256(kOffNj + kChainSystems * 4);
static_assert(kScratchBytes == NLS_NOALLOC_SCRATCH_BYTES, "scratch size differs from the one nls.h states");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current.
hipError_t scratch_address(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch[dev]);
  return hipSuccess;
}

int fail(int code, const std::string& m) {
  set_thread_error("nls_solve_batch_noalloc: " + m);
  return code;
}

}  // namespace

extern "C" int nls_solve_batch_noalloc(const nls_batch* b, const nls_results* r, void* stream) {
  int64_t bad = -1;
  std::string m = validate(b, &bad);
  if (m.empty()) m = check_results(r, b->count);
  if (!m.empty()) return fail(NLS_E_INVALID, m);
  if (b->mem_kind != NLS_MEM_DEVICE) return fail(NLS_E_INVALID, "params, u0 and the results must be device memory");
  int fam0, n0, alg0;
  if (!uniform_batch(b, &fam0, &n0, &alg0))
    return fail(NLS_E_INVALID, "the batch must be uniform (one family, size and algorithm, packed back to back)");
  const int64_t M = b->count;
  if (M == 0) return NLS_OK;
  const bool poly = alg0 == ALG_POLY;
  if (poly && (M > kChainSystems || M * (int64_t)n0 > kChainUnknowns)) {
    char buf[200];
    std::snprintf(buf, sizeof buf,
                  "fallback-chain batch of %lld systems / %lld unknowns exceeds the fixed scratch (at most %lld "
                  "systems and %lld unknowns)",
                  (long long)M, (long long)(M * n0), (long long)kChainSystems, (long long)kChainUnknowns);
    return fail(NLS_E_NOMEM, buf);
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(NLS_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(NLS_E_DEVICE, "device ordinal out of range");
  unsigned char* base = nullptr;
  if ((e = scratch_address(dev, &base)) != hipSuccess)
    return fail(NLS_E_DEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));

  nls_alg_options opts;
  fill_defaults(&opts);
  if (b->opts) opts = *b->opts;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KArgs a{};
  a.params = b->params;
  a.u0 = b->u0;
  a.u_out = r->u;
  a.fnorm = r->fnorm_inf;
  a.iters = r->iters;
  a.retcode = r->retcode;
  a.nfev = r->nfev;
  a.njev = r->njev;
  a.maxiters = b->maxiters;
  a.abstol = b->abstol;
  a.o = to_kopts(opts);
  a.count = M;
  a.P = nparams_of(fam0, n0);
  a.n = n0;
  a.counter = reinterpret_cast<int64_t*>(base + kOffCounters);
  const Mapping mp = fixed_mapping(n0);
  const int alg1 = poly ? ALG_NEWTON : alg0;  // the chain starts with Newton
  // the counter keeps the last call's value: zero it first (a kernel, so the
  // call can be captured into a graph)
  if (int z = launch_zero_counters(a.counter, 1, st); z < 0)
    return fail(NLS_E_DEVICE, std::string("zero counters: ") + hipGetErrorString((hipError_t)(-z)));
  int rc = launch(mp.key_n, mp.lane, fam0, alg1, b->precision, a, st);
  if (rc > 0) return fail(NLS_E_INVALID, "no kernel for this family/size/algorithm");
  if (rc < 0) return fail(NLS_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString((hipError_t)(-rc)));
  if (poly) {
    ChainScratch sc{reinterpret_cast<int32_t*>(base + kOffSel1), reinterpret_cast<int32_t*>(base + kOffSel2),
                    reinterpret_cast<int64_t*>(base + kOffCounters) + 1, reinterpret_cast<double*>(base + kOffUt),
                    reinterpret_cast<double*>(base + kOffFn), reinterpret_cast<int32_t*>(base + kOffIt),
                    reinterpret_cast<int32_t*>(base + kOffRc),
                    a.nfev ? reinterpret_cast<int32_t*>(base + kOffNf) : nullptr,
                    a.njev ? reinterpret_cast<int32_t*>(base + kOffNj) : nullptr};
    rc = run_chain(a, mp.lane, mp.key_n, fam0, b->precision, sc, st);
    if (rc > 0) return fail(NLS_E_INVALID, "no kernel for this family/size/algorithm");
    if (rc < 0) return fail(NLS_E_DEVICE, std::string("fallback chain: ") + hipGetErrorString((hipError_t)(-rc)));
  }
  return NLS_OK;
}
