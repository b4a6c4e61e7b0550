// nls_runtime.h -- host-side helpers shared by the batch runtime (nls_host.cpp)
// and the request server (nls_serve.cpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>

#include "nls.h"
#include "nls_types.h"

namespace nls {
namespace rt {

// message returned by nls_last_error(NULL) on this thread
void set_thread_error(const std::string& m);
const char* thread_error();

// parameters per system of a family at size n, or -1 if it is not defined there
int nparams_of(int family, int n);
// a family/size pair the kernels implement
bool supported(int family, int n);
// one family, size and algorithm for every system, packed back to back
bool uniform_batch(const nls_batch* b, int* fam0, int* n0, int* alg0);

void fill_defaults(nls_alg_options* o);
std::string check_options(const nls_alg_options& o);
// "" if the batch is well formed, else the reason (first_bad: offending system)
std::string validate(const nls_batch* b, int64_t* first_bad);
std::string check_results(const nls_results* r, int64_t M);
KOpts to_kopts(const nls_alg_options& o);

struct Mapping {
  bool lane;
  int key_n;  // n for the lane mapping, the size bucket for the group mapping
  hipError_t error;
  int rows = 0;  // group mapping, n <= 16 bucket: rows per lane (0 = the default, two)
};
// size bucket (16, 24, ..., 64) of the group mapping for n > 8
int group_bucket(int n);
// the mapping used without autotuning: one system per lane for n <= 8, else
// one system per 16/32/64-lane group
Mapping fixed_mapping(int n);

// one persistent launch; 0 on success, 1 if no kernel exists for the
// combination, a negative hipError_t value on a launch failure
int launch(int n_or_nb, bool lane, int fam, int alg, int prec, const KArgs& a, hipStream_t st);

// Device scratch of one segment of the fallback chain: two system lists of
// a.count entries, four work counts (zeroed by run_chain), and scratch
// outputs laid out like the results (u_t over the same offsets as u).
struct ChainScratch {
  int32_t* sel1;
  int32_t* sel2;
  int64_t* cnt;
  double* u_t;
  double* fnorm_t;
  int32_t* iters_t;
  int32_t* retcode_t;
  int32_t* nfev_t;  // may be null when a.nfev is
  int32_t* njev_t;  // may be null when a.njev is
};
// After the Newton-stage launch `a` of a segment (its outputs are the
// results; a.sys null = systems 0..a.count-1), run the chain's Armijo and
// dogleg stages on the systems still unsolved, on the same kernel mapping:
// select, solve from u0 into the scratch outputs, merge, all on stream st.
int run_chain(const KArgs& a, bool lane, int key_n, int fam, int prec, const ChainScratch& sc, hipStream_t st);

}  // namespace rt
}  // namespace nls
