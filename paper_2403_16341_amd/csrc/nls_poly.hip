// nls_poly.hip -- device steps of the fallback chain (the first-order part of
// the default poly-algorithm, Sec. 3.2): gather the systems a stage left
// unsolved, and fold a later stage's attempt into the results.  The counts
// stay on the device; the solver launches read them through KArgs::count_dev.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nls_launch.h"

namespace nls {

// Append to out the listed systems (in[j] for j < min(*in_count, cap), or j
// itself when in is null) whose retcode is neither SUCCESS nor INVALID;
// *out_count, zeroed before, ends as their number.  One atomic per wavefront;
// the order of out is arbitrary (each system's solve does not depend on it).
__global__ __launch_bounds__(256) void k_poly_select(const int32_t* in, const int64_t* in_count, int64_t cap,
                                                     const int32_t* rc, int32_t* out, int64_t* out_count) {
  int64_t count = cap;
  if (in_count) {
    const int64_t c = *in_count;
    count = c < cap ? (c > 0 ? c : 0) : cap;
  }
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t s = 0;
  bool keep = false;
  if (j < count) {
    s = in ? in[j] : (int32_t)j;
    const int32_t r = rc[s];
    keep = r != RC_SUCCESS && r != RC_INVALID;
  }
  const unsigned long long m = __ballot(keep);
  if (m == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)m) - 1;
  const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
  int64_t base = 0;
  if (lane == leader)
    base = (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(out_count), (unsigned long long)__popcll(m));
  base = __shfl(base, leader, 64);
  if (keep) out[base + rank] = s;
}

// Fold the attempt of a later stage (the *_t arrays, written for the listed
// systems only) into the results.  The counters add up over the attempts;
// u, ||F||_inf and the retcode follow the attempt when it succeeded or left a
// strictly smaller residual (so the earliest attempt wins ties).  An attempt
// that ended INVALID replaces everything, so the mark is never hidden.
__global__ __launch_bounds__(256) void k_poly_merge(const PolyMergeArgs a) {
  int64_t count = a.cap;
  {
    const int64_t c = *a.count;
    count = c < a.cap ? (c > 0 ? c : 0) : a.cap;
  }
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  const int64_t s = a.list[j];
  const int n = a.nsys ? (int)a.nsys[s] : a.n;
  const int64_t uo = a.u_off ? a.u_off[s] : s * (int64_t)n;
  const int32_t rt = a.retcode_t[s];
  const bool invalid = rt == RC_INVALID;
  const bool take = invalid || rt == RC_SUCCESS || a.fnorm_t[s] < a.fnorm[s];
  a.iters[s] = invalid ? a.iters_t[s] : a.iters[s] + a.iters_t[s];
  if (a.nfev) a.nfev[s] += a.nfev_t[s];
  if (a.njev) a.njev[s] += a.njev_t[s];
  if (take) {
    for (int i = 0; i < n; ++i) a.u[uo + i] = a.u_t[uo + i];
    a.fnorm[s] = a.fnorm_t[s];
    a.retcode[s] = rt;
  }
}

int launch_poly_select(const int32_t* in, const int64_t* in_count, int64_t cap, const int32_t* rc, int32_t* out,
                       int64_t* out_count, hipStream_t st) {
  if (cap <= 0) return 0;
  const int64_t blocks = (cap + 255) / 256;
  hipLaunchKernelGGL(k_poly_select, dim3((unsigned)blocks), dim3(256), 0, st, in, in_count, cap, rc, out, out_count);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : -(int)e;
}

int launch_poly_merge(const PolyMergeArgs& a, hipStream_t st) {
  if (a.cap <= 0) return 0;
  const int64_t blocks = (a.cap + 255) / 256;
  hipLaunchKernelGGL(k_poly_merge, dim3((unsigned)blocks), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : -(int)e;
}

}  // namespace nls
