// nls_launch.h -- launch entry points of the kernel translation units.
// Each returns 0 on success, 1 if no kernel exists for the combination, or
// a negative hipError_t value.
#pragma once

#include <hip/hip_runtime_api.h>

#include "nls_types.h"

namespace nls {

// one system per lane, 1 <= n <= 8
int launch_lane_f64(int n, int fam, int alg, const KArgs& a, hipStream_t st);
int launch_lane_f32(int n, int fam, int alg, const KArgs& a, hipStream_t st);

// one system per group of lanes, per size bucket nb (systems with n <= nb)
#define NLS_DECL_GROUP(P, NB) int launch_group_##P##_nb##NB(int fam, int alg, const KArgs& a, hipStream_t st);
#define NLS_DECL_GROUPS(P) \
  NLS_DECL_GROUP(P, 16) NLS_DECL_GROUP(P, 24) NLS_DECL_GROUP(P, 32) NLS_DECL_GROUP(P, 40) \
  NLS_DECL_GROUP(P, 48) NLS_DECL_GROUP(P, 56) NLS_DECL_GROUP(P, 64)
NLS_DECL_GROUPS(f64)
NLS_DECL_GROUPS(f32)

// zero `count` work counters on the stream
int launch_zero_counters(int64_t* c, int count, hipStream_t st);

// Fallback chain steps.  select: out <- the listed systems (in[j], j <
// min(*in_count, cap); in null = 0..cap-1, in_count null = cap) whose retcode
// is neither SUCCESS nor INVALID, *out_count (zeroed before) <- their number.
int launch_poly_select(const int32_t* in, const int64_t* in_count, int64_t cap, const int32_t* rc, int32_t* out,
                       int64_t* out_count, hipStream_t st);

// merge: for the systems list[j], j < min(*count, cap), fold the attempt in
// the *_t arrays into the results (see k_poly_merge).
struct PolyMergeArgs {
  const int32_t* list;
  const int64_t* count;
  int64_t cap;
  const uint8_t* nsys;  // per-system n, or null with n uniform
  int32_t n;
  const int64_t* u_off;  // null: system s at s * n
  double* u;
  double* fnorm;
  int32_t* iters;
  int32_t* retcode;
  int32_t* nfev;  // may be null
  int32_t* njev;  // may be null
  const double* u_t;
  const double* fnorm_t;
  const int32_t* iters_t;
  const int32_t* retcode_t;
  const int32_t* nfev_t;
  const int32_t* njev_t;
};
int launch_poly_merge(const PolyMergeArgs& a, hipStream_t st);

// Sensitivities at a solution (implicit function theorem).  Slot t handles
// system sys[t] (or t when sys is null); the parameters of system s start at
// params + p_off[s] (or s * P), its unknowns at u + u_off[s] (or s * n).
enum : int { SENS_TANGENT = 0, SENS_ADJOINT = 1 };
struct SensArgs {
  const double* params;
  const double* u;     // the solution u*
  const double* seed;  // tangent: v (laid out like params); adjoint: w (like u)
  double* out;         // tangent: du (like u); adjoint: the gradient (like params)
  double* lambda;      // adjoint: J^{-T} w (like u); may be null
  int32_t* status;     // [M]: RC_SUCCESS, RC_SINGULAR or RC_NONFINITE
  const int64_t* p_off;
  const int64_t* u_off;
  const int32_t* sys;
  const uint8_t* nsys;  // per-system n, or null with n uniform
  int64_t count;
  int64_t P;
  int32_t n;
};
// Persistent grid under a cap of pct percent of the resident wavefronts
// (pct <= 0 or >= 100: no cap; at least one wavefront).
inline int grid_cap(int waves, int pct) {
  if (pct <= 0 || pct >= 100) return waves;
  const int c = (int)((int64_t)waves * pct / 100);
  return c > 0 ? c : 1;
}

// size bucket of the sensitivity kernels: 8, 16, 24, ..., 64
inline int sens_bucket(int n) { return n <= 8 ? 8 : (n + 7) / 8 * 8; }
int launch_sens(int nb, int fam, int mode, const SensArgs& a, hipStream_t st);

// dispatch over the buckets 16, 24, ..., 64
inline int launch_group(int prec, int nb, int fam, int alg, const KArgs& a, hipStream_t st) {
#define NLS_CASE(NB) \
  case NB: return prec == PREC_FP64 ? launch_group_f64_nb##NB(fam, alg, a, st) : launch_group_f32_nb##NB(fam, alg, a, st);
  switch (nb) { NLS_CASE(16) NLS_CASE(24) NLS_CASE(32) NLS_CASE(40) NLS_CASE(48) NLS_CASE(56) NLS_CASE(64) }
#undef NLS_CASE
  return 1;
}

}  // namespace nls
