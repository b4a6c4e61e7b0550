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

// dispatch over the buckets 16, 24, ..., 64
inline int launch_group(int prec, int nb, int fam, int alg, const KArgs& a, hipStream_t st) {
#define NLS_CASE(NB) \
  case NB: return prec == PREC_FP64 ? launch_group_f64_nb##NB(fam, alg, a, st) : launch_group_f32_nb##NB(fam, alg, a, st);
  switch (nb) { NLS_CASE(16) NLS_CASE(24) NLS_CASE(32) NLS_CASE(40) NLS_CASE(48) NLS_CASE(56) NLS_CASE(64) }
#undef NLS_CASE
  return 1;
}

}  // namespace nls
