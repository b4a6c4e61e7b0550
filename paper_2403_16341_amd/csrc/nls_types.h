// nls_types.h -- internal types shared by the host runtime and the kernels.
#pragma once

#include <stdint.h>

namespace nls {

enum : int { FAM_CUBIC = 0, FAM_TANH = 1, FAM_ROSENBROCK = 2, FAM_PAPER = 3, FAM_COUNT = 4 };
enum : int { ALG_NEWTON = 0, ALG_ARMIJO = 1, ALG_DOGLEG = 2, ALG_COUNT = 3 };
// the fallback chain NEWTON -> ARMIJO -> DOGLEG, run by the host runtime as
// three stages of the kernels above (no kernel of its own); the Potra-Ptak
// two-step scheme (one Jacobian, two solves per iteration)
enum : int { ALG_POLY = 3, ALG_POTRA = 4, ALG_KEYS = 5 };
enum : int { PREC_FP64 = 0, PREC_FP32_INNER = 1 };
enum : int {
  RC_SUCCESS = 0,
  RC_MAXITERS = 1,
  RC_SINGULAR = 2,
  RC_NONFINITE = 3,
  RC_LINESEARCH_FAILED = 4,
  RC_TR_COLLAPSED = 5,
  RC_INVALID = 6
};

struct DoglegOpts {
  double delta0, delta_max, eta1, eta2, expand, shrink, collapse;
};

// Algorithm options as the kernels see them (validated on the host).
struct KOpts {
  double armijo_c;
  double armijo_rho;
  int32_t armijo_max_halvings;
  int32_t pad;
  double tr_delta0, tr_delta_max, tr_eta1, tr_eta2, tr_expand, tr_shrink, tr_collapse;
#ifdef __HIPCC__
  __host__ __device__
#endif
  DoglegOpts dogleg() const {
    return DoglegOpts{tr_delta0, tr_delta_max, tr_eta1, tr_eta2, tr_expand, tr_shrink, tr_collapse};
  }
};

// Arguments of one solver launch.  The launch handles `count` slots, or
// min(*count_dev, count) when count_dev is set (a count produced on the device
// by an earlier kernel); slot t solves system sys[t] (or t when sys is null).  Parameters of system s start
// at params + p_off[s] (or s * P), its unknowns at u0 + u_off[s] (or s * n).
struct KArgs {
  const double* params;
  const double* u0;
  double* u_out;
  double* fnorm;
  int32_t* iters;
  int32_t* retcode;
  int32_t* nfev;  // may be null
  int32_t* njev;  // may be null
  const int64_t* p_off;
  const int64_t* u_off;
  const int32_t* sys;
  const uint8_t* nsys;  // per-system n (group mapping, mixed sizes); may be null
  int64_t* counter;     // dynamic work counter (zeroed before the launch); may be null
  const int64_t* count_dev;  // may be null
  int64_t count;
  int64_t P;
  int32_t n;            // uniform n when nsys is null
  int32_t maxiters;
  double abstol;
  KOpts o;
  int32_t rows;         // group kernels of the n <= 16 bucket: rows per lane (1 or 2; 0 = the default)
  int32_t grid_pct;     // persistent grid cap, percent of the resident wavefronts (0 = no cap)
};

}  // namespace nls
