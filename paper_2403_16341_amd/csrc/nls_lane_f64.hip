// Lane-mapping kernels, plain FP64 form.
#include "nls_kernels.hpp"
#include "nls_launch.h"
#define NLS_TI double
#define NLS_LANE_ENTRY launch_lane_f64
#include "nls_lane_dispatch.inc"
