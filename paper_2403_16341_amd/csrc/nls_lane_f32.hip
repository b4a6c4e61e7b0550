// Lane-mapping kernels, FP32-inner form (Jacobian, LU and step algebra in FP32).
#include "nls_kernels.hpp"
#include "nls_launch.h"
#define NLS_TI float
#define NLS_LANE_ENTRY launch_lane_f32
#include "nls_lane_dispatch.inc"
