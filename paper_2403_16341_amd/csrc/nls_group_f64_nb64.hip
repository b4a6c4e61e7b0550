// Group-mapping kernels, double inner form, size bucket n <= 64.
#include "nls_kernels.hpp"
#include "nls_launch.h"
#define NLS_TI double
#define NLS_NB 64
#define NLS_GROUP_ENTRY launch_group_f64_nb64
#include "nls_group_dispatch.inc"
