// Group-mapping kernels, double inner form, size bucket n <= 56.
#include "nls_kernels.hpp"
#include "nls_launch.h"
#define NLS_TI double
#define NLS_NB 56
#define NLS_GROUP_ENTRY launch_group_f64_nb56
#include "nls_group_dispatch.inc"
