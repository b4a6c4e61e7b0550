// Group-mapping kernels, double inner form, size bucket n <= 48.
#include "nls_kernels.hpp"
#include "nls_launch.h"
#define NLS_TI double
#define NLS_NB 48
#define NLS_GROUP_ENTRY launch_group_f64_nb48
#include "nls_group_dispatch.inc"
