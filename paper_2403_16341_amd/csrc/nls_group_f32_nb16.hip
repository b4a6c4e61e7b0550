// Group-mapping kernels, float inner form, size bucket n <= 16.
#include "nls_kernels.hpp"
#include "nls_launch.h"
#define NLS_TI float
#define NLS_NB 16
#define NLS_GROUP_ENTRY launch_group_f32_nb16
#include "nls_group_dispatch.inc"
