// Group-mapping kernels, float inner form, size bucket n <= 24.
#include "nls_kernels.hpp"
#include "nls_launch.h"
#define NLS_TI float
#define NLS_NB 24
#define NLS_GROUP_ENTRY launch_group_f32_nb24
#include "nls_group_dispatch.inc"
