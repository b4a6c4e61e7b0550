// Small device utilities used by the host runtime.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nls_launch.h"

namespace nls {

// Zero the dynamic work counters of a launch.  A kernel rather than a memset,
// so that a captured graph holds no memset node.
__global__ void k_zero_counters(int64_t* c, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) c[i] = 0;
}

int launch_zero_counters(int64_t* c, int count, hipStream_t st) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(k_zero_counters, dim3((count + 255) / 256), dim3(256), 0, st, c, count);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : -(int)e;
}

}  // namespace nls
