// Instantiation unit of the two-wavefront Dyson kernel (band windows padded to 64).
#include "dyson64_impl.h"

namespace dmft {


hipError_t launch_dyson_64(int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
  if (var != 0) return hipErrorInvalidValue;
  if (a.mode & MODE_TRACE)
    hipLaunchKernelGGL(d64::kernel<KIND_TRACE>, grid, dim3(128), 0, s, a);
  else
    hipLaunchKernelGGL(d64::kernel<KIND_DENSITY>, grid, dim3(128), 0, s, a);
  return hipGetLastError();
}

int variants_64(int kind, int* out, int max) {
  (void)kind;
  if (max > 0 && out) out[0] = 0;
  return 1;
}

}  // namespace dmft
