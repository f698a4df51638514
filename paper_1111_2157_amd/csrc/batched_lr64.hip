// Batched low-rank pass: persistent class kernels for 64-band windows on
// two-wavefront work-groups (see batched_lr.h), one per column count of the
// row-layout inversions, and for nc <= 5 (class 5) on four-wavefront ones.
#include "batched_lr.h"

namespace dmft {

hipError_t launch_lr_class_64(int ncls, const void* items, int n_items, const DysonArgs* args, int* counter,
                              int grid, hipStream_t s) {
  const BatchItem* it = reinterpret_cast<const BatchItem*>(items);
  switch (ncls) {
    case 5: hipLaunchKernelGGL(lr_p3_quad_class_kernel<64>, dim3(grid), dim3(256), 0, s, it, n_items, args, counter); break;
    case 8: hipLaunchKernelGGL(lr_pair_class_kernel<8>, dim3(grid), dim3(128), 0, s, it, n_items, args, counter); break;
    case 12: hipLaunchKernelGGL(lr_pair_class_kernel<12>, dim3(grid), dim3(128), 0, s, it, n_items, args, counter); break;
    case 14: hipLaunchKernelGGL(lr_pair_class_kernel<14>, dim3(grid), dim3(128), 0, s, it, n_items, args, counter); break;
    case 16: hipLaunchKernelGGL(lr_pair_class_kernel<16>, dim3(grid), dim3(128), 0, s, it, n_items, args, counter); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dmft
