// Batched low-rank pass: persistent class kernels for band windows padded to 48
// (see batched_lr.h), one per column count of the row-layout inversions
// (class 5: nc <= 5, three frequencies per matrix-core tile).
#include "batched_lr.h"

namespace dmft {

hipError_t launch_lr_class_48(int ncls, const void* items, int n_items, const DysonArgs* args, int* counter,
                              int grid, hipStream_t s) {
  const BatchItem* it = reinterpret_cast<const BatchItem*>(items);
  switch (ncls) {
    case 5:
      hipLaunchKernelGGL((lr_p3_class_kernel<48, 1, true, true>), dim3(grid), dim3(64), 0, s, it, n_items, args, counter);
      break;
    case 8:
      hipLaunchKernelGGL((lr_class_kernel<48, 1, true, 8>), dim3(grid), dim3(64), 0, s, it, n_items, args, counter);
      break;
    case 12:
      hipLaunchKernelGGL((lr_class_kernel<48, 1, true, 12>), dim3(grid), dim3(64), 0, s, it, n_items, args, counter);
      break;
    case 14:
      hipLaunchKernelGGL((lr_class_kernel<48, 1, true, 14, true>), dim3(grid), dim3(64), 0, s, it, n_items, args, counter);
      break;
    case 16:
      hipLaunchKernelGGL((lr_class_kernel<48, 1, true, 16>), dim3(grid), dim3(64), 0, s, it, n_items, args, counter);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dmft
