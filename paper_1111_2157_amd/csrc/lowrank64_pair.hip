// Instantiation unit of the two-wavefront low-rank kernel for 64-band windows
// (lowrank_pair_impl.h): variant code 40 of the density kind (low-rank bit 3,
// pair bit 5).  Grid: one 128-thread work-group per (k tile, frequency tile).
#include "lowrank_pair_impl.h"

namespace dmft {

template <int NC>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(1))) lr_pair_kernel(DysonArgs a) {
  __shared__ LRPairShared sh;
  lr_pair_tile<NC, (NC >= 12)>(a, blockIdx.x / a.n_wtiles, blockIdx.x % a.n_wtiles, sh, threadIdx.x);
}

// Columns of the row-layout inversions: nc rounded up to 8, 12, 14 or 16.
int pair_nc_class(int nc) { return nc <= 8 ? 8 : nc <= 12 ? 12 : nc <= 14 ? 14 : 16; }

hipError_t launch_lowrank_pair64(const DysonArgs& a, dim3 grid, hipStream_t s) {
  if (!(a.mode & (MODE_S | MODE_GLOC)) || (a.mode & (MODE_TRACE | MODE_ADJ | MODE_GEN))) return hipErrorInvalidValue;
  switch (pair_nc_class(a.nc)) {
    case 8: hipLaunchKernelGGL(lr_pair_kernel<8>, grid, dim3(128), 0, s, a); break;
    case 12: hipLaunchKernelGGL(lr_pair_kernel<12>, grid, dim3(128), 0, s, a); break;
    case 14: hipLaunchKernelGGL(lr_pair_kernel<14>, grid, dim3(128), 0, s, a); break;
    default: hipLaunchKernelGGL(lr_pair_kernel<16>, grid, dim3(128), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace dmft
