// Instantiation unit of the low-rank density kernel with three frequencies per
// matrix-core tile (lowrank_p3_impl.h): variant code 42 of the density kind,
// nc <= 5, windows padded to 16, 32 or 48 bands (one wavefront per (k tile,
// frequency tile)) or 64 bands (four wavefronts per item).  48- and
// 64-band windows take the partial-fraction form of the running sum (on 32
// bands it measured slower than the direct form).
#include "lowrank_p3_impl.h"

namespace dmft {

template <int NBP, int RL, bool PF>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1))) lr_p3_kernel(DysonArgs a) {
  __shared__ LRP3Shared<NBP> sh;
  __shared__ double2 pfc[PF ? NBP / 16 * 4 * 64 : 1];
  lr_p3_tile<NBP, RL, true, PF>(a, blockIdx.x / a.n_wtiles, blockIdx.x % a.n_wtiles, sh, threadIdx.x, pfc);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1))) lr_p3_quad_kernel(DysonArgs a) {
  __shared__ LRP3QuadShared sh;
  lr_p3_quad_tile<true>(a, blockIdx.x / a.n_wtiles, blockIdx.x % a.n_wtiles, sh, threadIdx.x);
}

hipError_t launch_lowrank_p3(int nbp, const DysonArgs& a, dim3 grid, hipStream_t s) {
  if (!lowrank_p3_fits(nbp, a.nc) || (a.mode & (MODE_TRACE | MODE_ADJ | MODE_GEN)) || !(a.mode & (MODE_S | MODE_GLOC)))
    return hipErrorInvalidValue;
  switch (nbp) {
    case 16: hipLaunchKernelGGL((lr_p3_kernel<16, 0, false>), grid, dim3(64), 0, s, a); break;
    case 32: hipLaunchKernelGGL((lr_p3_kernel<32, 0, false>), grid, dim3(64), 0, s, a); break;
    case 48: hipLaunchKernelGGL((lr_p3_kernel<48, 1, true>), grid, dim3(64), 0, s, a); break;
    case 64: hipLaunchKernelGGL(lr_p3_quad_kernel, grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dmft
