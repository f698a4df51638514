// Dispatch of the low-rank Dyson kernel (lowrank_impl.h) over the padded
// band-window sizes; the kernels are instantiated in lowrank_{16,32,48,64}.hip.
#include <hip/hip_runtime.h>

#include "dmft_internal.h"

namespace dmft {

hipError_t launch_lowrank_16(int var, const DysonArgs& a, dim3 grid, hipStream_t s);
hipError_t launch_lowrank_32(int var, const DysonArgs& a, dim3 grid, hipStream_t s);
hipError_t launch_lowrank_48(int var, const DysonArgs& a, dim3 grid, hipStream_t s);
hipError_t launch_lowrank_64(int var, const DysonArgs& a, dim3 grid, hipStream_t s);
int lowrank_variants_16(int kind, int* out, int max);
int lowrank_variants_32(int kind, int* out, int max);
int lowrank_variants_48(int kind, int* out, int max);
int lowrank_variants_64(int kind, int* out, int max);

hipError_t launch_lowrank(int nbp, int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
  switch (nbp) {
    case 16: return launch_lowrank_16(var, a, grid, s);
    case 32: return launch_lowrank_32(var, a, grid, s);
    case 48: return launch_lowrank_48(var, a, grid, s);
    case 64: return launch_lowrank_64(var, a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

int lowrank_variants(int nbp, int kind, int* out, int max) {
  if (max <= 0) return 0;
  switch (nbp) {
    case 16: return lowrank_variants_16(kind, out, max);
    case 32: return lowrank_variants_32(kind, out, max);
    case 48: return lowrank_variants_48(kind, out, max);
    case 64: return lowrank_variants_64(kind, out, max);
    default: return 0;
  }
}

}  // namespace dmft
