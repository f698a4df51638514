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
hipError_t launch_lowrank_pair64(const DysonArgs& a, dim3 grid, hipStream_t s);
hipError_t launch_lowrank_p3(int nbp, const DysonArgs& a, dim3 grid, hipStream_t s);
hipError_t launch_lr_class_16(int ncls, const void* items, int n_items, const DysonArgs* args, int* counter, int grid,
                              hipStream_t s);
hipError_t launch_lr_class_32(int ncls, const void* items, int n_items, const DysonArgs* args, int* counter, int grid,
                              hipStream_t s);
hipError_t launch_lr_class_48(int ncls, const void* items, int n_items, const DysonArgs* args, int* counter, int grid,
                              hipStream_t s);
hipError_t launch_lr_class_64(int ncls, const void* items, int n_items, const DysonArgs* args, int* counter, int grid,
                              hipStream_t s);

hipError_t launch_lowrank(int nbp, int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
  if (var == kLowrankPairVariant) return nbp == 64 ? launch_lowrank_pair64(a, grid, s) : hipErrorInvalidValue;
  if (var == kLowrankP3Variant) return lowrank_p3_fits(nbp, a.nc) ? launch_lowrank_p3(nbp, a, grid, s) : hipErrorInvalidValue;
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
    case 16:
    case 32:
    case 48: {
      int n = nbp == 16 ? lowrank_variants_16(kind, out, max)
              : nbp == 32 ? lowrank_variants_32(kind, out, max) : lowrank_variants_48(kind, out, max);
      if (kind == 0 && n < max) out[n++] = kLowrankP3Variant;
      return n;
    }
    case 64: {
      int n = lowrank_variants_64(kind, out, max);
      if (kind == 0 && n < max) out[n++] = kLowrankPairVariant;
      if (kind == 0 && n < max) out[n++] = kLowrankP3Variant;
      return n;
    }
    default: return 0;
  }
}

// Column class of the batched kernels: 5 for nc <= 5 (three frequencies per
// matrix-core tile), else nc rounded up to 8, 10
// (32 bands), 12, 14 (32, 48 and 64 bands) or 16.  Every column costs a
// broadcast and four FMAs in each of the nc pivot steps of both inversions,
// which on small windows weighs as much as the matrix-core work.
int lr_nc_class(int nbp, int nc) {
  if (lowrank_p3_fits(nbp, nc)) return 5;
  if (nc <= 8) return 8;
  if (nbp == 32 && nc <= 10) return 10;
  if (nc <= 12) return 12;
  if (nbp >= 32 && nc <= 14) return 14;
  return 16;
}

int lr_class_wgs_per_cu(int nbp, int ncls) { return nbp < 64 ? 4 : ncls == 5 ? 1 : 2; }

hipError_t launch_lr_class(int nbp, int ncls, const void* items, int n_items, const DysonArgs* args, int* counter,
                           int grid, hipStream_t s) {
  switch (nbp) {
    case 16: return launch_lr_class_16(ncls, items, n_items, args, counter, grid, s);
    case 32: return launch_lr_class_32(ncls, items, n_items, args, counter, grid, s);
    case 48: return launch_lr_class_48(ncls, items, n_items, args, counter, grid, s);
    case 64: return launch_lr_class_64(ncls, items, n_items, args, counter, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dmft
