// Instantiation unit of the Dyson kernel for band windows padded to 16.
#include "dyson_impl.h"

namespace dmft {
using D16 = VariantSet<16, KIND_DENSITY, 5, 1>;
using T16 = VariantSet<16, KIND_TRACE, 5, 1>;
hipError_t launch_dyson_16(int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
  return (a.mode & MODE_TRACE) ? T16::launch(var, a, grid, s) : D16::launch(var, a, grid, s);
}
int variants_16(int kind, int* out, int max) { return kind ? T16::list(out, max) : D16::list(out, max); }
}  // namespace dmft
