// Instantiation unit of the Dyson kernel for band windows padded to 32.
#include "dyson_impl.h"

namespace dmft {
using D32 = VariantSet<32, KIND_DENSITY, 7, 6, 1>;
using T32 = VariantSet<32, KIND_TRACE, 1, 4>;
hipError_t launch_dyson_32(int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
  return (a.mode & MODE_TRACE) ? T32::launch(var, a, grid, s) : D32::launch(var, a, grid, s);
}
int variants_32(int kind, int* out, int max) { return kind ? T32::list(out, max) : D32::list(out, max); }
}  // namespace dmft
