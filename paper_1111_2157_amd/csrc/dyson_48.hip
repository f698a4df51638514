// Instantiation unit of the Dyson kernel for band windows padded to 48.
#include "dyson_impl.h"

namespace dmft {
using D48 = VariantSet<48, KIND_DENSITY, 2, 3>;
using T48 = VariantSet<48, KIND_TRACE, 0>;
hipError_t launch_dyson_48(int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
  return (a.mode & MODE_TRACE) ? T48::launch(var, a, grid, s) : D48::launch(var, a, grid, s);
}
int variants_48(int kind, int* out, int max) { return kind ? T48::list(out, max) : D48::list(out, max); }
}  // namespace dmft
