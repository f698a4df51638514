// Instantiation unit of the low-rank Dyson kernel (lowrank_impl.h) for band
// windows padded to 48: the variants that compile without register spills.
#include "lowrank_impl.h"

namespace dmft {
using LD48 = LRSet<48, KIND_DENSITY, 8, 24, 26, 9, 11, 90>;
using LA48 = LRSet<48, KIND_ADJ, 10, 8, 26>;
using LG48 = LRSet<48, KIND_GEN, 8, 9, 24>;
using LT48 = LRSet<48, KIND_TRACE, 15, 13, 8, 10, 24, 26>;
hipError_t launch_lowrank_48(int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
  if (a.mode & MODE_ADJ) return LA48::launch(var, a, grid, s);
  if (a.mode & MODE_GEN) return LG48::launch(var, a, grid, s);
  return (a.mode & MODE_TRACE) ? LT48::launch(var, a, grid, s) : LD48::launch(var, a, grid, s);
}
int lowrank_variants_48(int kind, int* out, int max) {
  if (kind == 3) return LG48::list(out, max);
  return kind == 2 ? LA48::list(out, max) : kind ? LT48::list(out, max) : LD48::list(out, max);
}
}  // namespace dmft
