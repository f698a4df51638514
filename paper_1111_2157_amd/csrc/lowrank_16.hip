// Instantiation unit of the low-rank Dyson kernel (lowrank_impl.h) for band
// windows padded to 16: the variants that compile without register spills.
#include "lowrank_impl.h"

namespace dmft {
using LD16 = LRSet<16, KIND_DENSITY, 14, 8, 10, 26, 30>;
using LA16 = LRSet<16, KIND_ADJ, 10, 8>;
using LG16 = LRSet<16, KIND_GEN, 8, 9, 24>;
using LT16 = LRSet<16, KIND_TRACE, 14, 12, 13, 15, 28, 30>;
hipError_t launch_lowrank_16(int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
  if (a.mode & MODE_ADJ) return LA16::launch(var, a, grid, s);
  if (a.mode & MODE_GEN) return LG16::launch(var, a, grid, s);
  return (a.mode & MODE_TRACE) ? LT16::launch(var, a, grid, s) : LD16::launch(var, a, grid, s);
}
int lowrank_variants_16(int kind, int* out, int max) {
  if (kind == 3) return LG16::list(out, max);
  return kind == 2 ? LA16::list(out, max) : kind ? LT16::list(out, max) : LD16::list(out, max);
}
}  // namespace dmft
