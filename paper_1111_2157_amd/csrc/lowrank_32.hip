// Instantiation unit of the low-rank Dyson kernel (lowrank_impl.h) for band
// windows padded to 32: the variants that compile without register spills.
#include "lowrank_impl.h"

namespace dmft {
using LD32 = LRSet<32, KIND_DENSITY, 10, 8, 24, 26, 9, 11, 74>;
using LA32 = LRSet<32, KIND_ADJ, 10, 8, 26>;
using LG32 = LRSet<32, KIND_GEN, 8, 9, 24>;
using LT32 = LRSet<32, KIND_TRACE, 14, 12, 28, 30, 13, 15>;
hipError_t launch_lowrank_32(int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
  if (a.mode & MODE_ADJ) return LA32::launch(var, a, grid, s);
  if (a.mode & MODE_GEN) return LG32::launch(var, a, grid, s);
  return (a.mode & MODE_TRACE) ? LT32::launch(var, a, grid, s) : LD32::launch(var, a, grid, s);
}
int lowrank_variants_32(int kind, int* out, int max) {
  if (kind == 3) return LG32::list(out, max);
  return kind == 2 ? LA32::list(out, max) : kind ? LT32::list(out, max) : LD32::list(out, max);
}
}  // namespace dmft
