// Instantiation unit of the low-rank Dyson kernel (lowrank_impl.h) for band
// windows padded to 64: the variants that compile without register spills.
#include "lowrank_impl.h"

namespace dmft {
using LD64 = LRSet<64, KIND_DENSITY, 24, 9, 11>;
using LA64 = LRSet<64, KIND_ADJ, 10, 8, 26>;
using LG64 = LRSet<64, KIND_GEN, 9>;
using LT64 = LRSet<64, KIND_TRACE, 13, 9, 11, 8, 10, 24>;
hipError_t launch_lowrank_64(int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
  if (a.mode & MODE_ADJ) return LA64::launch(var, a, grid, s);
  if (a.mode & MODE_GEN) return LG64::launch(var, a, grid, s);
  return (a.mode & MODE_TRACE) ? LT64::launch(var, a, grid, s) : LD64::launch(var, a, grid, s);
}
int lowrank_variants_64(int kind, int* out, int max) {
  if (kind == 3) return LG64::list(out, max);
  return kind == 2 ? LA64::list(out, max) : kind ? LT64::list(out, max) : LD64::list(out, max);
}
}  // namespace dmft
