// Instantiation unit of the low-rank Dyson kernel (lowrank_impl.h), one
// wavefront per work item for every padded band-window size.
//
// Variant id: bit 3 set (low-rank form); projector fragments kept in
// registers for the whole k-point (bits 0 and 4 clear), re-read at every use
// (bit 0) or loaded once per four-frequency group at the start of each stage
// (bit 4); bit 1 = three-product complex arithmetic on the matrix cores;
// bit 2 = two wavefronts per SIMD.  Each (size, kind) lists the combinations
// that compile without register spills.
#include "lowrank_impl.h"

namespace dmft {

template <int NBP, int KIND, int... VARS>
struct LRSet {
  template <int VAR>
  static hipError_t one(const DysonArgs& a, dim3 grid, hipStream_t s) {
    constexpr int parts = (NBP / 16) / lr_col_tiles<NBP, KIND>();
    constexpr int rl = (VAR & 16) ? 1 : (VAR & 1) ? 2 : 0;
    constexpr bool m3 = (VAR & 2) != 0;
    constexpr int occ = (VAR & 4) ? 2 : 1;
    grid.x *= parts;
    hipLaunchKernelGGL((lr_kernel<NBP, KIND, rl, m3, occ>), grid, dim3(64), 0, s, a);
    return hipGetLastError();
  }
  static hipError_t launch(int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
    hipError_t r = hipErrorInvalidValue;
    bool hit = ((var == VARS ? (r = one<VARS>(a, grid, s), true) : false) || ...);
    (void)hit;
    return r;
  }
  static int list(int* out, int max) {
    int n = 0;
    ((n < max ? (out[n++] = VARS, 0) : 0), ...);
    return n;
  }
};

using LD16 = LRSet<16, KIND_DENSITY, 14, 8, 10, 26, 30>;
using LD32 = LRSet<32, KIND_DENSITY, 10, 8, 24, 26, 9, 11>;
using LD48 = LRSet<48, KIND_DENSITY, 8, 24, 26, 9, 11>;
using LD64 = LRSet<64, KIND_DENSITY, 24, 9, 11>;
using LT16 = LRSet<16, KIND_TRACE, 14, 12, 13, 15, 28, 30>;
using LT32 = LRSet<32, KIND_TRACE, 14, 12, 28, 30, 13, 15>;
using LT48 = LRSet<48, KIND_TRACE, 15, 13, 8, 10, 24, 26>;
using LT64 = LRSet<64, KIND_TRACE, 13, 9, 11, 8, 10, 24>;

hipError_t launch_lowrank(int nbp, int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
  const bool tr = (a.mode & MODE_TRACE) != 0;
  switch (nbp) {
    case 16: return tr ? LT16::launch(var, a, grid, s) : LD16::launch(var, a, grid, s);
    case 32: return tr ? LT32::launch(var, a, grid, s) : LD32::launch(var, a, grid, s);
    case 48: return tr ? LT48::launch(var, a, grid, s) : LD48::launch(var, a, grid, s);
    case 64: return tr ? LT64::launch(var, a, grid, s) : LD64::launch(var, a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

int lowrank_variants(int nbp, int kind, int* out, int max) {
  if (max <= 0) return 0;
  switch (nbp) {
    case 16: return kind ? LT16::list(out, max) : LD16::list(out, max);
    case 32: return kind ? LT32::list(out, max) : LD32::list(out, max);
    case 48: return kind ? LT48::list(out, max) : LD48::list(out, max);
    case 64: return kind ? LT64::list(out, max) : LD64::list(out, max);
    default: return 0;
  }
}

}  // namespace dmft
