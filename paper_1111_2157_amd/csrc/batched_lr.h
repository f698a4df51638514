// Persistent kernels of the batched pass in the low-rank form: one kernel per
// class of work items (padded band-window size, columns of the row-layout
// inversions), each draining its own cost-sorted queue of (iterate, k tile,
// frequency tile) items from every self-energy iterate.  A class kernel has
// the register allocation and occupancy of its own size only; 64-band items
// run on two-wavefront work-groups (lowrank_pair_impl.h), the others on one
// wavefront (lr_tile of lowrank_impl.h, with the variant that is fastest for
// that size on its own, or for nc <= 5 lr_p3_tile of lowrank_p3_impl.h; 64-band
// items with nc <= 5 run on four wavefronts, lr_p3_quad_tile).  The classes are launched one after another on one
// stream, largest items first; every work-group pulls items until its queue
// is empty, so each launch drains.
#pragma once

#include "lowrank_p3_impl.h"
#include "lowrank_pair_impl.h"

namespace dmft {

struct BatchItem {
  int32_t args;   // index into the per-(iterate, size) argument array
  int32_t nbp;    // padded band-window size of the item
  int32_t ktile;  // k-tile within that (iterate, size) launch
  int32_t wtile;  // frequency tile
};

// Single-wavefront class: NBP in {16, 32, 48}; PF: the partial-fraction form of
// the running sum (lowrank_impl.h), with its LDS slots for close-pair sums.
template <int NBP, int RL, bool M3, int NC, bool PF = false>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1)))
lr_class_kernel(const BatchItem* items, int n_items, const DysonArgs* args, int* counter) {
  __shared__ LRShared sh;
  __shared__ double2 pfc[PF ? NBP / 16 * 4 * 64 : 1];
  const int lane = threadIdx.x;
  for (;;) {
    int it = 0;
    if (lane == 0) it = atomicAdd(counter, 1);
    it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
    if (it >= n_items) break;
    const BatchItem b = items[it];
    const DysonArgs a = args[b.args];
    lr_tile<NBP, KIND_DENSITY, RL, M3, NC, PF>(a, b.ktile, b.wtile, 0, sh, lane, pfc);
  }
}

// Single-wavefront class for nc <= 5, three frequencies per matrix-core tile
// (lowrank_p3_impl.h): NBP in {16, 32, 48}; PF: the partial-fraction form of
// the running sum, with its LDS slots for close-pair sums.
template <int NBP, int RL, bool M3, bool PF = false>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1)))
lr_p3_class_kernel(const BatchItem* items, int n_items, const DysonArgs* args, int* counter) {
  __shared__ LRP3Shared<NBP> sh;
  __shared__ double2 pfc[PF ? NBP / 16 * 4 * 64 : 1];
  const int lane = threadIdx.x;
  for (;;) {
    int it = 0;
    if (lane == 0) it = atomicAdd(counter, 1);
    it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
    if (it >= n_items) break;
    const BatchItem b = items[it];
    const DysonArgs a = args[b.args];
    lr_p3_tile<NBP, RL, M3, PF>(a, b.ktile, b.wtile, sh, lane, pfc);
  }
}

// Four-wavefront class for 64-band windows and nc <= 5 (lr_p3_quad_tile; a
// template so that the header defines no kernel of its own).
template <int NBP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1)))
lr_p3_quad_class_kernel(const BatchItem* items, int n_items, const DysonArgs* args, int* counter) {
  __shared__ LRP3QuadShared sh;
  __shared__ int next;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
    if (it >= n_items) break;
    const BatchItem b = items[it];
    const DysonArgs a = args[b.args];
    static_assert(NBP == 64, "four-wavefront items are 64-band windows");
    lr_p3_quad_tile<true>(a, b.ktile, b.wtile, sh, tid);
  }
}

// Two-wavefront class for 64-band windows.
template <int NC>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(1)))
lr_pair_class_kernel(const BatchItem* items, int n_items, const DysonArgs* args, int* counter) {
  __shared__ LRPairShared sh;
  __shared__ int next;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    // uniform by construction; readfirstlane tells the compiler, so the item and
    // its arguments are read into scalar registers
    const int it = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
    if (it >= n_items) break;
    const BatchItem b = items[it];
    const DysonArgs a = args[b.args];
    lr_pair_tile<NC, (NC >= 12)>(a, b.ktile, b.wtile, sh, tid);
  }
}

}  // namespace dmft
