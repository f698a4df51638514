// Persistent batched Dyson kernel: one launch walks a cost-sorted queue of
// (self-energy iterate, padded band-window size, k-tile, frequency-tile)
// work items with uneven band windows.
//
// Work-groups hold two wavefronts.  Phase 1 pulls the 64-band items, which
// need both wavefronts (dyson64_impl.h), one item per work-group at a time.
// When that queue is drained the two wavefronts part and, in phase 2, each
// pulls single-wavefront items (16-, 32- and 48-band windows) on its own
// from the second queue until it is empty; no work-group barrier is executed
// in phase 2.  Every wavefront reaches the end of both queues, so the grid
// always drains.  Queue counters are reset by a small kernel before each pass.
//
// batched_lr_kernel is the same persistent walk for the low-rank form of the
// step (lowrank_impl.h), where every band-window size fits one wavefront:
// single-wavefront work-groups pull items of any size from one queue.
#include "dyson64_impl.h"
#include "lowrank_impl.h"

namespace dmft {

struct BatchItem {
  int32_t args;   // index into the per-(iterate, size) argument array
  int32_t nbp;    // padded band-window size of the item
  int32_t ktile;  // k-tile within that (iterate, size) launch
  int32_t wtile;  // frequency tile
};

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
// Per-wavefront LDS slot of phase 2: large enough for every single-wavefront size,
// so the two wavefronts never overlap whatever sizes they are working on.
constexpr size_t kSlot = (cmax(sizeof(KernelShared<48, KIND_DENSITY, 1>),
                               cmax(sizeof(KernelShared<32, KIND_DENSITY, 1>), sizeof(KernelShared<16, KIND_DENSITY, 0>))) +
                          15) / 16 * 16;
constexpr size_t kBatchLds = cmax(sizeof(d64::Shared), 2 * kSlot);

__global__ void __launch_bounds__(128) batched_kernel(const BatchItem* items, int n_big, int n_small,
                                                      const DysonArgs* args, int* counters) {
  __shared__ __attribute__((aligned(16))) char raw[kBatchLds];
  __shared__ int next;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) next = atomicAdd(&counters[0], 1);
    __syncthreads();
    const int it = next;
    __syncthreads();
    if (it >= n_big) break;
    const BatchItem b = items[it];
    const DysonArgs a = args[b.args];
    d64::tile<KIND_DENSITY>(a, b.ktile, b.wtile, *reinterpret_cast<d64::Shared*>(raw), tid);
    __syncthreads();
  }
  const int w = tid >> 6, lane = tid & 63;
  for (;;) {
    int it = 0;
    if (lane == 0) it = atomicAdd(&counters[1], 1);
    it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
    if (it >= n_small) break;
    const BatchItem b = items[n_big + it];
    const DysonArgs a = args[b.args];
    switch (b.nbp) {
      case 48:
        dyson_tile<48, KIND_DENSITY, 0, 1>(a, b.ktile, b.wtile,
                                           *reinterpret_cast<KernelShared<48, KIND_DENSITY, 1>*>(raw + w * kSlot), lane);
        break;
      case 32:
        dyson_tile<32, KIND_DENSITY, 1, 1>(a, b.ktile, b.wtile,
                                           *reinterpret_cast<KernelShared<32, KIND_DENSITY, 1>*>(raw + w * kSlot), lane);
        break;
      default:
        dyson_tile<16, KIND_DENSITY, 1, 0>(a, b.ktile, b.wtile,
                                           *reinterpret_cast<KernelShared<16, KIND_DENSITY, 0>*>(raw + w * kSlot), lane);
        break;
    }
  }
}

hipError_t launch_batched(const void* items, int n_big, int n_small, const DysonArgs* args, int* counters,
                          int n_workgroups, hipStream_t s) {
  hipLaunchKernelGGL(batched_kernel, dim3(n_workgroups), dim3(128), 0, s, reinterpret_cast<const BatchItem*>(items),
                     n_big, n_small, args, counters);
  return hipGetLastError();
}

// One low-rank work item of the batched queue, per padded size.  All paths
// share one kernel's register allocation; these choices (projector fragments
// per use for 64 bands, per stage for 48, kept for 32 and 16) were the fastest
// measured.
template <int NC>
__device__ __forceinline__ void lr_batched_item(const DysonArgs& a, const BatchItem& b, int part, LRShared& sh,
                                                int lane) {
  switch (b.nbp & 255) {
    case 64: lr_tile<64, KIND_DENSITY, 2, true, NC>(a, b.ktile, b.wtile, part, sh, lane); break;
    case 48: lr_tile<48, KIND_DENSITY, 1, false, NC>(a, b.ktile, b.wtile, 0, sh, lane); break;
    case 32: lr_tile<32, KIND_DENSITY, 0, true, NC>(a, b.ktile, b.wtile, 0, sh, lane); break;
    default: lr_tile<16, KIND_DENSITY, 0, true, NC>(a, b.ktile, b.wtile, 0, sh, lane); break;
  }
}

__global__ void __launch_bounds__(64) batched_lr_kernel(const BatchItem* items, int n_items, const DysonArgs* args,
                                                        int* counters) {
  __shared__ LRShared sh;
  const int lane = threadIdx.x;
  for (;;) {
    int it = 0;
    if (lane == 0) it = atomicAdd(&counters[0], 1);
    it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
    if (it >= n_items) break;
    const BatchItem b = items[it];
    const DysonArgs a = args[b.args];
    // nbp: padded size in the low byte, column part of a 64-band item in bit 8,
    // bit 9 set when nc <= 8 and bit 10 when 8 < nc <= 14 (row-layout
    // inversions over 8 or 14 columns, else 16)
    const int part = (b.nbp >> 8) & 1;
    if (b.nbp & 512)
      lr_batched_item<8>(a, b, part, sh, lane);
    else if (b.nbp & 1024)
      lr_batched_item<14>(a, b, part, sh, lane);
    else
      lr_batched_item<16>(a, b, part, sh, lane);
  }
}

hipError_t launch_batched_lr(const void* items, int n_items, const DysonArgs* args, int* counters, int n_workgroups,
                             hipStream_t s) {
  hipLaunchKernelGGL(batched_lr_kernel, dim3(n_workgroups), dim3(64), 0, s,
                     reinterpret_cast<const BatchItem*>(items), n_items, args, counters);
  return hipGetLastError();
}

__global__ void copy_doubles_kernel(const double* src, double* dst, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t launch_copy_doubles(const double* src, double* dst, int n, hipStream_t s) {
  hipLaunchKernelGGL(copy_doubles_kernel, dim3((n + 63) / 64), dim3(64), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace dmft
