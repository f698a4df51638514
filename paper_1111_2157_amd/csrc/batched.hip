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
// The low-rank form of the step has one persistent kernel per class of items
// (batched_lr.h).
#include "batched_lr.h"
#include "dyson64_impl.h"

namespace dmft {

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

__global__ void copy_doubles_kernel(const double* src, double* dst, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t launch_copy_doubles(const double* src, double* dst, int n, hipStream_t s) {
  hipLaunchKernelGGL(copy_doubles_kernel, dim3((n + 63) / 64), dim3(64), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace dmft
