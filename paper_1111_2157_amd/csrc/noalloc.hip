// Scratch memory of the allocation-free entry point (density_matrix_noalloc).
//
// The workspace that density_matrix takes from its caller (error word, per-k
// metadata, partial sums) lives here in a file-scope device array instead, so
// that the entry point makes no allocating call.  Each GPU the library runs on
// holds its own copy of the array for the life of the process.  In host code
// the array's name is only a stand-in: its device address on each GPU is
// looked up once (noalloc_setup, from dmft_create with that device current)
// and kept per device; every host use goes through that address.  All calls
// on one GPU share the array, which keeps the last call's contents: the error
// word is cleared by a kernel at the start of every call, and calls that
// overlap on one GPU race.
#include <mutex>
#include <vector>

#include "dmft.h"
#include "dmft_internal.h"

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU

static __device__ __align__(256) char scratch[kScratchBytes];

namespace dmft {

namespace {

std::mutex g_mutex;
std::vector<void*> g_ptr;  // device address of `scratch`, per device

__global__ void uniform_meta_kernel(int nk, int nb, int nbp, int32_t* nbv, int64_t* offb, int64_t* offn,
                                    int32_t* nbpv, int32_t* klist, int64_t* offs, int* err) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) *err = 0;
  if (k > nk) return;
  offb[k] = (int64_t)k * nb;
  offn[k] = (int64_t)k * nb * nb;
  offs[k] = (int64_t)k * nbp * nbp;
  if (k < nk) {
    nbv[k] = nb;
    nbpv[k] = nbp;
    klist[k] = k;
  }
}

__global__ void status_code_kernel(const int* err, int32_t* status) {
  const int e = *err;
  *status = (e & ERR_SINGULAR) ? DMFT_ESINGULAR : (e & ERR_NONFINITE) ? DMFT_ENONFINITE : DMFT_OK;
}

}  // namespace

hipError_t noalloc_setup(int device) {
  std::lock_guard<std::mutex> lock(g_mutex);
  if ((int)g_ptr.size() <= device) g_ptr.resize(device + 1, nullptr);
  if (g_ptr[device]) return hipSuccess;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_ptr[device] = p;
  return hipSuccess;
}

void* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_mutex);
  return device >= 0 && device < (int)g_ptr.size() ? g_ptr[device] : nullptr;
}

size_t noalloc_scratch_bytes() { return kScratchBytes; }

hipError_t launch_uniform_meta(int nk, int nb, int nbp, int32_t* nbv, int64_t* offb, int64_t* offn, int32_t* nbpv,
                               int32_t* klist, int64_t* offs, int* err, hipStream_t s) {
  hipLaunchKernelGGL(uniform_meta_kernel, dim3((nk + 1 + 255) / 256), dim3(256), 0, s, nk, nb, nbp, nbv, offb, offn,
                     nbpv, klist, offs, err);
  return hipGetLastError();
}

hipError_t launch_status_code(const int* err, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(status_code_kernel, dim3(1), dim3(1), 0, s, err, status);
  return hipGetLastError();
}

}  // namespace dmft
