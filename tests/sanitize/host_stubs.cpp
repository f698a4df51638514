// Stand-ins for the device side of libdmft, for a host-only build of the C-ABI
// layer (dmft_host.cpp) under AddressSanitizer / UndefinedBehaviorSanitizer
// (tests/test_sanitizers.py).  Every launcher fails: the driver uses a
// planning handle, which the host layer refuses before any launch.  The few
// host-side size queries return the shapes' simple bounds.
#include "dmft_internal.h"

namespace dmft {

bool dyson_supported(int nbp) { return nbp == 16 || nbp == 32 || nbp == 48 || nbp == 64; }
int dyson_variants(int nbp, int kind, int* out, int max) {
  if (!dyson_supported(nbp) || kind < 0 || kind > 3 || max < 1) return 0;
  out[0] = 8;
  return 1;
}
int lr_nc_class(int, int nc) { return nc <= 5 ? 5 : nc <= 8 ? 8 : 16; }
int lr_class_wgs_per_cu(int nbp, int ncls) { return nbp < 64 ? 4 : ncls == 5 ? 1 : 2; }
size_t pole_eig_lds_bytes(int nb, int np) { return (size_t)(nb + np + 1) * (nb + np + 1) * 16; }
int pole_dos_kslices(int nk, int) { return nk < 8 ? nk : 8; }
int pole_energy_parts(int nk, int) { return nk < 64 ? nk : 64; }
size_t noalloc_scratch_bytes() { return size_t(64) << 20; }
void* noalloc_scratch(int) { return nullptr; }
hipError_t noalloc_setup(int) { return hipErrorInvalidValue; }

#define FAIL(...) \
  { return hipErrorInvalidValue; }
hipError_t launch_dyson(int, int, const DysonArgs&, int, hipStream_t) FAIL()
hipError_t launch_nk_epilogue(const EpilogueArgs&, double*, hipStream_t) FAIL()
hipError_t launch_trace_epilogue(const EpilogueArgs&, hipStream_t) FAIL()
hipError_t launch_gloc_reduce(int, int, int, const double*, double*, hipStream_t) FAIL()
hipError_t launch_scalar_reduce(int, const double*, const double*, int, double*, hipStream_t) FAIL()
hipError_t launch_scalar_reduce_mask(int, const double*, const double*, int, int, double*, hipStream_t) FAIL()
hipError_t launch_fill_zero(void*, size_t, hipStream_t) FAIL()
hipError_t launch_adjoint(int, int, const DysonArgs&, const double*, const int64_t*, const double*, double*, double*,
                          int, hipStream_t) FAIL()
hipError_t launch_sigma_bar_reduce(int, int, int, const double*, double, int, double*, hipStream_t) FAIL()
hipError_t launch_batched(const void*, int, int, const DysonArgs*, int*, int, hipStream_t) FAIL()
hipError_t launch_lr_class(int, int, const void*, int, const DysonArgs*, int*, int, hipStream_t) FAIL()
hipError_t launch_copy_doubles(const double*, double*, int, hipStream_t) FAIL()
hipError_t launch_self_consistency(int, int, int, int, const int32_t*, const int64_t*, const double*, const double*,
                                   const double*, const double*, double, double, const double*, const double*, double*,
                                   double*, double*, int*, hipStream_t) FAIL()
hipError_t launch_adj_epilogue(const EpilogueArgs&, const double*, hipStream_t) FAIL()
hipError_t launch_pole_eig(const PoleArgs&, size_t, hipStream_t) FAIL()
hipError_t launch_pole_density(const PoleArgs&, double, int, double*, double*, hipStream_t) FAIL()
hipError_t launch_pole_find_mu(const PoleArgs&, double, double, int, double, double, double, int, double*,
                               hipStream_t) FAIL()
hipError_t launch_pole_dos(const PoleArgs&, double, double, double, double, int, double*, double*, double*,
                           hipStream_t) FAIL()
hipError_t launch_pole_energy(const PoleArgs&, double, double*, double*, hipStream_t) FAIL()
hipError_t launch_hubbard1(int, int, const double*, const double*, const double*, double, double, double*, int32_t*,
                           double*, double*, double*, double*, hipStream_t) FAIL()
hipError_t launch_sigma_from_poles(int, int, int, double, double, const double*, const double*, const double*, double*,
                                   hipStream_t) FAIL()
hipError_t launch_hubbard1_poles(int, int, int, const int32_t*, const double*, const double*, double*, double*,
                                 int32_t*, hipStream_t) FAIL()
hipError_t launch_uniform_meta(int, int, int, int32_t*, int64_t*, int64_t*, int32_t*, int32_t*, int64_t*, int*,
                               hipStream_t) FAIL()
hipError_t launch_status_code(const int*, int32_t*, hipStream_t) FAIL()

}  // namespace dmft
