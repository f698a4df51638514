// Drives the C-ABI host layer through a planning handle (no device) for the
// sanitizer build: argument checks, ragged-window bucketing and workspace
// sizing of every entry point family, and the refusals before any launch.
// Exits 0 when every call returns the expected status; the sanitizers abort
// the process on a memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "dmft.h"

static int failures = 0;
#define EXPECT(cond)                                                       \
  do {                                                                     \
    if (!(cond)) {                                                         \
      std::fprintf(stderr, "line %d: expected %s\n", __LINE__, #cond);     \
      ++failures;                                                          \
    }                                                                      \
  } while (0)

// Addresses the planning handle only checks for being set (never dereferenced).
static void* fake(int i) { return reinterpret_cast<void*>(0x7f0000000000ull + 256ull * (unsigned)i); }

int main() {
  dmft_handle h = nullptr;
  EXPECT(dmft_create(&h, DMFT_NO_DEVICE) == DMFT_OK && h);

  std::vector<int32_t> nb;
  for (int v = 5; v <= 64; ++v) nb.push_back(v);  // every padded size, both ends of each
  dmft_lattice lat{(int32_t)nb.size(), 5, 64, nb.data(), (const double*)fake(1), (const double*)fake(2),
                   (const double*)fake(3)};
  dmft_sigma sig{48, 20.0, (const double*)fake(4), nullptr, (const double*)fake(5)};
  size_t bytes = 0;
  EXPECT(dmft_workspace_size(h, &lat, &sig, &bytes) == DMFT_OK && bytes > 0 && bytes % 256 == 0);

  // host checks
  dmft_lattice bad = lat;
  bad.nk = 0;
  EXPECT(dmft_workspace_size(h, &bad, &sig, &bytes) == DMFT_EINVAL);
  bad = lat;
  bad.nc = 17;
  EXPECT(dmft_workspace_size(h, &bad, &sig, &bytes) == DMFT_EINVAL);
  std::vector<int32_t> nb2 = nb;
  nb2[3] = 2;
  bad = lat;
  bad.nb = nb2.data();
  EXPECT(dmft_workspace_size(h, &bad, &sig, &bytes) == DMFT_EINVAL);
  EXPECT(std::strstr(dmft_last_error(h), "outside nc..nb_max") != nullptr);
  dmft_sigma bs = sig;
  bs.beta = NAN;
  EXPECT(dmft_workspace_size(h, &lat, &bs, &bytes) == DMFT_EINVAL);

  // every launching entry point: argument errors first, then the missing device
  void* ws = fake(100);
  double* out = (double*)fake(200);
  EXPECT(density_matrix(h, &lat, &sig, 0.0, 1, out, nullptr, nullptr, ws, bytes, nullptr) == DMFT_EINVAL);
  EXPECT(density_matrix(h, &lat, &sig, 0.0, 2, out, nullptr, nullptr, ws, bytes - 1, nullptr) == DMFT_EWORKSPACE);
  EXPECT(density_matrix(h, &lat, &sig, 0.0, 2, out, nullptr, nullptr, ws, bytes, nullptr) == DMFT_EINVAL);
  EXPECT(std::strstr(dmft_last_error(h), "planning handle") != nullptr);
  EXPECT(gloc_compute(h, &lat, &sig, 0.0, out, ws, bytes, nullptr) == DMFT_EINVAL);
  EXPECT(dmft_ntot(h, &lat, &sig, 0.0, 0, out, ws, bytes, nullptr) == DMFT_EINVAL);
  EXPECT(dmft_ntot_vjp(h, &lat, &sig, 0.0, 2, out, out, ws, bytes, nullptr) == DMFT_EINVAL);
  EXPECT(density_matrix_vjp(h, &lat, &sig, 0.0, 2, nullptr, nullptr, out, nullptr, ws, bytes, nullptr) ==
         DMFT_EINVAL);
  double mu = 0, n = 0;
  int passes = 0;
  EXPECT(find_mu(h, &lat, &sig, 2, 3.0, 1e-8, DMFT_NEWTON, 1.0, -1.0, 0.0, 10, &mu, &passes, &n, ws, bytes,
                 nullptr) == DMFT_EINVAL);
  EXPECT(find_mu(h, &lat, &sig, 2, 3.0, 1e-8, DMFT_NEWTON, -1.0, 1.0, 0.0, 10, &mu, &passes, &n, ws, bytes,
                 nullptr) == DMFT_EINVAL);
  EXPECT(dmft_hybridization(h, &lat, &sig, 0.0, out, out, nullptr, ws, bytes, nullptr) == DMFT_EINVAL);
  char rep[64];
  EXPECT(dmft_autotune(h, &lat, &sig, 0.0, ws, bytes, nullptr, rep, sizeof rep) == DMFT_EINVAL);
  EXPECT(density_matrix_noalloc(h, &lat, &sig, 0.0, 2, out, nullptr, nullptr, nullptr, nullptr) == DMFT_EINVAL);
  dmft_lattice uni = lat;
  uni.nb = nullptr;
  EXPECT(density_matrix_noalloc(h, &uni, &sig, 0.0, 2, out, nullptr, nullptr, nullptr, nullptr) == DMFT_EINVAL);
  EXPECT(std::strstr(dmft_last_error(h), "planning handle") != nullptr);

  // batched plan over two iterates with different nc
  dmft_lattice l14 = lat;
  l14.nc = 14;
  std::vector<int32_t> nb14;
  for (int v = 14; v <= 64; ++v) nb14.push_back(v);
  l14.nk = (int32_t)nb14.size();
  l14.nb = nb14.data();
  const dmft_lattice* lats[2] = {&lat, &l14};
  const dmft_sigma* sigs[2] = {&sig, &sig};
  size_t bb = 0;
  EXPECT(dmft_batched_workspace_size(h, 2, lats, sigs, &bb) == DMFT_OK && bb > bytes);
  EXPECT(dmft_batched_plan(h, 2, lats, sigs, 2, ws, bb, nullptr) == DMFT_EINVAL);
  EXPECT(dmft_batched_classes(h, 0, nullptr, nullptr, nullptr, nullptr) == 0);

  // pole route sizing
  dmft_poles pol{10, 20.0, (const double*)fake(6), (const double*)fake(7), nullptr, (const double*)fake(8)};
  dmft_lattice l16 = lat;
  l16.nb = nullptr;
  l16.nb_max = 60;
  size_t pb = 0;
  EXPECT(dmft_pole_workspace_size(h, &l16, &pol, 101, &pb) == DMFT_OK && pb > 0);
  pol.np = 30;  // nb_max + np > 80
  EXPECT(dmft_pole_workspace_size(h, &l16, &pol, 101, &pb) != DMFT_OK);

  // variant bookkeeping and timing need no device either
  int32_t v[16];
  EXPECT(dmft_variants(0, 32, (int*)v, 16) >= 1);
  EXPECT(dmft_set_variant(h, 0, 32, 12345) == DMFT_EINVAL);
  double kms = -1;
  int64_t launches = -1;
  EXPECT(dmft_timing(h, 1, &kms, &launches) == DMFT_OK && launches == 0);
  EXPECT(dmft_strerror(DMFT_ESINGULAR) != nullptr && dmft_strerror(12345) != nullptr);

  EXPECT(dmft_destroy(h) == DMFT_OK);
  if (failures) std::fprintf(stderr, "%d expectation(s) failed\n", failures);
  else std::printf("host driver ok\n");
  return failures ? 1 : 0;
}
