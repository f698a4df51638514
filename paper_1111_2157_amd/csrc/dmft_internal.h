// Internal interface between the C-ABI host layer (dmft_host.cpp) and the HIP
// kernels (dmft_kernels.hip).  Not part of the public ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace dmft {

// Kernel modes (bit set).
enum : int {
  MODE_S = 1,      // accumulate sum_n G_kn into per-(frequency tile, k) partials
  MODE_GLOC = 2,   // accumulate w_k S G S^dag into per-(k tile, n) partials
  MODE_TRACE = 4,  // accumulate sum_n Re tr G and sum_n Re tr G^2 per (frequency tile, k)
  MODE_ADJ = 8,    // low-rank fused scalar adjoint: MODE_TRACE's sums (stride 3 in tpart) and
                   // w_k S G^2 S^dag per (k tile, n) in xpart
  MODE_GEN = 16,   // low-rank general vector-Jacobian product: Sigmabar_n per (k tile, n) in xpart
                   // and the mubar share per (frequency tile, k) in tpart[.][.][2] (stride 3), as
                   // the dense adjoint kernel writes them
};

// Error bits raised on the device.
enum : int { ERR_SINGULAR = 1, ERR_NONFINITE = 2, ERR_NOCONV = 4 };

// Everything one launch of the Dyson kernel needs.  Pointers are device
// pointers.  A launch covers the k-points klist[0 .. nklist) (all with
// nb_k <= NBP of the instance) and all nw frequencies, tiled as
// ceil(nklist / kt) k-tiles x n_wtiles frequency tiles of wt frequencies.
struct DysonArgs {
  int nk, nc, nw;
  int nb_uniform;              // > 0: every k has this many bands and nb/off_b are unused
  const int32_t* nb;           // [nk]
  const int64_t* off_b;        // [nk+1] prefix sums of nb
  const double* eps;
  const double* wk;
  const double* proj;          // complex
  double beta;
  const double* sigma;         // complex [nw][nc][nc]
  const double* e_dc;          // [nc]
  const double* mu_ptr;        // if non-null, mu is read from here (device scalar)
  double mu;
  const int32_t* klist;        // [nklist] or null (identity)
  int nklist;
  int kt, wt, n_wtiles;
  int ktile_base;              // index of this launch's first k tile among all k tiles
  int mode;
  double* spart;               // MODE_S: per frequency tile, per k an NBP_k^2 complex slot (lane order)
  int64_t s_stride;            // complex elements per frequency tile of spart
  const int64_t* off_s;        // [nk+1] start of k's slot within a frequency tile
  double* xpart;               // MODE_GLOC: [n_ktiles_total][nw][256] complex, lane order
  double* tpart;               // MODE_TRACE:[n_wtiles][nk][2]
  int* err;                    // error word
  const double* nbar;          // MODE_GEN: complex N(k) cotangent (N(k) layout) or null
  const int64_t* off_n;        // MODE_GEN: [nk+1] offsets into nbar (ragged) or null (uniform)
  const double* gbar;          // MODE_GEN: complex G_loc cotangent [nw][nc][nc] or null
};

struct EpilogueArgs {
  int nk, nc, nw;
  int nb_uniform;
  const int32_t* nb;
  const int64_t* off_b;
  const int64_t* off_n;        // [nk+1] prefix sums of nb^2 (output layout)
  const int32_t* nbp;          // [nk] padded size (NBP) used for k's partials
  const double* eps;
  const double* wk;
  const double* proj;
  double beta;
  const double* sigma_inf;     // complex [nc][nc] or null
  const double* e_dc;
  const double* mu_ptr;
  double mu;
  int tail_order;
  int n_wtiles;
  const double* spart;
  int64_t s_stride;            // complex elements per frequency tile of spart
  const int64_t* off_s;        // [nk+1] start of k's slot within a frequency tile
  const double* tpart;
  double* nk_out;              // complex, ragged
  double* kscal;               // [nk][3] per-k  tr N, tr(S N S^dag), sum_v E_v N_vv
  double* ktrace;              // [nk][2] per-k  tr N, d tr N / dmu   (trace mode)
  double s2;                   // sum_n 1 / w_n^2, summed in increasing n
};

// Launchers (return hipError_t of the launch).
// var: kernel variant, bit 0 = next-step pivot column read ahead (PF), bit 1 =
// running sum of G in LDS (SLDS, density kind only), bit 2 = two wavefronts per
// SIMD, bit 3 = low-rank (Woodbury) form instead of the band-window inversion
// (lowrank_impl.h; there bit 0 = projector fragments re-read at every use).  dyson_variants lists the
// instantiated variants of a size and kind (kind 0 = density, 1 = trace); the
// first one is the default.
// Low-rank codes with bit 5 set: 40 = the two-wavefront kernel for 64-band
// windows (lowrank_pair_impl.h), 42 = three frequencies per matrix-core tile for
// nc <= 5 (lowrank_p3_impl.h; 64-band windows on four wavefronts); both density
// kind only.  A launch of either outside its shapes returns hipErrorInvalidValue.
constexpr int kLowrankPairVariant = 40;
constexpr int kLowrankP3Variant = 42;
inline bool lowrank_p3_fits(int nbp, int nc) { return nc <= 5 && nbp <= 64; }
hipError_t launch_dyson(int nbp, int var, const DysonArgs& a, int n_ktiles, hipStream_t s);
int dyson_variants(int nbp, int kind, int* out, int max);
bool dyson_supported(int nbp);
hipError_t launch_nk_epilogue(const EpilogueArgs& a, double* nk_out, hipStream_t s);
hipError_t launch_trace_epilogue(const EpilogueArgs& a, hipStream_t s);
hipError_t launch_gloc_reduce(int n_ktiles, int nw, int nc, const double* xpart, double* gloc,
                              hipStream_t s);
hipError_t launch_scalar_reduce(int nk, const double* wk, const double* kvals, int nvals,
                                double* out, hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
// Adjoint kernel: gen 0 = fused scalar adjoint of N_tot (partials of w_k S G^2 S^dag),
// gen 1 = general vector-Jacobian product.  tpart: [n_wtiles][nk][3].
hipError_t launch_adjoint(int nbp, int gen, const DysonArgs& a, const double* nbar, const int64_t* off_n,
                          const double* gbar, double* mpart, double* tpart, int n_ktiles, hipStream_t s);
hipError_t launch_sigma_bar_reduce(int n_ktiles, int nw, int nc, const double* mpart, double scale, int dagger,
                                   double* out, hipStream_t s);
// Persistent batched launch over a queue of items (see batched.hip): items[0 .. n_big)
// need a two-wavefront work-group, items[n_big .. n_big + n_small) one wavefront.
struct BatchItemHost {
  int32_t args, nbp, ktile, wtile;
};
hipError_t launch_batched(const void* items, int n_big, int n_small, const DysonArgs* args, int* counters,
                          int n_workgroups, hipStream_t s);
// The low-rank form: one persistent kernel per class (padded size nbp, ncls
// columns of the row-layout inversions, lr_nc_class) over items[0 .. n_items),
// pulling from *counter (reset to 0 before the launch); grid work-groups of 64
// threads, or for nbp = 64 128 (two-wavefront items) or 256 (class 5, four).
int lr_nc_class(int nbp, int nc);
int lr_class_wgs_per_cu(int nbp, int ncls);  // resident work-groups per CU of a class kernel
hipError_t launch_lr_class(int nbp, int ncls, const void* items, int n_items, const DysonArgs* args, int* counter,
                           int grid, hipStream_t s);
hipError_t launch_copy_doubles(const double* src, double* dst, int n, hipStream_t s);
// Allocation-free entry point (noalloc.hip): the library's device scratch array.
// noalloc_setup looks up its address on `device` (current) once per device;
// noalloc_scratch returns it (nullptr before setup), noalloc_scratch_bytes its size.
hipError_t noalloc_setup(int device);
void* noalloc_scratch(int device);
size_t noalloc_scratch_bytes();
// Per-k metadata of a uniform lattice (nb bands, padded size nbp) and a cleared error word.
hipError_t launch_uniform_meta(int nk, int nb, int nbp, int32_t* nbv, int64_t* offb, int64_t* offn, int32_t* nbpv,
                               int32_t* klist, int64_t* offs, int* err, hipStream_t s);
// status[0] = DMFT_ESINGULAR, DMFT_ENONFINITE or DMFT_OK from the error word.
hipError_t launch_status_code(const int* err, int32_t* status, hipStream_t s);
// DMFT self-consistency step: E_imp (device [nc][nc] complex) and Delta (device [nw][nc][nc]);
// part holds self_consistency_parts(nk) x nc x nc complex partials of E_imp.
constexpr int kScParts = 1024;
int self_consistency_parts(int nk);
hipError_t launch_self_consistency(int nk, int nc, int nw, int nb_uniform, const int32_t* nb, const int64_t* off_b,
                                   const double* eps, const double* wk, const double* proj, const double* e_dc,
                                   double beta, double mu, const double* gloc, const double* sigma, double* e_imp,
                                   double* delta, double* part, int* err, hipStream_t s);
// Per-k [tr N, d tr N/dmu, mubar_k] from the adjoint partials (tail terms included).
hipError_t launch_adj_epilogue(const EpilogueArgs& a, const double* nbar, hipStream_t s);
// out[j] = sum_k weight_j(k) kvals[k][j], weight = w_k, or 1 where bit j of unit_mask is set.
hipError_t launch_scalar_reduce_mask(int nk, const double* wk, const double* kvals, int nvals, int unit_mask,
                                     double* out, hipStream_t s);


// Pole-expansion route (pseudo-Hamiltonian eigensystems).  Pointers are device
// pointers; mp = nb_max + np is the padded stride of the per-k outputs.
struct PoleArgs {
  int nk, nc, np, mp, nb_max;
  int nb_uniform;              // > 0: every k has this many bands and nb/off_b are unused
  const int32_t* nb;
  const int64_t* off_b;
  const int64_t* off_n;        // [nk+1] prefix sums of nb^2 (N(k) output layout)
  const double* eps;
  const double* wk;
  const double* proj;          // complex [nc][nb_k] per k
  const double* p;             // [np] pole positions
  const double* v;             // complex [np][nc] pole vectors
  const double* sigma_inf;     // complex [nc][nc] or null
  const double* e_dc;          // [nc]
  double beta;
  double* evals;               // [nk][mp]
  double* evecs;               // complex [nk][nb_max][mp]
  double* wphys;               // [nk][mp]
  double* worb;                // [nk][mp][nc] or null
  int* sweeps;                 // [nk] Jacobi sweeps taken
  int* err;
  int max_sweeps;
};
// Dynamic LDS bytes of the eigensolver for one k with nb bands.
size_t pole_eig_lds_bytes(int nb, int np);
hipError_t launch_pole_eig(const PoleArgs& a, size_t lds_bytes, hipStream_t s);
// N(k) = sum_l u_l u_l^dag f(lam_l - mu) with f = n_F (nw_trunc = 0) or the
// truncated Matsubara weight f_Nw; per-k [tr N, tr S N S^dag, sum_v E_v N_vv] into kscal.
hipError_t launch_pole_density(const PoleArgs& a, double mu, int nw_trunc, double* nk_out, double* kscal,
                               hipStream_t s);
// Safeguarded Newton (method 0) or bisection (1) for sum_k w_k sum_l w_l n_F(lam_l - mu) = n_target,
// one work-group; res = [mu, N(mu), passes, status (0 converged, 1 not)].
hipError_t launch_pole_find_mu(const PoleArgs& a, double n_target, double tol, int method, double lo, double hi,
                               double mu0, int max_iter, double* res, hipStream_t s);
// Lorentzian-broadened DOS and PDOS on ne energies in [e_min, e_max]; part holds
// [kslices][ne][1 + nc] partial sums.
int pole_dos_kslices(int nk, int mp);
hipError_t launch_pole_dos(const PoleArgs& a, double mu, double eta, double e_min, double e_max, int ne,
                           double* part, double* dos, double* pdos, hipStream_t s);
// Energy-functional sums; part holds pole_energy_parts(nk, mp) x (3 + nc) partials,
// out = [B, N_tot, <H_KS>, <V_DC>, <H_U>, n_a (nc)].
int pole_energy_parts(int nk, int mp);
hipError_t launch_pole_energy(const PoleArgs& a, double mu, double* part, double* out, hipStream_t s);
// Hubbard-I atoms (one work-group per atom and orbital) and the Matsubara-axis
// self-energy of a pole form.
hipError_t launch_hubbard1(int natoms, int nc, const double* eps, const double* U, const double* mu, double beta,
                           double wtol, double* sigma_inf, int32_t* npoles, double* pos, double* wgt, double* occ,
                           double* e_u, hipStream_t s);
hipError_t launch_sigma_from_poles(int nw, int nc, int np, double beta, double mu, const double* p, const double* v,
                                   const double* sinf, double* sigma, hipStream_t s);
hipError_t launch_hubbard1_poles(int nc, int nc_lat, int a0, const int32_t* npoles, const double* pos,
                                 const double* wgt, double* p, double* v, int32_t* np_out, hipStream_t s);

}  // namespace dmft
