/*
 * dmft.h - C ABI of the MI355X lattice Dyson library (libdmft.so).
 *
 * The library computes the lattice Dyson step of charge-self-consistent
 * LDA+DMFT (Zhao et al., "Implementation of LDA+DMFT with pseudo-potential-
 * plane-wave method"), for every k-point of a band window and every positive
 * fermionic Matsubara frequency w_n = (2n+1) pi / beta, n = 0 .. nw-1:
 *
 *   A_kn     = (i w_n + mu) I - diag(E_k) - S_k^dag (Sigma(i w_n) - diag(V_DC)) S_k
 *                                      (Sec. 3.2.2 eq. dmftloop1 in the band window,
 *                                       embedding of Sec. 3.2 eq. f_operation,
 *                                       V_DC sign of Sec. 3.3 eq. rho_LDA+DMFT)
 *   G_kn     = A_kn^{-1}
 *   G_loc(n) = sum_k w_k S_k G_kn S_k^dag               (Sec. 3.2.2 eq. dmftloop2)
 *   M1_k     = diag(E_k) - mu I + S_k^dag (Sigma_inf - diag(V_DC)) S_k
 *   N(k)     = 1/2 I - (beta/4) M1_k + (1/beta) sum_n [G_kn + G_kn^dag + 2 M1_k / w_n^2]
 *                                      (Sec. 3.3 eq. rho_LDA+DMFT, summed on w_n > 0 with
 *                                       G(-iw) = G(iw)^dag and the analytic 1/(iw),
 *                                       1/(iw)^2 tails added back; tail_order 0 keeps
 *                                       only the 1/2 I term)
 *   N_tot    = sum_k w_k tr N(k)                        (Sec. 3.3 eq. fix_mu)
 *   n_corr   = sum_k w_k tr(S_k N(k) S_k^dag)           (Sec. 3.4 eq. nf_LDA+DMFT)
 *   <H_KS>   = sum_k w_k sum_v E_kv N_vv(k)             (Sec. 3.5.1 eq. H_KS)
 *
 * Here S_k is the paper's overlap S^k_{alpha n} = <alpha_k|phi_nk> (Sec. 3.1
 * eq. S_norm), E_k its Kohn-Sham energies (Sec. 3.1 eq. H_LDA; n is a joint
 * band+spin index, so no spin factor appears), Sigma the local self-energy and
 * V_DC the double-counting shift (Sec. 3.2.3 eqs. V_DC, V_DC_component).
 *
 * Conventions shared by every entry point:
 *   - complex numbers are interleaved (re, im) doubles, matrices row-major;
 *     this is the byte layout of torch.complex128 / std::complex<double>;
 *   - pointers marked DEVICE are device memory on the handle's GPU, HOST are
 *     host memory; the caller owns every buffer (inputs, outputs, workspace);
 *     the library never allocates device memory inside a call;
 *   - work is enqueued on the given stream and returns before it completes
 *     (find_mu and dmft_sync_status synchronise the stream); inputs must stay
 *     alive until the stream work completes;
 *   - errors are returned as dmft_status codes; host-side argument checks
 *     run before anything is enqueued; conditions found on the device
 *     (non-finite values, a vanishing pivot) set an error word inside the
 *     workspace that dmft_sync_status and find_mu report;
 *   - one handle per host thread; calls that share a workspace must be
 *     ordered on one stream.
 *
 * Limits: 1 <= nc <= 16, nc <= nb_k <= 64, nw >= 1, beta > 0.
 */
#ifndef DMFT_H
#define DMFT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dmft_handle_s* dmft_handle;

typedef enum dmft_status {
  DMFT_OK = 0,
  DMFT_EINVAL = -1,       /* bad argument (shape, NULL, limit, tail_order)      */
  DMFT_EHIP = -2,         /* a HIP runtime call failed                          */
  DMFT_ENONFINITE = -3,   /* a non-finite value reached a pivot or a trace      */
  DMFT_ESINGULAR = -4,    /* a Gauss-Jordan pivot vanished (non-causal Sigma)   */
  DMFT_ENOCONV = -5,      /* mu search or eigensolver did not converge          */
  DMFT_EWORKSPACE = -6,   /* workspace NULL, misaligned or smaller than needed  */
  DMFT_EUNSUPPORTED = -7  /* shape outside the compiled kernel variants         */
} dmft_status;

enum { DMFT_NEWTON = 0, DMFT_BISECT = 1 };

/* Lattice side (Sec. 3.1): band window, energies and projectors of every k. */
typedef struct dmft_lattice {
  int32_t nk;          /* number of k-points                                          */
  int32_t nc;          /* correlated orbitals alpha, 1..16                            */
  int32_t nb_max;      /* largest band window, nc..64                                 */
  const int32_t* nb;   /* HOST [nk] window size nb_k; NULL: every k has nb_max bands  */
  const double* eps;   /* DEVICE E_vk: nb_k doubles per k, k after k                   */
  const double* wk;    /* DEVICE [nk] k weights (the paper's sum over k; sum to 1)    */
  const double* proj;  /* DEVICE S_k: nc x nb_k complex, row-major, k after k          */
} dmft_lattice;

/* Local self-energy on the positive Matsubara grid (Sec. 3.2.4 eq. se_pole form
 * is not required: any Sigma(i w_n) is accepted). */
typedef struct dmft_sigma {
  int32_t nw;              /* frequencies n = 0 .. nw-1                              */
  double beta;             /* inverse temperature (1/eV)                             */
  const double* sigma;     /* DEVICE [nw][nc][nc] complex Sigma(i w_n)                */
  const double* sigma_inf; /* DEVICE [nc][nc] complex Sigma(i inf), or NULL for zero; */
                           /* used only in the 1/(iw)^2 tail moment M1                 */
  const double* e_dc;      /* DEVICE [nc] real V_DC^alpha                             */
} dmft_sigma;

/* Handle: host-side plans, the autotune cache and a pinned staging buffer.
 * Selects `device` as the handle's GPU.  Returns DMFT_OK or DMFT_EHIP.
 * device = DMFT_NO_DEVICE makes a planning handle that makes no HIP call:
 * it runs every host-side argument check and answers the workspace-size
 * queries, and any call that would reach the device returns DMFT_EINVAL
 * after those checks (for sizing workspaces, or checking inputs, on a host
 * without a GPU). */
enum { DMFT_NO_DEVICE = -1 };
int dmft_create(dmft_handle* out, int device);
int dmft_destroy(dmft_handle h);

/* Static text for a status code; never NULL. */
const char* dmft_strerror(int status);
/* Detail of the last error on this handle (empty string if none); owned by h. */
const char* dmft_last_error(dmft_handle h);

/* Workspace bytes needed by gloc_compute, density_matrix, dmft_ntot,
 * density_matrix_vjp and find_mu for this shape (one size serves all). */
int dmft_workspace_size(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig,
                        size_t* bytes);

/* G_loc(i w_n) = sum_k w_k S_k G_kn S_k^dag (Sec. 3.2.2 eq. dmftloop2).
 * gloc: DEVICE [nw][nc][nc] complex, written (not accumulated). */
int gloc_compute(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu,
                 double* gloc, void* ws, size_t ws_bytes, hipStream_t stream);

/* Band density matrices N(k) (Sec. 3.3 eq. rho_LDA+DMFT) with the fused G_loc.
 *   tail_order: 2 (analytic 1/(iw) and 1/(iw)^2 tails) or 0 (1/(iw) only);
 *   nk:       DEVICE, nb_k x nb_k complex per k, k after k (Hermitian), or NULL;
 *   gloc:     DEVICE [nw][nc][nc] complex, or NULL;
 *   scalars:  DEVICE [3] = { N_tot, n_corr, <H_KS> }, or NULL.
 * At least one output must be non-NULL. */
int density_matrix(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu,
                   int tail_order, double* nk, double* gloc, double* scalars, void* ws,
                   size_t ws_bytes, hipStream_t stream);

/* DMFT self-consistency step that consumes G_loc (Sec. 3.2.2 eq. dmftloop2,
 * the impurity level of eq. H_imp):
 *   e_imp: DEVICE [nc][nc] complex, written (may be NULL):
 *          E_imp = sum_k w_k S_k diag(E_k) S_k^dag - diag(V_DC);
 *   delta: DEVICE [nw][nc][nc] complex, written:
 *          Delta(i w_n) = i w_n + mu - E_imp - Sigma(i w_n) - G_loc(i w_n)^-1;
 *   gloc:  DEVICE [nw][nc][nc] complex, read: G_loc at the same mu, as written
 *          by gloc_compute or density_matrix.
 * G_loc^-1 is a Gauss-Jordan sweep without pivoting (the anti-Hermitian part
 * of G_loc(i w_n) is negative definite for w_n > 0); a zero pivot sets
 * DMFT_ESINGULAR and non-finite output DMFT_ENONFINITE in the error word
 * (dmft_sync_status).  ws as for density_matrix. */
int dmft_hybridization(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu,
                       const double* gloc, double* delta, double* e_imp, void* ws, size_t ws_bytes,
                       hipStream_t stream);

/* Trace-only pass of the mu search (Sec. 3.3 eq. fix_mu) with its adjoint:
 * out: DEVICE [2] = { N_tot(mu), dN_tot/dmu }, where
 *   dN_tot/dmu = sum_k w_k [ (beta/4) nb_k - (2/beta) sum_n (Re tr G_kn^2 + nb_k / w_n^2) ]
 * (tail_order 2; without the tail: -(2/beta) sum_k w_k sum_n Re tr G_kn^2). */
int dmft_ntot(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu,
              int tail_order, double* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* Vector-Jacobian product of density_matrix (derivative of the Dyson and
 * Matsubara-sum steps), in PyTorch's complex convention dL/dRe + i dL/dIm for
 * the loss L = sum_k Re<nk_bar_k, N(k)> + sum_n Re<gloc_bar_n, G_loc(n)>, with
 * Sigma(i w_n), n = 0..nw-1, the independent variables and Sigma_inf held fixed:
 *   sigma_bar_n = sum_k S_k G_kn^dag C_kn G_kn^dag S_k^dag,
 *   C_kn        = (1/beta)(nk_bar_k + nk_bar_k^dag) + w_k S_k^dag gloc_bar_n S_k,
 *   mu_bar      = -sum_kn Re<C_kn, G_kn^2> + tail_order/2 * (beta/4 - (2/beta) sum_n w_n^-2)
 *                 * sum_k Re tr nk_bar_k.
 *   nk_bar:    DEVICE, N(k) layout, or NULL (zero);
 *   gloc_bar:  DEVICE [nw][nc][nc], or NULL (zero);
 *   sigma_bar: DEVICE [nw][nc][nc] complex, written;
 *   mu_bar:    DEVICE [1], written, or NULL.
 * Kernel kind 3 (see dmft_variants).  The low-rank form (the default) uses,
 * with Gl = S G S^dag, Rl = I + Gl Sigma', Rr = I + Sigma' Gl, X_j = S D^j S^dag
 * and Nt = nk_bar + nk_bar^dag,
 *   sigma_bar_n^dag = sum_k [ (1/beta) Rl S D Nt D S^dag Rr + w_k Gl gloc_bar_n^dag Gl ],
 *   S G^2 S^dag     = Rl X_2 Rr,
 *   tr(Nt G^2)      = sum_v Nt_vv d_v^2 + tr(R S (D Nt D^2 + D^2 Nt D) S^dag)
 *                     + tr(R X_2 R S D Nt D S^dag),
 * and covers band windows up to 64; the dense adjoint kernel (code 0) windows
 * up to 48 (DMFT_EUNSUPPORTED above). */
int density_matrix_vjp(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu,
                       int tail_order, const double* nk_bar, const double* gloc_bar,
                       double* sigma_bar, double* mu_bar, void* ws, size_t ws_bytes,
                       hipStream_t stream);

/* Fused scalar adjoint of N_tot in one pass (the derivative of the Dyson and
 * Matsubara-sum steps, Sec. 3.3 eqs. rho_LDA+DMFT and fix_mu):
 *   out:       DEVICE [2] = { N_tot(mu), dN_tot/dmu } (as dmft_ntot), or NULL;
 *   sigma_bar: DEVICE [nw][nc][nc] complex
 *              dN_tot/dSigma(i w_n) = (2/beta) [ sum_k w_k S_k G_kn^2 S_k^dag ]^dag
 *              in PyTorch's complex convention, or NULL.  Equal to
 *              density_matrix_vjp with nk_bar_k = w_k I and no gloc_bar.
 * Kernel kind 2 (see dmft_variants): in the low-rank form the per-(k, n)
 * quantities come from S G^2 S^dag = (I + Gl Sigma') X2 (I + Sigma' Gl) with
 * X2 = S D^2 S^dag and Gl = S G S^dag; that form covers band windows up to 64,
 * the dense adjoint kernel (code 0) windows up to 48 (DMFT_EUNSUPPORTED above). */
int dmft_ntot_vjp(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu,
                  int tail_order, double* sigma_bar, double* out, void* ws, size_t ws_bytes,
                  hipStream_t stream);

/* Chemical potential with N_tot(mu) = n_target (Sec. 3.3 eq. fix_mu).
 *   method DMFT_NEWTON: Newton steps with dN/dmu from the adjoint, kept inside
 *     the bracket [mu_lo, mu_hi] (a step leaving the bracket, or not shrinking
 *     the residual, falls back to bisection), starting at mu0;
 *   method DMFT_BISECT: plain bisection of [mu_lo, mu_hi];
 * stops when |N - n_target| <= tol_n.  Each iteration is one dmft_ntot pass and
 * one 32-byte device-to-host copy (the workspace's error word and N, dN/dmu);
 * the stream is synchronised once per iteration.
 * Outputs (HOST): mu_out, passes_out (number of dmft_ntot passes), n_out; they
 * are written on DMFT_OK and DMFT_ENOCONV.
 * Returns DMFT_ENOCONV when max_iter passes are used up, or when the bracket
 * does not contain the target: N(mu) increases with mu, so the iterates then run
 * into one end of [mu_lo, mu_hi], and the search stops as soon as no double lies
 * strictly between the current ends (about 55 passes for [-40, 40] eV).  A
 * device error of a pass returns DMFT_ESINGULAR (vanishing pivot) or
 * DMFT_ENONFINITE and clears the error word. */
int find_mu(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, int tail_order,
            double n_target, double tol_n, int method, double mu_lo, double mu_hi, double mu0,
            int max_iter, double* mu_out, int* passes_out, double* n_out, void* ws,
            size_t ws_bytes, hipStream_t stream);

/* Batched pass over several self-energy iterates with uneven band windows
 * (the per-k window of Kohn-Sham states of Sec. 2 eq. 3, within which the
 * projectors of Sec. 3.1 eq. S_norm are normalised, so nb_k varies with k;
 * each iterate is a density_matrix of its own lattice and Sigma):
 * persistent launches over cost-sorted queues of (iterate, k, frequency
 * tile) items, followed by the reductions.  Build the plan once (it uploads
 * the queue and per-k offsets into ws with a synchronous copy), then run
 * dmft_batched_pass as often as needed; it only enqueues kernels, reads each
 * iterate's mu from mu_dev (DEVICE [n_iter]) and is safe to capture in a
 * hipGraph.  Per iterate s: nk_out[s] and gloc_out[s] (DEVICE, layouts as in
 * density_matrix; either may be NULL).  lat[s]/sig[s] must stay unchanged
 * between plan and pass.  The plan times the persistent launch for the dense
 * and the low-rank form of the step (see dmft_variants) and a few k- and
 * frequency-tile sizes, and keeps the fastest; this runs the kernel several
 * times.  dmft_batched_workspace_size covers every tile the plan may take
 * (smaller k-tiles hold more G_loc partials: for 8 iterates of Nk = 4096,
 * Nw = 2048 it asks for a few tens of GB). */
int dmft_batched_workspace_size(dmft_handle h, int n_iter, const dmft_lattice* const* lat,
                                const dmft_sigma* const* sig, size_t* bytes);
int dmft_batched_plan(dmft_handle h, int n_iter, const dmft_lattice* const* lat,
                      const dmft_sigma* const* sig, int tail_order, void* ws, size_t ws_bytes,
                      hipStream_t stream);
int dmft_batched_pass(dmft_handle h, const double* mu_dev, double* const* nk_out,
                      double* const* gloc_out, void* ws, size_t ws_bytes, hipStream_t stream);
/* Capture dmft_batched_pass into a hipGraph owned by the handle (replacing any
 * previous one) and launch it on `stream`. */
int dmft_batched_graph_capture(dmft_handle h, const double* mu_dev, double* const* nk_out,
                               double* const* gloc_out, void* ws, size_t ws_bytes,
                               hipStream_t stream);
int dmft_batched_graph_launch(dmft_handle h, hipStream_t stream);

/* Form of the step used by later batched plans on this handle: DMFT_FORM_AUTO
 * (default; the plan times both), DMFT_FORM_DENSE or DMFT_FORM_LOWRANK.
 * Returns DMFT_EINVAL for another value.  dmft_batched_form returns the form
 * of the current plan (DMFT_FORM_DENSE or DMFT_FORM_LOWRANK), or -1 if there
 * is none. */
enum { DMFT_FORM_AUTO = -1, DMFT_FORM_DENSE = 0, DMFT_FORM_LOWRANK = 1 };
int dmft_batched_set_form(dmft_handle h, int form);
int dmft_batched_form(dmft_handle h);

/* Item classes of the current low-rank batched plan.  Its items are grouped
 * by padded band-window size and column count of the nc x nc inversions; each
 * class is one persistent launch.  The launches of a pass run either
 * concurrently on side streams of the handle (joined back into the pass's
 * stream, also inside a captured graph) or one after another on the pass's
 * stream, whichever the plan timed faster, in the order (by cost, or the
 * widest work-groups first) it timed faster (dmft_batched_set_concurrent(h, 1)
 * or (h, 0) fixes it for later plans instead, (h, -1) restores the timing;
 * DMFT_EINVAL for another value); dmft_batched_concurrent returns 1 for the
 * first, 0 for the second and -1 without a low-rank plan.  Writes up
 * to max entries (HOST arrays, any may be
 * NULL): nbp, ncls, items per class, and the class kernel's summed duration in
 * ms over the dmft_batched_pass calls timed since dmft_timing(h, 1, ...) (graph
 * replays are timed as a whole; reading waits for the last timed pass).
 * Returns the number of classes (0 without a low-rank plan) or a negative
 * status. */
int dmft_batched_classes(dmft_handle h, int max, int32_t* nbp, int32_t* ncls, int32_t* items, double* kernel_ms);
int dmft_batched_concurrent(dmft_handle h);
int dmft_batched_set_concurrent(dmft_handle h, int mode);

/* Tile candidates of the batched plan, in the order the plan times them: the
 * default k- and frequency tiles of every iterate, the k-tile halved, the
 * k-tile quartered, the frequency tile halved, and the k-tile quartered with
 * the frequency tile rounded down to a multiple of 48 (candidates equal to an
 * earlier one are left out of the list).  dmft_batched_set_tile_candidate(h,
 * k) makes later plans take candidate k without timing the others (for
 * reproducible profiles; an index past the plan's list, or -1, restores the
 * timing; DMFT_EINVAL below -1); dmft_batched_tile_candidate returns the
 * candidate of the current plan (-1 without a plan). */
int dmft_batched_set_tile_candidate(dmft_handle h, int index);
int dmft_batched_tile_candidate(dmft_handle h);

/* Autotuner: times every compiled kernel variant of the three kinds (density
 * pass, trace pass, fused scalar adjoint) that fits this shape on the
 * handle's GPU, with a few frequency-tile sizes, after checking that each one
 * reproduces the reference variant to 1e-11, and caches the fastest in the
 * handle (used by all later calls of that shape).  best_out (HOST, may be
 * NULL) receives a short description. */
int dmft_autotune(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu,
                  void* ws, size_t ws_bytes, hipStream_t stream, char* best_out, size_t best_len);

/* Kernel variants.  kind 0 = density pass (density_matrix, gloc_compute),
 * kind 1 = trace pass (dmft_ntot, find_mu), kind 2 = fused scalar adjoint
 * (dmft_ntot_vjp), kind 3 = general vector-Jacobian product
 * (density_matrix_vjp; not autotuned); code 0 of kinds 2 and 3 is the dense
 * adjoint kernel; nbp = padded band-window size
 * (16, 32, 48 or 64).  dmft_variants writes up to max variant codes into out
 * (HOST) and returns their number (the first is the default); dmft_set_variant
 * pins one for later calls on this handle (var = -1 restores the default) and
 * returns DMFT_EINVAL for a code that is not instantiated; dmft_get_variant
 * returns the code later calls of that kind and size will use (the pinned or
 * autotuned one, else the default), or -1 for a size with no kernel.
 *
 * Codes with bit 3 (8) set select the low-rank form of the same step: with
 * D = diag(1 / (i w_n + mu - E_v)) and X = P D P^dag (nc x nc), the Woodbury
 * identity gives P G P^dag = (X^-1 - Sigma')^-1 and G = D + D P^dag R P D,
 * R = Sigma' (X^-1 - Sigma')^-1 X^-1, so only nc x nc matrices are inverted.
 * It gives the same outputs to rounding and needs only that P(k) has full row
 * rank (its nc x nc inversions run without pivoting: the anti-Hermitian part
 * of X is P Im(D) P^dag, negative definite for w_n > 0); other bits of a code
 * tune registers and occupancy only.  Code 40 (bits 3 and 5, 64-band windows,
 * density kind) runs the low-rank step on two-wavefront work-groups that
 * share the nc x nc part of the step. */
int dmft_variants(int kind, int nbp, int* out, int max);
int dmft_set_variant(dmft_handle h, int kind, int nbp, int var);
int dmft_get_variant(dmft_handle h, int kind, int nbp);

/* Kernel timing (for roofline reports).  enable = 1 clears the counters and
 * starts recording a pair of hipEvents around every launch of the Dyson kernel
 * (on the stream it is launched on); enable = 0 stops recording.  A batched
 * pass counts as one launch: its events bracket all class kernels of the pass
 * (from before the fork to after the join); a graph replay is bracketed by a
 * pair around hipGraphLaunch on the launch stream, which also covers the
 * pass's epilogue reductions (dmft_batched_graph_launch reads the previous
 * replay's events before launching the next).  Every call first
 * waits for the events recorded so far and returns, in HOST memory, the
 * summed kernel time in ms and the number of timed launches (either pointer
 * may be NULL).  Timing adds two event records per launch. */
int dmft_timing(dmft_handle h, int enable, double* kernel_ms, int64_t* launches);

/* Synchronise `stream` and report the error word kept in ws (then clear it). */
int dmft_sync_status(dmft_handle h, void* ws, hipStream_t stream);

/* density_matrix without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid allocation): the call makes no allocating runtime call
 * (no device, pinned or event allocation) and runs on the library's own scratch
 * array, 64 MiB per GPU, held from library load until the process ends.
 * Arguments and outputs are those of density_matrix, except:
 *   - band windows must be uniform (lat->nb NULL, or every entry nb_max),
 *     DMFT_EINVAL otherwise;
 *   - tiles are coarsened until the pass fits the scratch; a shape whose
 *     smallest layout needs more returns DMFT_EWORKSPACE before any launch;
 *   - status: DEVICE int32 [1] or NULL, written on the stream with DMFT_OK,
 *     DMFT_ESINGULAR or DMFT_ENONFINITE for this call (the scratch's error
 *     word is cleared at the start of every call).
 * All calls on one GPU share its scratch array: calls that overlap on one GPU
 * (two streams, two threads) race and must be ordered by the caller. */
int density_matrix_noalloc(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu,
                           int tail_order, double* nk, double* gloc, double* scalars, int32_t* status,
                           hipStream_t stream);


/* ------------------------------------------------------------------------
 * Pole-expansion route (Sec. 3.3 eqs. pseudo_H_k, rho_LDA+DMFT_componet_final
 * and fix_mu; Sec. 3.5.2 eqs. DOS and PDOS).  For a self-energy in the pole
 * form of Sec. 3.2.4 eq. se_pole,
 *   Sigma(i w) = Sigma_inf + sum_i V_i^dag V_i / (i w - p_i)   (V_i a row over alpha),
 * the band-window resolvent is the physical block of (i w - H_ps(k))^-1 with
 *   H_ps(k) = [[ diag(E_k) + P^dag (Sigma_inf - diag(V_DC)) P,  -(V P)^dag ],
 *              [ -(V P),                                       diag(p)    ]]
 * (m_k = nb_k + np rows).  With H_ps = Psi diag(E^ps) Psi^dag and u_l the first
 * nb_k entries of column l of Psi (<phi_n|psi_l>):
 *   N(k) = sum_l u_l u_l^dag n_F(E^ps_l - mu),  N_tot = sum_k w_k sum_l |u_l|^2 n_F(E^ps_l - mu).
 * The eigensystems do not depend on mu: one dmft_pole_eig serves every later
 * density, mu search and DOS at any mu.  Limit: nb_max + np <= 80.
 *
 * Per-k outputs use the padded stride mp = nb_max + np; for k with m_k < mp the
 * entries m_k .. mp-1 are zero (eigenvalue 0 with weight 0, zero vectors).
 * All calls are stream-ordered; the workspace layout is shared by all of them
 * (size from dmft_pole_workspace_size with the largest DOS grid used). */
typedef struct dmft_poles {
  int32_t np;              /* number of poles, 0 .. 80 - nb_max                    */
  double beta;             /* inverse temperature (1/eV)                           */
  const double* p;         /* DEVICE [np] real pole positions p_i                  */
  const double* v;         /* DEVICE [np][nc] complex pole vectors V_i             */
  const double* sigma_inf; /* DEVICE [nc][nc] complex Sigma(inf), or NULL for zero */
  const double* e_dc;      /* DEVICE [nc] real V_DC^alpha                          */
} dmft_poles;

/* Workspace bytes for the pole-route calls, with DOS grids up to ne_max points. */
int dmft_pole_workspace_size(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, int ne_max,
                             size_t* bytes);

/* Eigensystems of H_ps(k) for every k (batched Jacobi, one work-group per k).
 *   evals: DEVICE [nk][mp] real, ascending per k (ties by index);
 *   evecs: DEVICE [nk][nb_max][mp] complex, row n = band, column l = eigenvector
 *          (the physical part u_l; the pole components are not returned);
 *   wphys: DEVICE [nk][mp] = |u_l|^2;
 *   worb:  DEVICE [nk][mp][nc] = |P_alpha u_l|^2 (for the PDOS), or NULL.
 * A k whose iteration does not converge within 30 sweeps raises DMFT_ENOCONV,
 * non-finite input DMFT_ENONFINITE, in the error word (dmft_sync_status). */
int dmft_pole_eig(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, double* evals, double* evecs,
                  double* wphys, double* worb, void* ws, size_t ws_bytes, hipStream_t stream);

/* Jacobi sweeps each k took in the last dmft_pole_eig on ws (HOST [nk]); synchronises. */
int dmft_pole_sweeps(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, const void* ws, int32_t* out,
                     hipStream_t stream);

/* N(k) = sum_l u_l u_l^dag f(E^ps_l - mu) from dmft_pole_eig's output, with
 * f = n_F (nw_trunc = 0, the paper's exact sum) or, for nw_trunc > 0, the
 * weight the positive-frequency Matsubara sum truncated at nw_trunc
 * frequencies with the analytic 1/(iw) and 1/(iw)^2 tails gives one level,
 *   f(x) = 1/2 - beta x / 4 + (2/beta) sum_{n<nw_trunc} x^3 / (w_n^2 (w_n^2 + x^2)),
 * which makes the result equal density_matrix's N(k) at nw = nw_trunc.
 *   nk:      DEVICE, N(k) layout of density_matrix, or NULL;
 *   scalars: DEVICE [3] = { N_tot, n_corr, <H_KS> } as in density_matrix, or NULL. */
int dmft_pole_density(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, double mu, int nw_trunc,
                      const double* evals, const double* evecs, double* nk, double* scalars, void* ws,
                      size_t ws_bytes, hipStream_t stream);

/* mu with N_tot(mu) = n_target (Sec. 3.3 eq. fix_mu) from the eigenvalues and
 * weights alone: the whole search runs in one work-group on the device
 * (safeguarded Newton with dN/dmu = sum_k w_k sum_l |u_l|^2 beta n_F (1 - n_F),
 * or bisection), starting at the middle of [mu_lo, mu_hi]; N(mu) is increasing.
 * Stops at |N - n_target| <= tol_n; DMFT_ENOCONV after max_iter evaluations.
 * mu_out, passes_out (evaluations of N) and n_out are HOST; synchronises. */
int dmft_pole_find_mu(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, const double* evals,
                      const double* wphys, double n_target, double tol_n, int method, double mu_lo, double mu_hi,
                      int max_iter, double* mu_out, int* passes_out, double* n_out, void* ws, size_t ws_bytes,
                      hipStream_t stream);

/* DOS and PDOS on ne energies e_i = e_min + i (e_max - e_min) / (ne - 1)
 * (Sec. 3.5.2 eqs. DOS and PDOS, k-sum with the weights w_k), with the
 * Lorentzian of half-width eta > 0 for the eta -> 0+ limit:
 *   D(e)   = sum_k w_k sum_l |u_l|^2 (eta/pi) / ((e + mu - E^ps_l)^2 + eta^2),
 *   D_a(e) = the same with |P_alpha u_l|^2.
 *   dos:  DEVICE [ne];  pdos: DEVICE [ne][nc] or NULL (needs worb). */
int dmft_pole_dos(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, const double* evals,
                  const double* wphys, const double* worb, double mu, double eta, double e_min, double e_max, int ne,
                  double* dos, double* pdos, void* ws, size_t ws_bytes, hipStream_t stream);


/* Energy-functional sums of the pole route (Sec. 3.5.1 eqs. H_KS, H_U_energy,
 * <V_DC>) from dmft_pole_eig's output (worb required):
 *   out: DEVICE [5 + nc] = { B, N_tot, <H_KS>, <V_DC>, <H_U>, n_alpha (nc) } with
 *   B       = sum_k w_k sum_l E^ps_l |u_l|^2 n_F(E^ps_l - mu),
 *   <H_KS>  = sum_k w_k sum_n E_n N(k)_nn,
 *   n_alpha = sum_k w_k sum_l |P_alpha u_l|^2 n_F(E^ps_l - mu),
 *   <V_DC>  = sum_alpha V_DC^alpha n_alpha,
 *   <H_U>   = (B - <H_KS> + <V_DC>) / 2 = (1/2) tr[Sigma G] (Galitskii-Migdal).
 * With E^ps absolute this <H_U> is the printed eq. H_U_energy plus mu N_tot;
 * the double-counting energy of eq. E_DC follows from n_alpha per site. */
int dmft_pole_energy(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, double mu, const double* evals,
                     const double* evecs, const double* wphys, const double* worb, double* out, void* ws,
                     size_t ws_bytes, hipStream_t stream);

/* Hubbard-I atoms (Sec. 3.2.4 eqs. Dyson and G_imp_atom; appendix eq.
 * dyson_pole), batched: atom i has nc spin-orbitals with levels eps[i][a]
 * (the diagonal of E_imp), interaction H_U = (U_i/2) sum_{a != b} n_a n_b
 * (eq. H_U at J = 0) and chemical potential mu[i]; all Fock states are
 * enumerated (2^nc, nc <= 16).  Its Green's function is diagonal with poles
 * e_a - mu + U N weighted by Boltzmann factors; the self-energy
 *   Sigma_aa(i w) = sigma_inf[i][a] + sum_j wgt[i][a][j] / (i w + mu - pos[i][a][j])
 * has npoles[i][a] <= nc - 1 poles, placed by bisection between adjacent
 * Green's-function poles, with positions on the absolute energy axis (as
 * dmft_poles takes them).  G poles of weight <= wtol are dropped and the rest
 * renormalised (1e-13 is a good value; 0 keeps every nonzero weight).
 *   eps: DEVICE [natoms][nc]; U, mu: DEVICE [natoms];
 *   sigma_inf: DEVICE [natoms][nc]; npoles: DEVICE int32 [natoms][nc];
 *   pos, wgt: DEVICE [natoms][nc][nc] (entries past npoles are zero);
 *   occ: DEVICE [natoms][nc] thermal <n_a>, or NULL; e_u: DEVICE [natoms] <H_U>, or NULL.
 * No workspace.  The pole vectors of dmft_poles are V = sqrt(wgt) e_a. */
int dmft_hubbard1(dmft_handle h, int natoms, int nc, const double* eps, const double* U, const double* mu,
                  double beta, double wtol, double* sigma_inf, int32_t* npoles, double* pos, double* wgt, double* occ,
                  double* e_u, hipStream_t stream);

/* Matsubara-axis self-energy of a pole form (Sec. 3.2.4 eq. se_pole) at chemical
 * potential mu, for the frequency-sum route:
 *   sigma[n] = Sigma_inf + sum_i V_i^dag V_i / (i w_n + mu - p_i),  w_n = (2n+1) pi / beta,
 * sigma: DEVICE [nw][nc][nc] complex.  pol->e_dc is not used. */
int dmft_sigma_from_poles(dmft_handle h, int nc, const dmft_poles* pol, int nw, double mu, double* sigma,
                          hipStream_t stream);


/* One atom's dmft_hubbard1 output (npoles [nc], pos and wgt [nc][nc], DEVICE)
 * as a dmft_poles pole list: pole j of orbital a becomes p = pos[a][j] with
 * V = sqrt(wgt[a][j]) e_{a0 + a} among nc_lat correlated orbitals, packed
 * orbital after orbital.  p: DEVICE [nc (nc - 1)], v: DEVICE [nc (nc - 1)][nc_lat]
 * complex, np_out: DEVICE int32 [1] = number of poles written. */
int dmft_hubbard1_poles(dmft_handle h, int nc, int nc_lat, int a0, const int32_t* npoles, const double* pos,
                        const double* wgt, double* p, double* v, int32_t* np_out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* DMFT_H */
