/*
 * Plain FP64 CPU oracle for the lattice Dyson step of charge-self-consistent
 * LDA+DMFT (Zhao et al., "Implementation of LDA+DMFT with pseudo-potential-
 * plane-wave method").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU path is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the product
 * library never links, calls or includes anything from here, and this file
 * includes nothing from the product.
 *
 * What it computes, in the paper's notation (all energies in eV):
 *   z_n      = i w_n + mu,  w_n = (2n+1) pi / beta,  n = 0 .. nw-1
 *   A_kn     = z_n I - diag(E_k) - S_k^dag (Sigma(i w_n) - diag(V_DC)) S_k
 *              (lattice Dyson equation, Sec. 3.2.2 eq. dmftloop1, written in
 *               the Bloch band window with the embedding f = S c of
 *               Sec. 3.2 eq. f_operation and the sign of V_DC from
 *               Sec. 3.3 eq. rho_LDA+DMFT)
 *   G_kn     = A_kn^{-1}
 *   G_loc(n) = sum_k w_k S_k G_kn S_k^dag      (Sec. 3.2.2 eq. dmftloop2)
 *   M1_k     = diag(E_k) - mu I + S_k^dag (Sigma_inf - diag(V_DC)) S_k
 *   N(k)     = 1/2 I - (beta/4) M1_k
 *              + (1/beta) sum_{n=0}^{nw-1} [G_kn + G_kn^dag + 2 M1_k / w_n^2]
 *              (the Matsubara sum of Sec. 3.3 eq. rho_LDA+DMFT, folded onto
 *               positive frequencies with G(-iw) = G(iw)^dag, with the
 *               e^{iw0+} convergence factor and the analytic sums of the
 *               1/(iw) and 1/(iw)^2 tails added back; tail_order = 0 keeps
 *               only the 1/2 I term)
 *   N_tot    = sum_k w_k tr N(k)                 (Sec. 3.3 eq. fix_mu)
 *   n_corr   = sum_k w_k tr(S_k N(k) S_k^dag)    (Sec. 3.4 eq. nf_LDA+DMFT)
 *   <H_KS>   = sum_k w_k sum_v E_kv N_vv(k)      (Sec. 3.5.1 eq. H_KS)
 *
 * Derivatives (PyTorch complex convention dL/dRe + i dL/dIm, positive-frequency
 * Sigma(i w_n) independent, Sigma_inf fixed) follow from dG = -G dA G:
 *   dN_tot/dmu     = sum_k w_k [ (beta/4) nb_k
 *                     - (2/beta) sum_n ( Re tr G_kn^2 + nb_k / w_n^2 ) ]
 *   dN_tot/dSigma_n = (2/beta) [ sum_k w_k S_k G_kn^2 S_k^dag ]^dag
 *   general VJP with upstream Nbar_k, Gbar_n:
 *     Sigmabar_n = sum_k S_k G^dag C G^dag S_k^dag,
 *     C = (1/beta)(Nbar_k + Nbar_k^dag) + w_k S_k^dag Gbar_n S_k
 *
 * The inverse is Gaussian elimination with partial pivoting, written out here
 * with a hand-rolled complex multiply-add; no BLAS or LAPACK is used.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cplx;

static inline cplx c_make(double re, double im) { cplx z; z.re = re; z.im = im; return z; }
static inline cplx c_add(cplx a, cplx b) { return c_make(a.re + b.re, a.im + b.im); }
static inline cplx c_sub(cplx a, cplx b) { return c_make(a.re - b.re, a.im - b.im); }
static inline cplx c_mul(cplx a, cplx b) {
  return c_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
static inline cplx c_conj(cplx a) { return c_make(a.re, -a.im); }
/* acc + a*b */
static inline cplx c_mac(cplx acc, cplx a, cplx b) {
  acc.re += a.re * b.re - a.im * b.im;
  acc.im += a.re * b.im + a.im * b.re;
  return acc;
}
static inline double c_abs2(cplx a) { return a.re * a.re + a.im * a.im; }
static inline cplx c_div(cplx a, cplx b) {
  double d = c_abs2(b);
  return c_make((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}

/* ---- problem description (host arrays, interleaved complex) ---------------- */
typedef struct {
  int nk, nc;
  const int* nb;         /* [nk] band-window size per k (Sec. 2, eq. 3 window) */
  const int64_t* off_b;  /* [nk+1] offset of k's bands into eps */
  const int64_t* off_p;  /* [nk+1] offset (complex elements) of S_k into proj */
  const double* eps;     /* E_{vk}                                            */
  const double* wk;      /* [nk] k weights                                    */
  const double* proj;    /* S_k: nc x nb_k complex, row-major                 */
} orc_lattice;

typedef struct {
  int nw;
  double beta;
  const double* sigma;     /* [nw][nc][nc] complex, Sigma(i w_n), n >= 0   */
  const double* sigma_inf; /* [nc][nc] complex or NULL (= 0)               */
  const double* e_dc;      /* [nc] V_DC^alpha                               */
} orc_sigma;

static double omega_n(int n, double beta) { return (double)(2 * n + 1) * M_PI / beta; }

/* ---- dense complex helpers --------------------------------------------------- */

/* Inverse of the n x n matrix a (row-major, destroyed) into g, by Gaussian
 * elimination with partial pivoting on [a | I].  Returns 0, or -1 when a pivot
 * is exactly zero. */
static int invert(int n, cplx* a, cplx* g) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) g[i * n + j] = c_make(i == j ? 1.0 : 0.0, 0.0);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    double best = c_abs2(a[col * n + col]);
    for (int r = col + 1; r < n; ++r) {
      double v = c_abs2(a[r * n + col]);
      if (v > best) { best = v; piv = r; }
    }
    if (best == 0.0) return -1;
    if (piv != col) {
      for (int j = 0; j < n; ++j) {
        cplx t = a[col * n + j]; a[col * n + j] = a[piv * n + j]; a[piv * n + j] = t;
        t = g[col * n + j]; g[col * n + j] = g[piv * n + j]; g[piv * n + j] = t;
      }
    }
    cplx p = a[col * n + col];
    for (int r = col + 1; r < n; ++r) {
      cplx f = c_div(a[r * n + col], p);
      if (f.re == 0.0 && f.im == 0.0) continue;
      for (int j = col; j < n; ++j) a[r * n + j] = c_sub(a[r * n + j], c_mul(f, a[col * n + j]));
      for (int j = 0; j < n; ++j) g[r * n + j] = c_sub(g[r * n + j], c_mul(f, g[col * n + j]));
    }
  }
  /* back substitution, one right-hand side column at a time */
  for (int j = 0; j < n; ++j) {
    for (int r = n - 1; r >= 0; --r) {
      cplx s = g[r * n + j];
      for (int c = r + 1; c < n; ++c) s = c_sub(s, c_mul(a[r * n + c], g[c * n + j]));
      g[r * n + j] = c_div(s, a[r * n + r]);
    }
  }
  return 0;
}

/* E = S^dag M S for S (nc x nb), M (nc x nc): result nb x nb */
static void embed(int nc, int nb, const cplx* s, const cplx* m, cplx* out) {
  for (int v = 0; v < nb; ++v)
    for (int w = 0; w < nb; ++w) {
      cplx acc = c_make(0, 0);
      for (int a = 0; a < nc; ++a) {
        cplx t = c_make(0, 0);
        for (int b = 0; b < nc; ++b) t = c_mac(t, m[a * nc + b], s[b * nb + w]);
        acc = c_mac(acc, c_conj(s[a * nb + v]), t);
      }
      out[v * nb + w] = acc;
    }
}

/* X = S M S^dag for S (nc x nb), M (nb x nb): result nc x nc */
static void project(int nc, int nb, const cplx* s, const cplx* m, cplx* out) {
  for (int a = 0; a < nc; ++a)
    for (int b = 0; b < nc; ++b) {
      cplx acc = c_make(0, 0);
      for (int v = 0; v < nb; ++v) {
        cplx t = c_make(0, 0);
        for (int w = 0; w < nb; ++w) t = c_mac(t, m[v * nb + w], c_conj(s[b * nb + w]));
        acc = c_mac(acc, s[a * nb + v], t);
      }
      out[a * nc + b] = acc;
    }
}

static void matmul(int n, const cplx* x, const cplx* y, cplx* out) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cplx acc = c_make(0, 0);
      for (int l = 0; l < n; ++l) acc = c_mac(acc, x[i * n + l], y[l * n + j]);
      out[i * n + j] = acc;
    }
}

static void dagger(int n, const cplx* x, cplx* out) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[j * n + i] = c_conj(x[i * n + j]);
}

/* Sigma(i w_n) - diag(V_DC) into m (nc x nc) */
static void sigma_shifted(const orc_sigma* sg, int nc, int n, cplx* m) {
  const cplx* s = (const cplx*)sg->sigma + (size_t)n * nc * nc;
  for (int a = 0; a < nc * nc; ++a) m[a] = s[a];
  for (int a = 0; a < nc; ++a) m[a * nc + a].re -= sg->e_dc[a];
}

/* A_kn of eq. dmftloop1 in the band window of k */
static void build_a(const orc_lattice* lat, const orc_sigma* sg, int k, int n, double mu,
                    cplx* a, cplx* sig, cplx* work) {
  int nc = lat->nc, nb = lat->nb[k];
  const double* e = lat->eps + lat->off_b[k];
  const cplx* s = (const cplx*)lat->proj + lat->off_p[k];
  sigma_shifted(sg, nc, n, sig);
  embed(nc, nb, s, sig, work);
  double w = omega_n(n, sg->beta);
  for (int v = 0; v < nb; ++v)
    for (int u = 0; u < nb; ++u) {
      cplx d = c_make(0, 0);
      if (u == v) d = c_make(mu - e[v], w);
      a[v * nb + u] = c_sub(d, work[v * nb + u]);
    }
}

/* M1_k = diag(E_k) - mu + S^dag (Sigma_inf - V_DC) S */
static void first_moment(const orc_lattice* lat, const orc_sigma* sg, int k, double mu,
                         cplx* m1, cplx* sig) {
  int nc = lat->nc, nb = lat->nb[k];
  const double* e = lat->eps + lat->off_b[k];
  const cplx* s = (const cplx*)lat->proj + lat->off_p[k];
  const cplx* si = (const cplx*)sg->sigma_inf;
  for (int a = 0; a < nc * nc; ++a) sig[a] = si ? si[a] : c_make(0, 0);
  for (int a = 0; a < nc; ++a) sig[a * nc + a].re -= sg->e_dc[a];
  embed(nc, nb, s, sig, m1);
  for (int v = 0; v < nb; ++v) m1[v * nb + v].re += e[v] - mu;
}

static int max_nb(const orc_lattice* lat) {
  int m = 0;
  for (int k = 0; k < lat->nk; ++k) if (lat->nb[k] > m) m = lat->nb[k];
  return m;
}

typedef struct { cplx *a, *g, *t, *u, *sig; } scratch;
static int scratch_alloc(scratch* s, int nb, int nc) {
  size_t n2 = (size_t)nb * nb;
  s->a = (cplx*)malloc(sizeof(cplx) * n2);
  s->g = (cplx*)malloc(sizeof(cplx) * n2);
  s->t = (cplx*)malloc(sizeof(cplx) * n2);
  s->u = (cplx*)malloc(sizeof(cplx) * n2);
  s->sig = (cplx*)malloc(sizeof(cplx) * (size_t)nc * nc);
  return (s->a && s->g && s->t && s->u && s->sig) ? 0 : -1;
}
static void scratch_free(scratch* s) { free(s->a); free(s->g); free(s->t); free(s->u); free(s->sig); }

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

/* ---- public entry points ------------------------------------------------------- */

/* N(k) for each k in klist (count nsel), written densely nb_k x nb_k complex,
 * one after another in klist order, to nk_out; also tr N(k) into ntr[sel]. */
int orc_density(const orc_lattice* lat, const orc_sigma* sg, double mu, int tail_order,
                const int* klist, int nsel, double* nk_out, double* ntr, int nthreads) {
  int nc = lat->nc, nbm = max_nb(lat), err = 0;
  int64_t* outoff = (int64_t*)malloc(sizeof(int64_t) * (nsel + 1));
  outoff[0] = 0;
  for (int i = 0; i < nsel; ++i) outoff[i + 1] = outoff[i] + (int64_t)lat->nb[klist[i]] * lat->nb[klist[i]];
  double s2 = 0.0; /* sum_n 1/w_n^2, summed in increasing n */
  for (int n = 0; n < sg->nw; ++n) { double w = omega_n(n, sg->beta); s2 += 1.0 / (w * w); }
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int i = 0; i < nsel; ++i) {
    scratch sc;
    if (scratch_alloc(&sc, nbm, nc)) { err |= 1; continue; }
    int k = klist[i], nb = lat->nb[k];
    cplx* acc = (cplx*)calloc((size_t)nb * nb, sizeof(cplx));
    for (int n = 0; n < sg->nw; ++n) {
      build_a(lat, sg, k, n, mu, sc.a, sc.sig, sc.t);
      if (invert(nb, sc.a, sc.g)) { err |= 2; break; }
      for (int v = 0; v < nb; ++v)
        for (int u = 0; u < nb; ++u)
          acc[v * nb + u] = c_add(acc[v * nb + u], c_add(sc.g[v * nb + u], c_conj(sc.g[u * nb + v])));
    }
    cplx* out = (cplx*)nk_out + outoff[i];
    double beta = sg->beta;
    if (tail_order == 2) first_moment(lat, sg, k, mu, sc.u, sc.sig);
    double tr = 0.0;
    for (int v = 0; v < nb; ++v)
      for (int u = 0; u < nb; ++u) {
        cplx x = c_make(acc[v * nb + u].re / beta, acc[v * nb + u].im / beta);
        if (u == v) x.re += 0.5;
        if (tail_order == 2) {
          cplx m = sc.u[v * nb + u];
          x.re += -0.25 * beta * m.re + 2.0 * s2 * m.re / beta;
          x.im += -0.25 * beta * m.im + 2.0 * s2 * m.im / beta;
        }
        out[v * nb + u] = x;
        if (u == v) tr += x.re;
      }
    if (ntr) ntr[i] = tr;
    free(acc);
    scratch_free(&sc);
  }
  free(outoff);
  return err ? -1 : 0;
}

/* G_loc(i w_n) for each n in nlist (count nsel), nc x nc complex each. */
int orc_gloc(const orc_lattice* lat, const orc_sigma* sg, double mu, const int* nlist, int nsel,
             double* gloc_out, int nthreads) {
  int nc = lat->nc, nbm = max_nb(lat), err = 0;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int i = 0; i < nsel; ++i) {
    scratch sc;
    if (scratch_alloc(&sc, nbm, nc)) { err |= 1; continue; }
    int n = nlist[i];
    cplx* out = (cplx*)gloc_out + (size_t)i * nc * nc;
    cplx* x = (cplx*)malloc(sizeof(cplx) * nc * nc);
    for (int a = 0; a < nc * nc; ++a) out[a] = c_make(0, 0);
    for (int k = 0; k < lat->nk; ++k) {
      int nb = lat->nb[k];
      const cplx* s = (const cplx*)lat->proj + lat->off_p[k];
      build_a(lat, sg, k, n, mu, sc.a, sc.sig, sc.t);
      if (invert(nb, sc.a, sc.g)) { err |= 2; break; }
      project(nc, nb, s, sc.g, x);
      for (int a = 0; a < nc * nc; ++a) {
        out[a].re += lat->wk[k] * x[a].re;
        out[a].im += lat->wk[k] * x[a].im;
      }
    }
    free(x);
    scratch_free(&sc);
  }
  return err ? -1 : 0;
}

/* N_tot(mu) and dN_tot/dmu over all k (the trace-only pass of the mu search). */
int orc_trace(const orc_lattice* lat, const orc_sigma* sg, double mu, int tail_order,
              double* n_out, double* dndmu_out, int nthreads) {
  int nc = lat->nc, nbm = max_nb(lat), nk = lat->nk, err = 0;
  double* nk_tr = (double*)calloc(nk, sizeof(double));
  double* nk_d = (double*)calloc(nk, sizeof(double));
  double s2 = 0.0;
  for (int n = 0; n < sg->nw; ++n) { double w = omega_n(n, sg->beta); s2 += 1.0 / (w * w); }
  double beta = sg->beta;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int k = 0; k < nk; ++k) {
    scratch sc;
    if (scratch_alloc(&sc, nbm, nc)) { err |= 1; continue; }
    int nb = lat->nb[k];
    double trg = 0.0, trg2 = 0.0;
    for (int n = 0; n < sg->nw; ++n) {
      build_a(lat, sg, k, n, mu, sc.a, sc.sig, sc.t);
      if (invert(nb, sc.a, sc.g)) { err |= 2; break; }
      for (int v = 0; v < nb; ++v) trg += sc.g[v * nb + v].re;
      for (int v = 0; v < nb; ++v)
        for (int u = 0; u < nb; ++u) trg2 += c_mul(sc.g[v * nb + u], sc.g[u * nb + v]).re;
    }
    double tr = 0.5 * nb + 2.0 * trg / beta;
    double d = -2.0 * trg2 / beta;
    if (tail_order == 2) {
      first_moment(lat, sg, k, mu, sc.u, sc.sig);
      double trm = 0.0;
      for (int v = 0; v < nb; ++v) trm += sc.u[v * nb + v].re;
      tr += -0.25 * beta * trm + 2.0 * s2 * trm / beta;
      d += 0.25 * beta * nb - 2.0 * s2 * nb / beta;
    }
    nk_tr[k] = tr;
    nk_d[k] = d;
    scratch_free(&sc);
  }
  double ntot = 0.0, dn = 0.0;
  for (int k = 0; k < nk; ++k) { ntot += lat->wk[k] * nk_tr[k]; dn += lat->wk[k] * nk_d[k]; }
  free(nk_tr);
  free(nk_d);
  if (n_out) *n_out = ntot;
  if (dndmu_out) *dndmu_out = dn;
  return err ? -1 : 0;
}

/* General vector-Jacobian product.  nbar: upstream of N(k), ragged like the
 * N(k) layout of all k in order (NULL = 0); gbar: [nw][nc][nc] upstream of
 * G_loc (NULL = 0).  Writes sigma_bar [nw][nc][nc] and mu_bar [1]. */
int orc_vjp(const orc_lattice* lat, const orc_sigma* sg, double mu, int tail_order,
            const double* nbar, const double* gbar, double* sigma_bar, double* mu_bar,
            int nthreads) {
  int nc = lat->nc, nbm = max_nb(lat), nk = lat->nk, nw = sg->nw, err = 0;
  double beta = sg->beta;
  int64_t* off_n = (int64_t*)malloc(sizeof(int64_t) * (nk + 1));
  off_n[0] = 0;
  for (int k = 0; k < nk; ++k) off_n[k + 1] = off_n[k] + (int64_t)lat->nb[k] * lat->nb[k];
  double s2 = 0.0;
  for (int n = 0; n < nw; ++n) { double w = omega_n(n, beta); s2 += 1.0 / (w * w); }
  double* mu_n = (double*)calloc(nw, sizeof(double));
  set_threads(nthreads);
  /* one frequency per task: the k sum for sigma_bar(n) runs in fixed order */
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int n = 0; n < nw; ++n) {
    scratch sc;
    if (scratch_alloc(&sc, nbm, nc)) { err |= 1; continue; }
    cplx* c = (cplx*)malloc(sizeof(cplx) * nbm * nbm);
    cplx* gd = (cplx*)malloc(sizeof(cplx) * nbm * nbm);
    cplx* y = (cplx*)malloc(sizeof(cplx) * nbm * nbm);
    cplx* x = (cplx*)malloc(sizeof(cplx) * nc * nc);
    cplx* out = (cplx*)sigma_bar + (size_t)n * nc * nc;
    for (int a = 0; a < nc * nc; ++a) out[a] = c_make(0, 0);
    double mub = 0.0;
    for (int k = 0; k < nk; ++k) {
      int nb = lat->nb[k];
      const cplx* s = (const cplx*)lat->proj + lat->off_p[k];
      double w = lat->wk[k];
      build_a(lat, sg, k, n, mu, sc.a, sc.sig, sc.t);
      if (invert(nb, sc.a, sc.g)) { err |= 2; break; }
      /* C = (1/beta)(Nbar + Nbar^dag) + w S^dag Gbar S */
      for (int v = 0; v < nb * nb; ++v) c[v] = c_make(0, 0);
      if (nbar) {
        const cplx* nb_k = (const cplx*)nbar + off_n[k];
        for (int v = 0; v < nb; ++v)
          for (int u = 0; u < nb; ++u) {
            cplx t = c_add(nb_k[v * nb + u], c_conj(nb_k[u * nb + v]));
            c[v * nb + u] = c_make(t.re / beta, t.im / beta);
          }
      }
      if (gbar) {
        const cplx* gb = (const cplx*)gbar + (size_t)n * nc * nc;
        embed(nc, nb, s, gb, sc.t);
        for (int v = 0; v < nb * nb; ++v) {
          c[v].re += w * sc.t[v].re;
          c[v].im += w * sc.t[v].im;
        }
      }
      /* Sigma_bar += S G^dag C G^dag S^dag */
      dagger(nb, sc.g, gd);
      matmul(nb, gd, c, sc.t);
      matmul(nb, sc.t, gd, y);
      project(nc, nb, s, y, x);
      for (int a = 0; a < nc * nc; ++a) out[a] = c_add(out[a], x[a]);
      /* mu_bar += Re<C, dG/dmu + dG^dag/dmu> / 2-part: with dG/dmu = -G^2,
       * d/dmu of (1/beta)(G + G^dag) paired with Nbar, and w S G S^dag paired
       * with Gbar, collapses to -Re tr(C^dag G^2). */
      matmul(nb, sc.g, sc.g, sc.t);
      double acc = 0.0;
      for (int v = 0; v < nb; ++v)
        for (int u = 0; u < nb; ++u) {
          cplx cv = c[v * nb + u];
          cplx g2 = sc.t[v * nb + u];
          acc += cv.re * g2.re + cv.im * g2.im; /* Re(conj(C_vu) G2_vu) */
        }
      mub -= acc;
    }
    mu_n[n] = mub;
    free(c); free(gd); free(y); free(x);
    scratch_free(&sc);
  }
  /* tail terms: d/dmu of -(beta/4) M1 + (2/beta) s2 M1 with dM1/dmu = -I, paired with Nbar */
  double mt = 0.0;
  if (tail_order == 2 && nbar) {
    for (int k = 0; k < nk; ++k) {
      int nb = lat->nb[k];
      const cplx* nb_k = (const cplx*)nbar + off_n[k];
      double tr = 0.0;
      for (int v = 0; v < nb; ++v) tr += nb_k[v * nb + v].re;
      mt += (0.25 * beta - 2.0 * s2 / beta) * tr;
    }
  }
  double total = mt;
  for (int n = 0; n < nw; ++n) total += mu_n[n];
  if (mu_bar) *mu_bar = total;
  free(mu_n);
  free(off_n);
  return err ? -1 : 0;
}

/* Plain bisection for N_tot(mu) = n_target on [lo, hi] (Sec. 3.3 eq. fix_mu).
 * Stops when |N - n_target| <= tol.  Returns 0, or -1 when the bracket does not
 * bracket the target or max_iter is reached. */
int orc_find_mu_bisect(const orc_lattice* lat, const orc_sigma* sg, int tail_order, double n_target,
                       double tol, double lo, double hi, int max_iter, double* mu_out,
                       int* passes_out, double* n_out, int nthreads) {
  double nlo, nhi, nm = 0.0, mid = 0.5 * (lo + hi);
  int passes = 0;
  if (orc_trace(lat, sg, lo, tail_order, &nlo, NULL, nthreads)) return -2;
  if (orc_trace(lat, sg, hi, tail_order, &nhi, NULL, nthreads)) return -2;
  passes = 2;
  if ((nlo - n_target) * (nhi - n_target) > 0) return -1;
  int ok = 0;
  for (int it = 0; it < max_iter; ++it) {
    mid = 0.5 * (lo + hi);
    if (orc_trace(lat, sg, mid, tail_order, &nm, NULL, nthreads)) return -2;
    ++passes;
    if (fabs(nm - n_target) <= tol) { ok = 1; break; }
    if (nm < n_target) lo = mid; else hi = mid;
  }
  if (mu_out) *mu_out = mid;
  if (passes_out) *passes_out = passes;
  if (n_out) *n_out = nm;
  return ok ? 0 : -1;
}

/* Exposed for the oracle's own unit tests: inverse of one dense matrix. */
int orc_invert(int n, const double* a_in, double* g_out) {
  cplx* a = (cplx*)malloc(sizeof(cplx) * n * n);
  memcpy(a, a_in, sizeof(cplx) * n * n);
  int r = invert(n, a, (cplx*)g_out);
  free(a);
  return r;
}

/* Exposed for tests: G_kn itself for one (k, n). */
int orc_green(const orc_lattice* lat, const orc_sigma* sg, double mu, int k, int n, double* g_out) {
  int nc = lat->nc, nb = lat->nb[k];
  scratch sc;
  if (scratch_alloc(&sc, nb, nc)) return -1;
  build_a(lat, sg, k, n, mu, sc.a, sc.sig, sc.t);
  int r = invert(nb, sc.a, (cplx*)g_out);
  scratch_free(&sc);
  return r;
}
