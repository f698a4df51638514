/* Drives every entry point of oracle/dmft_oracle.c on small ragged inputs for
 * the sanitizer build (tests/test_sanitizers.py): memory safety and undefined
 * behaviour only -- the values are pinned by tests/test_oracle_pins.py.
 * Inputs come from a fixed linear congruential sequence. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int nk, nc;
  const int* nb;
  const int64_t* off_b;
  const int64_t* off_p;
  const double* eps;
  const double* wk;
  const double* proj;
} orc_lattice;

typedef struct {
  int nw;
  double beta;
  const double* sigma;
  const double* sigma_inf;
  const double* e_dc;
} orc_sigma;

int orc_density(const orc_lattice*, const orc_sigma*, double, int, const int*, int, double*, double*, int);
int orc_gloc(const orc_lattice*, const orc_sigma*, double, const int*, int, double*, int);
int orc_trace(const orc_lattice*, const orc_sigma*, double, int, double*, double*, int);
int orc_vjp(const orc_lattice*, const orc_sigma*, double, int, const double*, const double*, double*, double*, int);
int orc_find_mu_bisect(const orc_lattice*, const orc_sigma*, int, double, double, double, double, int, double*, int*,
                       double*, int);
int orc_invert(int, const double*, double*);
int orc_green(const orc_lattice*, const orc_sigma*, double, int, int, double*);

static uint64_t state = 12345;
static double uniform(void) { /* in [-1, 1) */
  state = state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(state >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

int main(void) {
  enum { NK = 4, NC = 3, NW = 12 };
  int nb[NK] = {3, 5, 8, 4};
  int64_t off_b[NK + 1], off_p[NK + 1], off_n = 0;
  off_b[0] = off_p[0] = 0;
  for (int k = 0; k < NK; ++k) {
    off_b[k + 1] = off_b[k] + nb[k];
    off_p[k + 1] = off_p[k] + (int64_t)NC * nb[k];
    off_n += (int64_t)nb[k] * nb[k];
  }
  double* eps = malloc(sizeof(double) * off_b[NK]);
  double* proj = malloc(sizeof(double) * 2 * off_p[NK]);
  double wk[NK], e_dc[NC], sinf[2 * NC * NC];
  double* sigma = malloc(sizeof(double) * 2 * NW * NC * NC);
  for (int64_t i = 0; i < off_b[NK]; ++i) eps[i] = 3.0 * uniform();
  for (int64_t i = 0; i < 2 * off_p[NK]; ++i) proj[i] = uniform();
  for (int k = 0; k < NK; ++k) wk[k] = 1.0 / NK;
  for (int a = 0; a < NC; ++a) e_dc[a] = 0.5 * uniform();
  for (int i = 0; i < 2 * NC * NC; ++i) sinf[i] = 0.1 * uniform();
  for (int n = 0; n < NW; ++n)
    for (int i = 0; i < NC * NC; ++i) {
      sigma[2 * (n * NC * NC + i)] = 0.2 * uniform();
      sigma[2 * (n * NC * NC + i) + 1] = -0.3 - 0.1 * fabs(uniform()); /* causal-looking imaginary part */
    }
  orc_lattice lat = {NK, NC, nb, off_b, off_p, eps, wk, proj};
  orc_sigma sig = {NW, 9.0, sigma, sinf, e_dc};
  int ks[NK] = {0, 1, 2, 3}, ns[3] = {0, 5, NW - 1};
  double* nkm = malloc(sizeof(double) * 2 * off_n);
  double ntr[NK], gl[2 * 3 * NC * NC], n0, d0;
  int bad = 0;
  for (int tail = 0; tail <= 2; tail += 2) {
    bad |= orc_density(&lat, &sig, 0.1, tail, ks, NK, nkm, ntr, 1);
    bad |= orc_trace(&lat, &sig, 0.1, tail, &n0, &d0, 1);
  }
  bad |= orc_gloc(&lat, &sig, 0.1, ns, 3, gl, 1);
  double* nbar = malloc(sizeof(double) * 2 * off_n);
  double* gbar = malloc(sizeof(double) * 2 * NW * NC * NC);
  double* sbar = malloc(sizeof(double) * 2 * NW * NC * NC);
  for (int64_t i = 0; i < 2 * off_n; ++i) nbar[i] = uniform();
  for (int i = 0; i < 2 * NW * NC * NC; ++i) gbar[i] = uniform();
  double mub;
  bad |= orc_vjp(&lat, &sig, -0.2, 2, nbar, gbar, sbar, &mub, 1);
  bad |= orc_vjp(&lat, &sig, -0.2, 0, NULL, gbar, sbar, &mub, 1);
  double mu;
  int passes;
  bad |= orc_find_mu_bisect(&lat, &sig, 2, 2.0, 1e-9, -20.0, 20.0, 200, &mu, &passes, &n0, 1) != 0;
  /* a target outside the bracket must be refused, not loop */
  if (orc_find_mu_bisect(&lat, &sig, 2, 100.0, 1e-9, -20.0, 20.0, 200, &mu, &passes, &n0, 1) != -1) bad |= 1;
  double a[2 * 9] = {0, 0, 2, 0, 1, 0, 1, 0, 0, 0, 0, 0, 0, 0, 1, 0, 0, 3}, g[2 * 9];
  bad |= orc_invert(3, a, g);
  double z[2 * 4] = {0};
  if (orc_invert(2, z, g) != -1) bad |= 1; /* singular */
  double gk[2 * 64];
  bad |= orc_green(&lat, &sig, 0.0, 2, 3, gk);
  free(eps); free(proj); free(sigma); free(nkm); free(nbar); free(gbar); free(sbar);
  if (bad) {
    fprintf(stderr, "an oracle call failed\n");
    return 1;
  }
  printf("oracle driver ok\n");
  return 0;
}
