// Low-rank Dyson step for 64-band windows on a pair of wavefronts (gfx950).
//
// The low-rank form (lowrank_impl.h) keeps the running frequency sum of G,
// a 64 x 64 complex matrix, in the registers of the wavefront that owns the
// k-point.  With one wavefront that sum only fits in the four-product form and
// leaves no room for the rest, so a single-wavefront item covers half of the
// columns and the nc x nc part of the step (X, both inversions, R) is computed
// twice, once per half.  Here a work-group of two wavefronts shares one item
// (k-tile, frequency tile):
//
//   wavefront w owns the column tiles b = 2w, 2w + 1 of the running sum
//   (eight 16 x 16 tiles, three-product form) and, for each group of eight
//   frequencies, the stage of frequencies 4w .. 4w + 3 of the group:
//
//   0. d_r = 1 / (i w_n + mu - E_r) of its four frequencies into an LDS table,
//      and Sigma(i w_n) of the same frequencies staged into LDS;
//   1. X_f = S D_f S^dag on the matrix cores (contraction over the bands; for
//      nc <= 8 two frequencies per product, see lr_x_packed);
//   2. lane 16 g + i takes row i of X_g: both inversions in the row layout
//      (rsweep), Gl_g = (X_g^-1 - Sigma'_g)^-1 back to LDS, and the lane's
//      row of w_k Gl_g added to the G_loc partial (read during the second
//      inversion);
//   2b. R = Sigma' + Sigma' Gl Sigma' of its four frequencies (a few nc x nc
//      products), written over Gl in the output layout;
//   -- work-group barrier: the d tables and R of all eight frequencies are
//      now in LDS --
//   3. for each of the eight frequencies, both wavefronts: for the owned
//      columns Q_b = (R S D)_b and sum_n G[t][b] += (D S^dag)_t Q_b for all
//      four row tiles t.
//   -- work-group barrier before the next group overwrites the LDS --
//
// so X, the inversions and R are computed once per frequency, and the running sum
// uses three matrix-core products per complex product.  Results and partial
// layouts are those of lr_tile (the same epilogues reduce them).
#pragma once

#include <type_traits>

#include "lowrank_impl.h"

namespace dmft {

struct LRPairShared {
  double2 buf[8][16 * 17];  // X, then Gl, of the group's eight frequencies (rows padded to 17)
  double2 sg[8][16 * 17];   // Sigma(i w_n) of the same frequencies (V_DC is taken off where read)
  double2 dtab[8][64];      // d_r of the same frequencies (zero past nb)
};

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Three-product complex multiply-add with the operand sums given.
__device__ __forceinline__ void mac3(v4d& p1, v4d& p2, v4d& p3, double ar, double ai, double as, double br, double bi,
                                     double bs) {
  p1 = mma(ar, br, p1);
  p2 = mma(ai, bi, p2);
  p3 = mma(as, bs, p3);
}

// ---------------------------------------------------------------------------
// Partial-fraction form of the running sum (64-band windows, nc > 8).
//
// The running sum needs F[v][v'] = sum_n d_v d_v' M_n[v][v'], M_n = S^dag R_n S,
// with d_v = 1 / (z_n - E_v).  Since d_v d_v' = (d_v - d_v') / (E_v - E_v')
// exactly, for E_v != E_v'
//     F[v][v'] = ((W S)[v][v'] - (S^dag Y)[v][v']) / (E_v - E_v'),
//     W = sum_n D_n S^dag R_n  (nb x nc),   Y = sum_n R_n S D_n  (nc x nb),
// so each frequency adds two rank-nc products of nb x nc instead of the nb x nb
// update (D S^dag)(R S D), and the nb x nb products are formed once per k.  The
// subtraction loses about |d| / |E_v - E_v'| digits, so pairs closer than
// delta = pi / (16 beta) (a sixteenth of the first Matsubara frequency;
// normwise relative errors below 1e-12 on the test and benchmark inputs, and
// near 3e-11 on the element of a pair just outside delta at beta = 100) and the diagonal are
// summed directly: per owned column v' the diagonal sum_n d_v'^2 (R_n S)[.][v']
// and, for at most one close partner v, sum_n d_v d_v' (R_n S)[.][v'], each
// contracted with S^dag at the end of the k-point.  A k-point on which some
// column has more than one close partner takes the direct running sum.

// Close partners of the two owned columns v0 and v0 + 16 (v0 = 32 w + c16);
// returns whether the partial-fraction form applies to the k-point (the same
// answer in every thread of the work-group).
__device__ __forceinline__ bool pf_pairs(const double* eps, int nb, int v0, double beta, int (&partner)[2]) {
  const double delta = M_PI / (16.0 * beta);
  int over = 0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int vc = v0 + 16 * c;
    const double ec = vc < nb ? eps[vc] : 0.0;
    int cnt = 0, pv = -1;
    for (int v = 0; v < nb; ++v) {
      const bool close = vc < nb && v != vc && __builtin_fabs(eps[v] - ec) < delta;
      pv = close ? v : pv;
      cnt += close ? 1 : 0;
    }
    partner[c] = pv;
    over |= cnt > 1;
  }
  return !__syncthreads_or(over);
}

// Register map of the partial-fraction accumulators onto the running sum's
// three-product accumulators s1, s2, s3 [4][2] (compile-time indices only):
//   W of owned row tile l (l = 0, 1)      s1[l][0], s2[l][0], s3[l][0]  (three products)
//   Y of owned column c (re, im)          s1[2][c], s2[2][c]
//   diagonal sum of owned column c        s3[2][c], s1[3][c]
//   close-pair sum of owned column c      s2[3][c], s3[3][c]
// Y, the diagonal and the close-pair sums are in the output layout of R S:
// register i holds row (orbital) q + 4 i, the lane's column.

// One frequency: R^T (registers, R[c16][q + 4 i]) and R read transposed from
// the LDS tile that holds R^T; Q = R S for the owned columns, Y += Q d_v',
// diagonal += Q d_v'^2, close += Q d_p d_v', and W += (D S^dag) R for the owned
// row tiles.
template <int NC>
__device__ __forceinline__ void pf_step(v4d (&s1)[4][2], v4d (&s2)[4][2], v4d (&s3)[4][2], double2 (&dsum)[2],
                                        const v4d& rtr, const v4d& rti, const double2* rt, const double2* dt,
                                        const double (&par)[4][4], const double (&pai)[4][4],
                                        const int (&partner)[2], int kc, int w, int q, int c16) {
  v4d rnr, rni;  // R[q + 4 i][c16]
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 v = rt[c16 * 17 + q + 4 * i];
    rnr[i] = v.x;
    rni[i] = v.y;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const double2 d = dt[16 * (2 * w + c) + c16];
    dsum[c].x += d.x;
    dsum[c].y += d.y;
    const double2 d2 = cmul(d, d);
    const double2 dp = partner[c] >= 0 ? cmul(d, dt[partner[c]]) : make_double2(0.0, 0.0);
    CAcc<true> qa;
    qa.zero();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j >= kc) break;
      qa.mac(rtr[j], rti[j], w ? par[j][2 + c] : par[j][c], w ? pai[j][2 + c] : pai[j][c]);
    }
    const v4d xr = qa.re(), xi = qa.im();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double2 x = make_double2(xr[i], xi[i]);
      const double2 y = cmul(x, d), g = cmul(x, d2), p = cmul(x, dp);
      s1[2][c][i] += y.x;
      s2[2][c][i] += y.y;
      s3[2][c][i] += g.x;
      s1[3][c][i] += g.y;
      s2[3][c][i] += p.x;
      s3[3][c][i] += p.y;
    }
  }
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    const double2 dr = dt[16 * (2 * w + l) + c16];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j >= kc) break;
      const double sr = w ? par[j][2 + l] : par[j][l], si = w ? pai[j][2 + l] : pai[j][l];
      const double2 aa = cmul(dr, make_double2(sr, -si));
      mac3(s1[l][0], s2[l][0], s3[l][0], aa.x, aa.y, aa.x + aa.y, rnr[j], rni[j], rnr[j] + rni[j]);
    }
  }
}

// End of a k-point: W of both wavefronts and the wavefront's Y through LDS,
// the diagonal and close-pair sums contracted first, then for the owned
// columns and every row tile F = (W S - S^dag Y) / (E_v - E_v'), the diagonal
// and the close pair from their direct sums, plus the D term on the diagonal;
// stored in the running sum's partial layout.  The tiles run in a loop (not
// unrolled) with their operands read where they are used, so that little is
// live at once.
template <int NC>
__device__ __forceinline__ void pf_finish(v4d (&s1)[4][2], v4d (&s2)[4][2], v4d (&s3)[4][2],
                                          const double2 (&dsum)[2], LRPairShared& sh, const double2* P,
                                          const double* eps, int nb, int nc, int kc, const int (&partner)[2],
                                          double2* sp, int w, int q, int c16, int tid) {
  constexpr int T = 4;
  const int lane = tid & 63;
  // the frequency loop ended with a work-group barrier: the Gl/R and Sigma tiles are free
  double2* wl = &sh.buf[0][0];  // W[v][beta] at v * 17 + beta (64 x 17 < 8 x 16 x 17)
  double2* yl = &sh.sg[0][0];   // Y of owned column c, register i, at ((2 w + c) 4 + i) 64 + lane
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    const v4d re = s1[l][0] - s2[l][0], im = s3[l][0] - s1[l][0] - s2[l][0];
#pragma unroll
    for (int i = 0; i < 4; ++i) wl[(16 * (2 * w + l) + q + 4 * i) * 17 + c16] = make_double2(re[i], im[i]);
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < 4; ++i) yl[((2 * w + c) * 4 + i) * 64 + lane] = make_double2(s1[2][c][i], s2[2][c][i]);
  // the diagonal and the close pair: sum over the orbitals q + 4 i (this lane's
  // registers, then the four lanes of the column)
  double2 dg[2], cl[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int vc = 16 * (2 * w + c) + c16;
    const int pv = partner[c];
    dg[c] = cl[c] = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double2 s = lr_proj_here(P, q + 4 * i, vc, nc, nb);
      dg[c] = cadd(dg[c], cmul(make_double2(s.x, -s.y), make_double2(s3[2][c][i], s1[3][c][i])));
      const double2 sp_ = pv >= 0 ? lr_proj_here(P, q + 4 * i, pv, nc, nb) : make_double2(0.0, 0.0);
      cl[c] = cadd(cl[c], cmul(make_double2(sp_.x, -sp_.y), make_double2(s2[3][c][i], s3[3][c][i])));
    }
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
      dg[c].x += __shfl_xor(dg[c].x, off);
      dg[c].y += __shfl_xor(dg[c].y, off);
      cl[c].x += __shfl_xor(cl[c].x, off);
      cl[c].y += __shfl_xor(cl[c].y, off);
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int b = 2 * w + c;
    const int vc = 16 * b + c16;
    const double ec = vc < nb ? eps[vc] : 0.0;
    const int pv = partner[c];
    const double2 dgc = make_double2(dg[c].x + dsum[c].x, dg[c].y + dsum[c].y), clc = cl[c];
#pragma unroll 1
    for (int t = 0; t < T; ++t) {
      CAcc<true> acc;
      acc.zero();
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j >= kc) break;
        const double2 wv = wl[(16 * t + c16) * 17 + q + 4 * j];  // W[16 t + c16][q + 4 j]
        const double2 sb = lr_proj_here(P, q + 4 * j, vc, nc, nb);
        acc.mac(wv.x, wv.y, sb.x, sb.y);
        const double2 st = lr_proj_here(P, q + 4 * j, 16 * t + c16, nc, nb);  // - S^dag: -(S[q + 4 j][16 t + c16])^*
        const double2 yv = yl[(b * 4 + j) * 64 + lane];
        acc.mac(-st.x, st.y, yv.x, yv.y);
      }
      const v4d fr = acc.re(), fi = acc.im();
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int v = 16 * t + q + 4 * i;
        double2 val;
        if (v == vc) {
          val = dgc;
        } else if (v == pv) {
          val = clc;
        } else {
          const double ev = v < nb ? eps[v] : 0.0;
          const double inv = (v < nb && vc < nb) ? 1.0 / (ev - ec) : 0.0;
          val = make_double2(fr[i] * inv, fi[i] * inv);
        }
        sp[((t * T + b) * 4 + i) * 64 + lane] = val;
      }
    }
  }
  __syncthreads();  // W's and Y's LDS are the next k-point's X and Sigma tiles
}

// NC: columns kept in the row-layout inversions (nc <= NC).  PF: the running sum
// in the partial-fraction form (see pf_pairs below) on every k-point where it
// applies.
template <int NC, bool PF = false>
__device__ __forceinline__ void lr_pair_tile(const DysonArgs& a, int ktile, int wtile, LRPairShared& sh, int tid) {
  constexpr int NBP = 64, T = 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int q = lane >> 4, c16 = lane & 15;
  const int n0 = wtile * a.wt;
  const int n1 = min(n0 + a.wt, a.nw);
  const int kk0 = ktile * a.kt;
  const int kk1 = min(kk0 + a.kt, a.nklist);
  const double mu = uniform_d(a.mu_ptr ? *a.mu_ptr : a.mu);
  const int nc = a.nc;
  const int kc = (nc + 3) >> 2;
  // the launch keeps nc <= NC columns and takes more than 8 only for nc > 8
  __builtin_assume(kc >= 1 && kc <= 4);
  __builtin_assume(nc >= 1 && nc <= NC);
  if constexpr (NC > 8) __builtin_assume(nc > 8);
  const double beta = a.beta;
  const bool want_s = (a.mode & MODE_S) != 0;
  const bool want_x = (a.mode & MODE_GLOC) != 0;
  const bool hasdiag = c16 >= q && ((c16 - q) & 3) == 0;
  const int idg = (c16 - q) >> 2;
  // V_DC of orbital c16: every diagonal element of Sigma' a lane reads is (c16, c16)
  const double edc = c16 < nc ? a.e_dc[c16] : 0.0;
  int bad = 0, nonfinite = 0;

  for (int kk = kk0; kk < kk1; ++kk) {
    const int k = uniform_i(a.klist ? a.klist[kk] : kk);
    const int nb = uniform_i(a.nb_uniform > 0 ? a.nb_uniform : a.nb[k]);
    // every k of a 64-band bucket has 48 < nb <= 64 (checked on the host)
    __builtin_assume(nb > NBP - 16 && nb <= NBP);
    const int64_t ob = uniform_l(a.nb_uniform > 0 ? (int64_t)k * nb : a.off_b[k]);
    const double* eps = a.eps + ob;
    const double2* P = reinterpret_cast<const double2*>(a.proj) + ob * nc;
    const double wk = uniform_d(a.wk[k]);
    // partial-fraction form: the close partner (if any) of each owned column,
    // and whether every column of the work-group has at most one
    int partner[2] = {-1, -1};
    bool pfk = false;
    if constexpr (PF) pfk = pf_pairs(eps, nb, 16 * 2 * w + c16, a.beta, partner);
    // one k-point, with the running sum in the direct (PFK false) or the
    // partial-fraction form; the two instantiations keep separate registers
    auto k_body = [&](auto pf_tag) {
      constexpr bool PFK = decltype(pf_tag)::value;
      // running sum of G: all four row tiles of the two owned column tiles; in the
      // partial-fraction form the same registers hold W of the owned row tiles and
      // Y, the diagonal and the close-pair sums of the owned columns (PfAcc)
      v4d s1[T][2], s2[T][2], s3[T][2];
  #pragma unroll
      for (int t = 0; t < T; ++t)
  #pragma unroll
        for (int c = 0; c < 2; ++c) s1[t][c] = s2[t][c] = s3[t][c] = (v4d){0.0, 0.0, 0.0, 0.0};
      double2 dsum[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};

      for (int n = n0; n < n1; n += 8) {
        // ---- 0. resolvent table and Sigma of this wavefront's four frequencies
        const int nw0 = n + 4 * w;
        {
          const double er = lane < nb ? eps[lane] : 0.0;  // band lane of the table
  #pragma unroll
          for (int f = 0; f < 4; ++f) {
            const int nf = min(nw0 + f, n1 - 1);
            const double wn = (double)(2 * nf + 1) * M_PI / beta;
            sh.dtab[4 * w + f][lane] = lane < nb ? inv_z_minus(mu, wn, er) : make_double2(0.0, 0.0);
          }
        }
        // Sigma of the four frequencies, NC x NC positions each, loaded now and
        // stored to LDS after the X products (their latency hides behind them)
        constexpr int NPOS = 4 * NC * NC;
        constexpr int NLD = (NPOS + 63) / 64;
        // The positions come from a lane index the compiler cannot see through:
        // hoisted out of the frequency loop they would be kept (and spilled) as
        // one 64-bit address per load, each reloaded before its load.
        int lane_l = lane;
        asm volatile("" : "+v"(lane_l));
        // One base address per group (uniform) and 32-bit offsets per load.
        const double2* sgb = reinterpret_cast<const double2*>(a.sigma) + (int64_t)nw0 * nc * nc;
        const int flast = n1 - 1 - nw0;
        double2 sgl[NLD];
  #pragma unroll
        for (int m = 0; m < NLD; ++m) {
          const int idx = lane_l + 64 * m;
          const int f = idx / (NC * NC), rem = idx - f * (NC * NC);
          const int ra = rem / NC, cb = rem - ra * NC;
          const bool in = idx < NPOS && ra < nc && cb < nc;
          sgl[m] = in ? sgb[min(f, flast) * nc * nc + ra * nc + cb] : make_double2(0.0, 0.0);
        }
        wave_sync();
        // ---- 1. X_f = S D_f S^dag of the four frequencies into LDS
        {
          double ptr_[T][4], pti_[T][4];
  #pragma unroll
          for (int t = 0; t < T; ++t)
  #pragma unroll
            for (int i = 0; i < 4; ++i) {
              const double2 v = lr_proj(fresh(P), c16, 16 * t + 4 * i + q, nc, nb);
              ptr_[t][i] = v.x;
              pti_[t][i] = v.y;
            }
          if constexpr (NC <= 8) {
            // two frequencies per product, stacked in the A rows (see lr_x_packed)
  #pragma unroll
            for (int c = 0; c < 2; ++c) {
              const int fa = 4 * w + 2 * c + (c16 >> 3);
              CAcc<true> x;
              x.zero();
  #pragma unroll
              for (int t = 0; t < T; ++t)
  #pragma unroll
                for (int i = 0; i < 4; ++i) {
                  if (16 * t + 4 * i >= nb) break;
                  const double2 s = make_double2(ptr_[t][i], pti_[t][i]);
                  const double2 sa = lower_rows8(s);
                  const double2 dd = sh.dtab[fa][16 * t + 4 * i + q];
                  const double2 a1 = cmul(sa, dd);
                  x.mac_cb(a1.x, a1.y, s.x, s.y);
                }
              const v4d xr = x.re(), xi = x.im();
  #pragma unroll
              for (int i = 0; i < 4; ++i)
                sh.buf[4 * w + 2 * c + (i >> 1)][(4 * (i & 1) + q) * 17 + c16] = make_double2(xr[i], xi[i]);
            }
          } else {
  #pragma unroll
            for (int f = 0; f < 4; ++f) {
              CAcc<true> x;
              x.zero();
  #pragma unroll
              for (int t = 0; t < T; ++t)
  #pragma unroll
                for (int i = 0; i < 4; ++i) {
                  if (16 * t + 4 * i >= nb) break;
                  const double2 s = make_double2(ptr_[t][i], pti_[t][i]);
                  const double2 dd = sh.dtab[4 * w + f][16 * t + 4 * i + q];
                  const double2 a1 = cmul(s, dd);
                  x.mac_cb(a1.x, a1.y, s.x, s.y);
                }
              const v4d xr = x.re(), xi = x.im();
  #pragma unroll
              for (int i = 0; i < 4; ++i) sh.buf[4 * w + f][(q + 4 * i) * 17 + c16] = make_double2(xr[i], xi[i]);
            }
          }
        }
        // Sigma to LDS.  The positions are recomputed from a lane index the
        // compiler cannot see through, so that they are not kept (and spilled)
        // across the X products.
        int lane_r = lane;
        asm volatile("" : "+v"(lane_r));
  #pragma unroll
        for (int m = 0; m < NLD; ++m) {
          const int idx = lane_r + 64 * m;
          const int f = idx / (NC * NC), rem = idx - f * (NC * NC);
          const int ra = rem / NC, cb = rem - ra * NC;
          if (idx < NPOS && ra < nc && cb < nc) sh.sg[4 * w + f][ra * 17 + cb] = sgl[m];
        }
        wave_sync();
        // ---- 2. row layout: invert X, subtract Sigma', invert K -> Gl; G_loc partial
        {
          const int g = 4 * w + q, ri = c16;
          const int nfg = n + g;  // frequencies past n1 were clamped copies: no partial
          // rows past nc start as zero rows and stay zero through both sweeps (the
          // packed X of nc <= 8 leaves rows 8 .. 15 of the tile unwritten)
          const bool rin = ri < nc;
          double rr[NC], rim[NC];
  #pragma unroll
          for (int j = 0; j < NC; ++j) {
            const double2 v = rin ? sh.buf[g][ri * 17 + j] : make_double2(0.0, 0.0);
            rr[j] = v.x;
            rim[j] = v.y;
          }
          rsweep<0, NC>(rr, rim, ri, nc, bad);
          // this lane's row of the G_loc partial of frequency nfg: element
          // (ri, j) sits at (ri / 4) * 64 + 16 (ri % 4) + j in the partial's
          // matrix-core lane order; read now, used after the second inversion
          const bool gl_row = want_x && rin && nfg < n1;
          double2* prow = reinterpret_cast<double2*>(a.xpart) +
                          ((int64_t)(a.ktile_base + ktile) * a.nw + min(nfg, n1 - 1)) * 256 + (ri >> 2) * 64 +
                          16 * (ri & 3);
          double2 prev[NC];
  #pragma unroll
          for (int j = 0; j < NC; ++j)
            prev[j] = (gl_row && kk != kk0 && j < nc) ? prow[j] : make_double2(0.0, 0.0);
  #pragma unroll
          for (int j = 0; j < NC; ++j) {
            if (j < nc && rin) {
              double2 v = sh.sg[g][ri * 17 + j];
              if (j == ri) v.x -= edc;
              rr[j] -= v.x;
              rim[j] -= v.y;
            }
          }
          rsweep<0, NC>(rr, rim, ri, nc, bad);
  #pragma unroll
          for (int j = 0; j < NC; ++j) sh.buf[g][ri * 17 + j] = make_double2(rr[j], rim[j]);
          // the packed X of nc <= 8 leaves rows 8 .. 15 unwritten: complete the
          // tile, so that every element outside Gl's nc x nc corner read later is zero
          if constexpr (NC <= 8) {
  #pragma unroll
            for (int j = NC; j < 16; ++j) sh.buf[g][ri * 17 + j] = make_double2(0.0, 0.0);
          }
          if (gl_row) {
  #pragma unroll
            for (int j = 0; j < NC; ++j)
              if (j < nc) prow[j] = make_double2(wk * rr[j] + prev[j].x, wk * rim[j] + prev[j].y);
          }
        }
        wave_sync();
        // ---- 2b. R of this wavefront's four frequencies, in the output layout, in
        //     place of Gl (each lane overwrites only the elements it has read), so
        //     that stage 3 reads R instead of both wavefronts forming it
  #pragma unroll 1
        for (int f = 0; f < 4; ++f) {
          const int g = 4 * w + f;
          if (n + g >= n1) break;
          v4d glr, gli;
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double2 v = sh.buf[g][(q + 4 * i) * 17 + c16];
            glr[i] = v.x;
            gli[i] = v.y;
          }
          double sa_r[4], sa_i[4];
          v4d sbr, sbi;
  #pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int be = q + 4 * j;
            const bool in = c16 < nc && be < nc;
            double2 v = in ? sh.sg[g][c16 * 17 + be] : make_double2(0.0, 0.0);
            double2 u = in ? sh.sg[g][be * 17 + c16] : make_double2(0.0, 0.0);
            if (in && be == c16) {
              v.x -= edc;
              u.x -= edc;
            }
            sa_r[j] = v.x;
            sa_i[j] = v.y;
            sbr[j] = u.x;
            sbi[j] = u.y;
          }
          // V = Gl^T Sigma'^T, R^T = Sigma'^T + Sigma'^T V
          CAcc<true> va;
          va.zero();
  #pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (j >= kc) break;
            va.mac(glr[j], gli[j], sa_r[j], sa_i[j]);
          }
          const v4d vr = va.re(), vi = va.im();
          CAcc<true> ra;
          ra.set((v4d){sa_r[0], sa_r[1], sa_r[2], sa_r[3]}, (v4d){sa_i[0], sa_i[1], sa_i[2], sa_i[3]});
  #pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (j >= kc) break;
            ra.mac(sbr[j], sbi[j], vr[j], vi[j]);
          }
          const v4d rtr = ra.re(), rti = ra.im();
          double chk = 0.0;
  #pragma unroll
          for (int i = 0; i < 4; ++i) chk += glr[i] + gli[i] + rtr[i] + rti[i];
          if (!__builtin_isfinite(chk)) nonfinite = 1;
  #pragma unroll
          for (int i = 0; i < 4; ++i) sh.buf[g][(q + 4 * i) * 17 + c16] = make_double2(rtr[i], rti[i]);
        }
        __syncthreads();
        // ---- 3. all eight frequencies: the owned columns of sum_n G
        // projector fragments S[q + 4 j][16 t + c16] for every row tile (A operands of
        // (D S^dag)_t and, for the owned columns, B operands of Q)
        double par[4][T], pai[4][T];
  #pragma unroll
        for (int j = 0; j < 4; ++j)
  #pragma unroll
          for (int t = 0; t < T; ++t) {
            const double2 v = lr_proj(fresh(P), q + 4 * j, 16 * t + c16, nc, nb);
            par[j][t] = v.x;
            pai[j][t] = v.y;
          }
  #pragma unroll 1
        for (int f8 = 0; f8 < 8; ++f8) {
          const int nf = n + f8;
          if (nf >= n1) break;
          v4d rtr, rti;  // R^T of the frequency (R[c16][q + 4 i])
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double2 v = sh.buf[f8][(q + 4 * i) * 17 + c16];
            rtr[i] = v.x;
            rti[i] = v.y;
          }
          if (!want_s) continue;
          if constexpr (PFK) {
            pf_step<NC>(s1, s2, s3, dsum, rtr, rti, sh.buf[f8], sh.dtab[f8], par, pai, partner, kc, w, q, c16);
            continue;
          }
          // (register arrays are indexed by compile-time values only: the owned
          // column tiles 2w, 2w + 1 are picked by selects, not by indexing with w)
          double2 dcol[T];
  #pragma unroll
          for (int t = 0; t < T; ++t) dcol[t] = sh.dtab[f8][16 * t + c16];
          double2 down[2];
  #pragma unroll
          for (int c = 0; c < 2; ++c) {
            down[c] = w ? dcol[2 + c] : dcol[c];
            dsum[c].x += down[c].x;
            dsum[c].y += down[c].y;
          }
          // Q_b = (R S)_b D_b for the owned column tiles, operand sums formed once
          double qr[2][4], qi[2][4], qs[2][4];
  #pragma unroll
          for (int c = 0; c < 2; ++c) {
            CAcc<true> qa;
            qa.zero();
  #pragma unroll
            for (int j = 0; j < 4; ++j) {
              if (j >= kc) break;
              qa.mac(rtr[j], rti[j], w ? par[j][2 + c] : par[j][c], w ? pai[j][2 + c] : pai[j][c]);
            }
            const v4d xr = qa.re(), xi = qa.im();
            const double2 db = down[c];
  #pragma unroll
            for (int i = 0; i < 4; ++i) {
              const double2 v = cmul(make_double2(xr[i], xi[i]), db);
              qr[c][i] = v.x;
              qi[c][i] = v.y;
              qs[c][i] = v.x + v.y;
            }
          }
          // sum_n G[t][b] += (D S^dag)_t Q_b, contraction over the orbitals
  #pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (j >= kc) break;
  #pragma unroll
            for (int t = 0; t < T; ++t) {
              const double2 aa = cmul(dcol[t], make_double2(par[j][t], -pai[j][t]));
              const double as = aa.x + aa.y;
  #pragma unroll
              for (int c = 0; c < 2; ++c) mac3(s1[t][c], s2[t][c], s3[t][c], aa.x, aa.y, as, qr[c][j], qi[c][j], qs[c][j]);
            }
          }
        }
        __syncthreads();
      }  // frequency groups

      if (PFK && want_s) {
        double2* sp = reinterpret_cast<double2*>(a.spart) + (int64_t)wtile * a.s_stride + a.off_s[k];
        pf_finish<NC>(s1, s2, s3, dsum, sh, P, eps, nb, nc, kc, partner, sp, w, q, c16, tid);
      } else if (want_s) {
        double2* sp = reinterpret_cast<double2*>(a.spart) + (int64_t)wtile * a.s_stride + a.off_s[k];
  #pragma unroll
        for (int t = 0; t < T; ++t)
  #pragma unroll
          for (int c = 0; c < 2; ++c) {
            const int b = 2 * w + c;
            const v4d re = s1[t][c] - s2[t][c], im = s3[t][c] - s1[t][c] - s2[t][c];
  #pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int e = (t * T + b) * 4 + i;  // address only: no register indexed by w
              double2 v = make_double2(re[i], im[i]);
              if (t == b && hasdiag && idg == i) {
                v.x += dsum[c].x;
                v.y += dsum[c].y;
              }
              sp[e * 64 + lane] = v;
            }
          }
      }
    };
    if (PF && pfk)
      k_body(std::true_type{});
    else
      k_body(std::false_type{});
  }  // k
  if (bad) atomicOr(a.err, ERR_SINGULAR);
  if (nonfinite) atomicOr(a.err, ERR_NONFINITE);
}

}  // namespace dmft
