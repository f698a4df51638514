// Low-rank density step for at most five correlated orbitals, three
// frequencies per matrix-core tile (gfx950 / CDNA4).
//
// The step is the one of lowrank_impl.h (Woodbury form of the lattice Dyson
// equation, embedding of the DMFT-loop section):
//     X = S D S^dag,  Gl = (X^-1 - Sigma')^-1,  R = Sigma' + Sigma' Gl Sigma',
//     sum_n G += D + (D S^dag)(R S D),   G_loc partial += w_k Gl.
// With nc <= 5 an nc x nc matrix fills at most a 5 x 5 corner of a 16 x 16
// tile, so here three frequencies share every tile, block-diagonally: packed
// index p = 5 h + alpha (h = 0, 1, 2 the frequency of the slot, alpha < 5 the
// orbital; p = 15 is unused).  Block-diagonal operands give block-diagonal
// products, so one chain of 16x16x4 products serves three frequencies:
//   X    A row p = S[alpha][r] d_h[r], B column beta = S[beta][r]^*  ->  row p, column
//        beta holds X_h[alpha][beta]  (one product for three frequencies);
//   V, R  Gl and Sigma' of the slot block-diagonal, contraction over the packed
//        index: four steps for three frequencies;
//   Q    = R S_3 D with S_3[5 h + beta][v] = S[beta][v] (the same projector for
//        every block) and row p scaled by d_h[v];
//   sum_n G += [D_0 S^dag | D_1 S^dag | D_2 S^dag] Q: the contraction over the
//        packed index sums the three frequencies' updates at once.
// Per three frequencies that is X T x 4, V 4, R 4, Q T x 4 and the running sum
// T^2 x 4 steps (T = padded bands / 16), against three times X T x 2 and V 2,
// R 2, Q T x 2, sum T^2 x 2 of the two-frequency packing of lowrank_impl.h: a
// third fewer matrix-core products.
//
// A wavefront walks a (k-tile, frequency-tile) item twelve frequencies at a
// time, in four slots of three:
//   0. d_r of the twelve frequencies into LDS;
//   1. X of the four slots (one packed product each) into LDS;
//   2. row layout, three sub-sweeps: lane 16 g + i holds row i of X of the
//      frequency 3 g + h of sub-sweep h; both Gauss-Jordan inversions of
//      lowrank_impl.h (rsweep, five columns), the w_k Gl partial of G_loc
//      added row by row, and Gl written back block-diagonally;
//   3. per slot, in the output layout: V, R, Q, the running sum.
// Frequencies past the tile's end repeat its last one in stages 0-2 (so every
// inversion is of a valid matrix) and enter stage 3 with d = 0, which removes
// them from Q and from the running sum.  64-band windows run the same steps on
// four wavefronts (lr_p3_quad_tile, below).  Both kernels also carry the
// partial-fraction form of the running sum (PF, on the k-points where every
// band has at most one close partner; see p3q_pf_step below and
// lowrank_pair_impl.h): stage 3 then forms P = S^dag R and Q = R S of each slot
// instead of the nb x nb update.
#pragma once

#include "lowrank_impl.h"
#include "lowrank_pair_impl.h"  // mac3

namespace dmft {

template <int NBP>
struct LRP3Shared {
  double2 buf[4][16 * 17];  // per slot: X of its three frequencies, then their block-diagonal Gl
  double2 dtab[12][NBP];    // d_r = 1 / (i w + mu - E_r) of the group's frequencies (zero past nb)
};

// S[c16 mod 5][r] from the lane's S[c16][r] when nc <= 5 (rows 5 .. 15 of S are
// zero): the values five and ten lanes back along the 16-lane row (row_shr:5,
// row_shr:10; lanes before the row's start read zero) are added.  Lane 15 gets
// zero, as rows 5, 10 and 15 are zero.
__device__ __forceinline__ double2 spread5(double2 s) {
  const double x = s.x + __builtin_amdgcn_update_dpp(0.0, s.x, 0x115, 0xf, 0xf, true) +
                   __builtin_amdgcn_update_dpp(0.0, s.x, 0x11a, 0xf, 0xf, true);
  const double y = s.y + __builtin_amdgcn_update_dpp(0.0, s.y, 0x115, 0xf, 0xf, true) +
                   __builtin_amdgcn_update_dpp(0.0, s.y, 0x11a, 0xf, 0xf, true);
  return make_double2(x, y);
}

// Projector fragments of the X products: pt[t][i] = S[c16][16 t + 4 i + q] (B
// operand, conjugated) and ps[t][i] = S[c16 mod 5][16 t + 4 i + q] (A operand).
template <int T>
__device__ __forceinline__ void p3_load_x(double2 (&pt)[T][4], double2 (&ps)[T][4], const double2* P, int nc, int nb,
                                          int q, int c16) {
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      pt[t][i] = lr_proj_here(P, c16, 16 * t + 4 * i + q, nc, nb);
      ps[t][i] = spread5(pt[t][i]);
    }
}
// pk[j][b] = S[aj][16 b + c16]: B operand of R S_3, and (conjugated) of D S^dag.
template <int T>
__device__ __forceinline__ void p3_load_k(double2 (&pk)[4][T], const double2* P, const int (&hj)[4],
                                          const int (&aj)[4], int nc, int nb, int c16) {
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int b = 0; b < T; ++b)
      pk[j][b] = hj[j] < 3 ? lr_proj_here(P, aj[j], 16 * b + c16, nc, nb) : make_double2(0.0, 0.0);
}

// RL = 0: projector fragments kept in registers for the whole k; RL = 1: loaded
// per group of twelve frequencies at the start of the stage that uses them
// (48-band windows, whose fragments would not fit next to the running sum).
template <int NBP, int RL, bool M3, bool PF = false>
__device__ __forceinline__ void lr_p3_tile(const DysonArgs& a, int ktile, int wtile, LRP3Shared<NBP>& sh, int lane,
                                           double2* pfc = nullptr) {
  constexpr int T = NBP / 16;
  constexpr int NDT = 12 * NBP / 64;  // resolvent-table entries per lane
  const int q = lane >> 4, c16 = lane & 15;
  const int g = q, ri = c16;  // row layout: slot g, row ri
  const int n0 = wtile * a.wt;
  const int n1 = min(n0 + a.wt, a.nw);
  const int kk0 = ktile * a.kt;
  const int kk1 = min(kk0 + a.kt, a.nklist);
  const double mu = uniform_d(a.mu_ptr ? *a.mu_ptr : a.mu);
  const int nc = a.nc;
  // the dispatchers take this kernel for nc <= 5 only
  __builtin_assume(nc >= 1 && nc <= 5);
  const double beta = a.beta;
  const bool want_s = (a.mode & MODE_S) != 0;
  const bool want_x = (a.mode & MODE_GLOC) != 0;
  const bool hasdiag = c16 >= q && ((c16 - q) & 3) == 0;
  const int idg = (c16 - q) >> 2;
  // packed index of the lane's output column (and A row): c16 = 5 hc + ac
  const int hc = c16 / 5;  // 3 for c16 = 15: no block
  const int ac = c16 - 5 * hc;
  const bool cin = hc < 3 && ac < nc;
  // packed index q + 4 j of the lane's contraction slot j: 5 hj + aj
  int hj[4], aj[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    hj[j] = (q + 4 * j) / 5;
    aj[j] = q + 4 * j - 5 * hj[j];
  }
  const double edc_c = cin ? a.e_dc[ac] : 0.0;
  const double edc_r = ri < nc ? a.e_dc[ri] : 0.0;
  int bad = 0, nonfinite = 0;

  for (int kk = kk0; kk < kk1; ++kk) {
    const int k = uniform_i(a.klist ? a.klist[kk] : kk);
    const int nb = uniform_i(a.nb_uniform > 0 ? a.nb_uniform : a.nb[k]);
    __builtin_assume(nb >= 1 && nb <= NBP);
    // bucketed by padded size (checked on the host before any launch)
    __builtin_assume(nb > NBP - 16);
    const int64_t ob = uniform_l(a.nb_uniform > 0 ? (int64_t)k * nb : a.off_b[k]);
    const double* eps = a.eps + ob;
    // band of table entry lane + 64 it: (lane + 64 it) mod NBP takes NE distinct
    // values per lane (64 it mod 48 = 16 (it mod 3); one value for 16 and 32)
    constexpr int NE = NBP == 48 ? 3 : 1;
    double epl[NE];
#pragma unroll
    for (int it = 0; it < NE; ++it) {
      const int r = (lane + 64 * it) % NBP;
      epl[it] = r < nb ? eps[r] : 0.0;
    }
    const double2* P = reinterpret_cast<const double2*>(a.proj) + ob * nc;
    const double wk = uniform_d(a.wk[k]);
    // partial-fraction form: the close partner (if any) of each owned column,
    // and whether every column has at most one
    int partner[T];
#pragma unroll
    for (int t = 0; t < T; ++t) partner[t] = -1;
    bool pfk = false;
    if constexpr (PF) pfk = want_s && lr_pf_pairs<T>(eps, nb, c16, beta, partner);
    // one k-point, with the running sum in the direct (PFK false) or the
    // partial-fraction form; the two instantiations keep separate registers
    auto k_body = [&](auto pf_tag) {
    constexpr bool PFK = decltype(pf_tag)::value;
    double2 pt[T][4], ps[T][4], pk[4][T];
    if constexpr (RL == 0) {
      p3_load_x<T>(pt, ps, P, nc, nb, q, c16);
      p3_load_k<T>(pk, P, hj, aj, nc, nb, c16);
    }
    // direct form: the running sum; partial-fraction form: W (rows 16 t + q + 4 i,
    // packed column c16), Y (packed rows q + 4 i, column 16 t + c16), this
    // lane's part of the diagonal sum of column 16 t + c16 (already contracted
    // with S_3^dag over its packed rows), the close-pair sums in the LDS slots pfc
    CAcc<M3 && T * T <= 4> sacc[PFK ? 1 : T][PFK ? 1 : T];
    CAcc<M3 && T <= 2> pw[PFK ? T : 1];
    v4d yr[PFK ? T : 1], yi[PFK ? T : 1];
    double2 dgl[PFK ? T : 1];
    bool anyc[PFK ? T : 1];
    double2 dsum[T];
#pragma unroll
    for (int t = 0; t < T; ++t) dsum[t] = make_double2(0.0, 0.0);
    if constexpr (PFK) {
#pragma unroll
      for (int t = 0; t < T; ++t) {
        pw[t].zero();
        yr[t] = yi[t] = (v4d){0.0, 0.0, 0.0, 0.0};
        dgl[t] = make_double2(0.0, 0.0);
        anyc[t] = __any(partner[t] >= 0);
        if (anyc[t]) {
#pragma unroll
          for (int i = 0; i < 4; ++i) pfc[(t * 4 + i) * 64 + lane] = make_double2(0.0, 0.0);
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int c = 0; c < T; ++c) sacc[t][c].zero();
    }

    for (int n = n0; n < n1; n += 12) {
      // 0. d_r of the twelve frequencies (the last one of the tile repeated past n1)
#pragma unroll
      for (int it = 0; it < NDT; ++it) {
        const int idx = lane + 64 * it;
        const int f = idx / NBP, r = idx - f * NBP;
        const int nf = min(n + f, n1 - 1);
        const double wn = (double)(2 * nf + 1) * M_PI / beta;
        sh.dtab[f][r] = r < nb ? inv_z_minus(mu, wn, epl[it % NE]) : make_double2(0.0, 0.0);
      }
      // row ri of Sigma of the three frequencies of slot g, for stage 2 (rows
      // past nc read row nc - 1 and are discarded there)
      double2 sgr[3][5];
#pragma unroll
      for (int h = 0; h < 3; ++h) {
        const double2* sp = reinterpret_cast<const double2*>(a.sigma) +
                            (int64_t)min(n + 3 * g + h, n1 - 1) * nc * nc + min(ri, nc - 1) * nc;
#pragma unroll
        for (int j = 0; j < 5; ++j) sgr[h][j] = j < nc ? sp[j] : make_double2(0.0, 0.0);
      }
      wave_sync();
      // 1. X of the four slots, three frequencies per product
      if constexpr (RL == 1) p3_load_x<T>(pt, ps, P, nc, nb, q, c16);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (n + 3 * c >= n1) break;
        const int fa = 3 * c + min(hc, 2);  // frequency of this lane's A row (lane 15: its row is zero)
        CAcc<M3> x;
        x.zero();
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (16 * t + 4 * i >= nb) break;
            const double2 dd = sh.dtab[fa][16 * t + 4 * i + q];
            const double2 a1 = cmul(ps[t][i], dd);
            x.mac_cb(a1.x, a1.y, pt[t][i].x, pt[t][i].y);
          }
        const v4d xr = x.re(), xi = x.im();
#pragma unroll
        for (int i = 0; i < 4; ++i) sh.buf[c][(q + 4 * i) * 17 + c16] = make_double2(xr[i], xi[i]);
      }
      wave_sync();
      // 2. row layout: invert X, subtract Sigma', invert K -> Gl; G_loc partial;
      //    Gl back into the slot's tile, block-diagonally
      // (slots past the tile's end have no X: their lanes skip the stage, which
      // leaves every 16-lane row either wholly active or wholly idle)
      const bool rin = ri < nc;
      const bool slot_ok = n + 3 * g < n1;
#pragma unroll
      for (int h = 0; h < 3; ++h) {
        if (!slot_ok) break;
        const int nf = n + 3 * g + h;
        double rr[5], rim[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          const double2 v = (rin && j < nc) ? sh.buf[g][(5 * h + ri) * 17 + j] : make_double2(0.0, 0.0);
          rr[j] = v.x;
          rim[j] = v.y;
        }
        rsweep<0, 5>(rr, rim, ri, nc, bad);
        // this row of the k-tile's G_loc partial (element (r, j) at (r / 4) 64 +
        // 16 (r % 4) + j), read here so that the load overlaps the second sweep
        const bool rmw = want_x && rin && nf < n1;
        double2* prow = reinterpret_cast<double2*>(a.xpart) +
                        ((int64_t)(a.ktile_base + ktile) * a.nw + min(nf, n1 - 1)) * 256 + (ri >> 2) * 64 +
                        16 * (ri & 3);
        double2 prev[5];
#pragma unroll
        for (int j = 0; j < 5; ++j)
          prev[j] = (rmw && kk != kk0 && j < nc) ? prow[j] : make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          if (j < nc) {
            double2 v = sgr[h][j];
            if (j == ri) v.x -= edc_r;
            rr[j] -= rin ? v.x : 0.0;
            rim[j] -= rin ? v.y : 0.0;
          }
        }
        rsweep<0, 5>(rr, rim, ri, nc, bad);
        if (rmw) {
#pragma unroll
          for (int j = 0; j < 5; ++j)
            if (j < nc) prow[j] = make_double2(wk * rr[j] + prev[j].x, wk * rim[j] + prev[j].y);
        }
        if (ri < 5) {
#pragma unroll
          for (int col = 0; col < 16; ++col) {
            const int j = col - 5 * h;
            const bool in = j >= 0 && j < 5 && rin && j < nc;
            double2 v = make_double2(0.0, 0.0);
#pragma unroll
            for (int jj = 0; jj < 5; ++jj)
              if (jj == j) v = make_double2(rr[jj], rim[jj]);
            sh.buf[g][(5 * h + ri) * 17 + col] = in ? v : make_double2(0.0, 0.0);
          }
        }
      }
      wave_sync();
      // 3. per slot: R, Q, the running sum of G
      if constexpr (RL == 1) p3_load_k<T>(pk, P, hj, aj, nc, nb, c16);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int fb = n + 3 * c;
        if (fb >= n1) break;
        v4d glr, gli;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double2 v = sh.buf[c][(q + 4 * i) * 17 + c16];
          glr[i] = v.x;
          gli[i] = v.y;
        }
        // Sigma' of the slot, block-diagonal: sa[j] = Sigma'[c16][q + 4 j], sb[j] =
        // Sigma'[q + 4 j][c16].  With RL = 1 the positions come from a lane index
        // the compiler cannot see through, from the slot's (uniform) base: hoisted
        // out of the loops they would be kept, or spilled, as one 64-bit offset per
        // load next to the 48-band running sum.
        int lo = lane;
        if constexpr (RL == 1) asm volatile("" : "+v"(lo));
        const int co = lo & 15, qo = lo >> 4;
        const int hco = co / 5, aco = co - 5 * hco;
        const double2* sg = reinterpret_cast<const double2*>(a.sigma) + (int64_t)fb * nc * nc;
        const int fo = (min(fb + hco, n1 - 1) - fb) * nc * nc;
        double sa_r[4], sa_i[4];
        v4d sbr, sbi;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int hjo = (qo + 4 * j) / 5, ajo = qo + 4 * j - 5 * hjo;
          const bool in = hco < 3 && aco < nc && hjo == hco && ajo < nc;
          double2 v = in ? sg[fo + aco * nc + ajo] : make_double2(0.0, 0.0);
          double2 u = in ? sg[fo + ajo * nc + aco] : make_double2(0.0, 0.0);
          if (in && ajo == aco) {
            v.x -= edc_c;
            u.x -= edc_c;
          }
          sa_r[j] = v.x;
          sa_i[j] = v.y;
          sbr[j] = u.x;
          sbi[j] = u.y;
        }
        // V = Gl^T Sigma'^T, R^T = Sigma'^T + Sigma'^T V
        CAcc<M3> va;
        va.zero();
#pragma unroll
        for (int j = 0; j < 4; ++j) va.mac(glr[j], gli[j], sa_r[j], sa_i[j]);
        const v4d vr = va.re(), vi = va.im();
        CAcc<M3> ra;
        ra.set((v4d){sa_r[0], sa_r[1], sa_r[2], sa_r[3]}, (v4d){sa_i[0], sa_i[1], sa_i[2], sa_i[3]});
#pragma unroll
        for (int j = 0; j < 4; ++j) ra.mac(sbr[j], sbi[j], vr[j], vi[j]);
        const v4d rtr = ra.re(), rti = ra.im();
        double chk = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) chk += glr[i] + gli[i] + rtr[i] + rti[i];
        if (!__builtin_isfinite(chk)) nonfinite = 1;
        // d of the slot's frequencies at band 16 t + c16, for contraction slot j
        // (zero for frequencies past the tile's end)
        double2 dk[4][T];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool ok = hj[j] < 3 && fb + hj[j] < n1;
#pragma unroll
          for (int t = 0; t < T; ++t)
            dk[j][t] = ok ? sh.dtab[3 * c + min(hj[j], 2)][16 * t + c16] : make_double2(0.0, 0.0);
        }
        // the D term of sum_n G, added to the diagonal once per k
#pragma unroll
        for (int h = 0; h < 3; ++h) {
          if (fb + h >= n1) break;
#pragma unroll
          for (int t = 0; t < T; ++t) {
            const double2 d = sh.dtab[3 * c + h][16 * t + c16];
            dsum[t].x += d.x;
            dsum[t].y += d.y;
          }
        }
        if constexpr (PFK) {
          // R[q + 4 i][c16] from R^T through the slot's LDS tile, which every
          // lane has read Gl from
          v4d rnr, rni;
          wave_sync();
          tile_transpose(rtr, rti, rnr, rni, sh.buf[c], q, c16);
#pragma unroll
          for (int b = 0; b < T; ++b) {
            // Q = R S_3 for column tile b, row p scaled by d of its frequency:
            // Y += Q, diagonal += S_3^dag Q d, close += Q d(partner)
            CAcc<M3> qa;
            qa.zero();
#pragma unroll
            for (int j = 0; j < 4; ++j) qa.mac(rtr[j], rti[j], pk[j][b].x, pk[j][b].y);
            const v4d xr = qa.re(), xi = qa.im();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const double2 y = cmul(make_double2(xr[i], xi[i]), dk[i][b]);
              yr[b][i] += y.x;
              yi[b][i] += y.y;
              const double2 g = cmul(y, dk[i][b]);
              dgl[b] = cadd(dgl[b], cmul(make_double2(pk[i][b].x, -pk[i][b].y), g));
              if (anyc[b]) {
                const bool ok = partner[b] >= 0 && hj[i] < 3 && fb + hj[i] < n1;
                const double2 dp =
                    ok ? sh.dtab[3 * c + min(hj[i], 2)][max(partner[b], 0)] : make_double2(0.0, 0.0);
                const double2 pp = cmul(y, dp);
                double2* slot = &pfc[(b * 4 + i) * 64 + lane];
                const double2 o = *slot;
                *slot = make_double2(o.x + pp.x, o.y + pp.y);
              }
            }
          }
          // W_t += [D_h S^dag]_h R over the packed index
#pragma unroll
          for (int t = 0; t < T; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const double2 aa = cmul(dk[j][t], make_double2(pk[j][t].x, -pk[j][t].y));
              pw[t].mac(aa.x, aa.y, rnr[j], rni[j]);
            }
        } else if (want_s) {
#pragma unroll
          for (int b = 0; b < T; ++b) {
            // Q = R S_3, row p scaled by d of its frequency at band 16 b + c16
            CAcc<M3> qa;
            qa.zero();
#pragma unroll
            for (int j = 0; j < 4; ++j) qa.mac(rtr[j], rti[j], pk[j][b].x, pk[j][b].y);
            v4d qr = qa.re(), qi = qa.im();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const double2 v = cmul(make_double2(qr[i], qi[i]), dk[i][b]);
              qr[i] = v.x;
              qi[i] = v.y;
            }
            // sum_n G (column tile b) += [D_h S^dag]_h Q
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                const double2 aa = cmul(dk[j][t], make_double2(pk[j][t].x, -pk[j][t].y));
                sacc[t][b].mac(aa.x, aa.y, qr[j], qi[j]);
              }
          }
        }
      }
      wave_sync();
    }  // frequency groups

    if constexpr (PFK) {
      double2* sp = reinterpret_cast<double2*>(a.spart) + (int64_t)wtile * a.s_stride + a.off_s[k];
      // S_3 of the k-point (the frequency loop reloads it per group when RL = 1)
      double2 sk[4][T];
      p3_load_k<T>(sk, P, hj, aj, nc, nb, c16);
      // W through LDS (row v, packed column p' at v * 17 + p'; the slot tiles
      // are free after the last group), read back as the A operand of W S_3
      double2* wl = &sh.buf[0][0];
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const v4d re = pw[t].re(), im = pw[t].im();
#pragma unroll
        for (int i = 0; i < 4; ++i) wl[(16 * t + q + 4 * i) * 17 + c16] = make_double2(re[i], im[i]);
      }
      // the diagonal and the close pair: S_3^dag over the packed rows of this
      // lane (the diagonal is contracted already), then over the four lanes of
      // the column
      double2 dg[T], cl[T];
#pragma unroll
      for (int c = 0; c < T; ++c) {
        dg[c] = dgl[c];
        cl[c] = make_double2(0.0, 0.0);
        const int pv = partner[c];
        if (anyc[c]) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double2 spv = (pv >= 0 && hj[i] < 3) ? lr_proj_here(P, aj[i], pv, nc, nb) : make_double2(0.0, 0.0);
            cl[c] = cadd(cl[c], cmul(make_double2(spv.x, -spv.y), pfc[(c * 4 + i) * 64 + lane]));
          }
        }
#pragma unroll
        for (int off = 16; off <= 32; off <<= 1) {
          dg[c].x += __shfl_xor(dg[c].x, off);
          dg[c].y += __shfl_xor(dg[c].y, off);
          cl[c].x += __shfl_xor(cl[c].x, off);
          cl[c].y += __shfl_xor(cl[c].y, off);
        }
      }
      // Y into the close-pair slots (read), for the B operand of S_3^dag Y
      wave_sync();
#pragma unroll
      for (int c = 0; c < T; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i) pfc[(c * 4 + i) * 64 + lane] = make_double2(yr[c][i], yi[c][i]);
      wave_sync();
      // the tiles in a loop, operands read where they are used (little is live
      // at once at the end of the k-point)
#pragma unroll
      for (int c = 0; c < T; ++c) {
        const int vc = 16 * c + c16;
        const double ec = vc < nb ? eps[vc] : 0.0;
        const int pv = partner[c];
        const double2 dgc = make_double2(dg[c].x + dsum[c].x, dg[c].y + dsum[c].y), clc = cl[c];
#pragma unroll 1
        for (int t = 0; t < T; ++t) {
          // W S_3 - S_3^dag Y for tile (t, c), contraction over the packed index
          CAcc<M3 && T <= 2> acc;
          acc.zero();
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const double2 wv = wl[(16 * t + c16) * 17 + q + 4 * j];
            const double2 sb = hj[j] < 3 ? lr_proj_here(P, aj[j], vc, nc, nb) : make_double2(0.0, 0.0);
            acc.mac(wv.x, wv.y, sb.x, sb.y);
            const double2 st = hj[j] < 3 ? lr_proj_here(P, aj[j], 16 * t + c16, nc, nb) : make_double2(0.0, 0.0);
            const double2 yv = pfc[(c * 4 + j) * 64 + lane];
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
            sp[((t * T + c) * 4 + i) * 64 + lane] = val;
          }
        }
      }
      wave_sync();  // the W tile is the next k-point's slot tiles
    } else if (want_s) {
      double2* sp = reinterpret_cast<double2*>(a.spart) + (int64_t)wtile * a.s_stride + a.off_s[k];
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int c = 0; c < T; ++c)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int e = (t * T + c) * 4 + i;
            double2 v = make_double2(sacc[t][c].re()[i], sacc[t][c].im()[i]);
            if (t == c && hasdiag && idg == i) {
              v.x += dsum[t].x;
              v.y += dsum[t].y;
            }
            sp[e * 64 + lane] = v;
          }
    }
    };
    if (pfk)
      k_body(std::true_type{});
    else
      k_body(std::false_type{});
  }  // k
  if (bad) atomicOr(a.err, ERR_SINGULAR);
  if (nonfinite) atomicOr(a.err, ERR_NONFINITE);
}

}  // namespace dmft

namespace dmft {

// 64-band windows on four wavefronts: the work-group (one per CU, 119 KB of
// LDS) shares one item; each group of 48 frequencies is sixteen slots of
// three.  Wavefront w runs stages 0-2 (d table, X, the inversions, the G_loc
// partial) for slots 4 w .. 4 w + 3 and forms their R in place of Gl; a
// work-group barrier publishes the sixteen R tiles, and then each wavefront
// runs stage 3 for all sixteen slots on its own column tile w of the running
// sum (all four row tiles, three products per complex product, 48 registers).
// Two wavefronts owning two column tiles each would need twice the
// accumulators, which do not fit next to the rest.
struct LRP3QuadShared {
  double2 buf[16][16 * 17];  // per slot: X of its three frequencies, then their Gl, then their R^T
  double2 dtab[48][64];      // d_r of the group's frequencies (zero past nb)
  double2 sproj[5][64];      // S of the k-point (zero outside nc x nb), staged once per k
  double2 sgm[48][25];       // Sigma of the group's frequencies (nc x nc, row stride 5)
};

// Partial-fraction form of the running sum on four wavefronts (the identity of
// lowrank_pair_impl.h: F[v][v'] = ((W S - S^dag Y) / (E_v - E_v'))[v][v'] with
// W = sum_n D_n S^dag R_n and Y = sum_n R_n S D_n, the diagonal and at most one
// close partner per column summed directly).  In the packed index the slot's R
// is block-diagonal, so per slot
//     P = S^dag_w R  (rows: bands of tile w; column p' = 5 h + alpha'),
//     Q = R S_w      (rows p = 5 h + alpha; columns: bands of tile w),
// two products of four steps each in place of the T + T^2 products of Q and
// the running sum, and the frequency of a packed index scales its row (Q) or
// column (P) with d:
//     W[v][p']  += d_h(p')(v) P[v][p'],        Y[p][v'] += d_h(p)(v') Q[p][v'],
//     diag[p][v'] += d^2 Q[p][v'],             close[p][v'] += d(partner) d Q[p][v'].
// W and Y keep the three frequencies of a slot in their own blocks of the
// packed index; the products W S_3 and S_3^dag Y over the packed index at the
// end of the k-point add them up (S_3[5 h + beta][v] = S[beta][v]).

// Close partner of the owned column vc; whether the partial-fraction form
// applies to the k-point (every column of the work-group has at most one).
__device__ __forceinline__ bool p3q_pairs(const double* eps, int nb, int vc, double beta, int& partner) {
  const double delta = M_PI / (16.0 * beta);
  const double ec = vc < nb ? eps[vc] : 0.0;
  int cnt = 0, pv = -1;
  for (int v = 0; v < nb; ++v) {
    const bool close = vc < nb && v != vc && __builtin_fabs(eps[v] - ec) < delta;
    pv = close ? v : pv;
    cnt += close ? 1 : 0;
  }
  partner = pv;
  return !__syncthreads_or(cnt > 1);
}

// One slot (three frequencies, the first fb) of the partial-fraction sums of
// wavefront w.  Register map (re, im):
//   W, rows 16 w + q + 4 i, column c16           s1[0], s1[1]
//   Y, rows q + 4 i, column 16 w + c16           s1[2], s1[3]
//   diagonal sums (same layout as Y)             s2[0], s2[1]
//   close-pair sums (same layout as Y)           s2[2], s2[3]
// rtr/rti: R[c16][q + 4 i] of the slot; pw[j] = S[alpha_j][16 w + c16] for the
// packed index q + 4 j (zero for p = 15).
template <class Shared>
__device__ __forceinline__ void p3q_pf_step(v4d (&s1)[4], v4d (&s2)[4], const v4d& rtr, const v4d& rti,
                                            const Shared& sh, const double2 (&pw)[4], const int (&hj)[4], int s,
                                            int fb, int n1, int partner, int w, int q, int c16, double2& dsum) {
  const int vc = 16 * w + c16;
  const int hc = c16 / 5;
  v4d rnr, rni;  // R[q + 4 i][c16], read transposed from the tile that holds R^T
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 v = sh.buf[s][c16 * 17 + q + 4 * i];
    rnr[i] = v.x;
    rni[i] = v.y;
  }
  // the D term of the owned column
#pragma unroll
  for (int h = 0; h < 3; ++h) {
    if (fb + h >= n1) break;
    const double2 d = sh.dtab[3 * s + h][vc];
    dsum.x += d.x;
    dsum.y += d.y;
  }
  CAcc<true> qa, pa;
  qa.zero();
  pa.zero();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    qa.mac(rtr[j], rti[j], pw[j].x, pw[j].y);
    pa.mac(pw[j].x, -pw[j].y, rnr[j], rni[j]);
  }
  const v4d xr = qa.re(), xi = qa.im();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int h = hj[i];
    const bool ok = h < 3 && fb + h < n1;
    const int row = 3 * s + (h < 3 ? h : 2);
    const double2 d = ok ? sh.dtab[row][vc] : make_double2(0.0, 0.0);
    const double2 dp = (ok && partner >= 0) ? sh.dtab[row][partner] : make_double2(0.0, 0.0);
    const double2 y = cmul(make_double2(xr[i], xi[i]), d);
    s1[2][i] += y.x;
    s1[3][i] += y.y;
    const double2 g = cmul(y, d), c = cmul(y, dp);
    s2[0][i] += g.x;
    s2[1][i] += g.y;
    s2[2][i] += c.x;
    s2[3][i] += c.y;
  }
  const v4d pr = pa.re(), pi = pa.im();
  const bool okc = hc < 3 && fb + hc < n1;
  const int rowc = 3 * s + (hc < 3 ? hc : 2);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 dv = okc ? sh.dtab[rowc][16 * w + q + 4 * i] : make_double2(0.0, 0.0);
    const double2 x = cmul(make_double2(pr[i], pi[i]), dv);
    s1[0][i] += x.x;
    s1[1][i] += x.y;
  }
}

// End of a k-point: W of the four wavefronts through LDS, then for the owned
// column tile w and every row tile F = (W S_3 - S_3^dag Y) / (E_v - E_v'), the
// diagonal and the close pair from their direct sums, plus the D term on the
// diagonal; stored in the running sum's partial layout.
template <class Shared>
__device__ __forceinline__ void p3q_pf_finish(const v4d (&s1)[4], const v4d (&s2)[4], const double2& dsum,
                                              Shared& sh, const double* eps, int nb, int partner, double2* sp, int w,
                                              int q, int c16, const int (&hj)[4], const int (&aj)[4], int tid) {
  constexpr int T = 4;
  const int vc = 16 * w + c16;
  // the frequency loop ended with a work-group barrier: the slot tiles are free
  double2* wl = &sh.buf[0][0];  // W[v][p'] at v * 17 + p' (64 x 17 < 16 x 16 x 17)
#pragma unroll
  for (int i = 0; i < 4; ++i) wl[(16 * w + q + 4 * i) * 17 + c16] = make_double2(s1[0][i], s1[1][i]);
  __syncthreads();
  double2 pw[4];  // S_3[q + 4 j][vc]
#pragma unroll
  for (int j = 0; j < 4; ++j) pw[j] = hj[j] < 3 ? sh.sproj[aj[j]][vc] : make_double2(0.0, 0.0);
  // the diagonal and the close pair: S^dag contracted over the packed rows of
  // this lane, then over the four lanes of the column
  double2 dg = make_double2(0.0, 0.0), cl = make_double2(0.0, 0.0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 sq = (hj[i] < 3 && partner >= 0) ? sh.sproj[aj[i]][partner] : make_double2(0.0, 0.0);
    dg = cadd(dg, cmul(make_double2(pw[i].x, -pw[i].y), make_double2(s2[0][i], s2[1][i])));
    cl = cadd(cl, cmul(make_double2(sq.x, -sq.y), make_double2(s2[2][i], s2[3][i])));
  }
#pragma unroll
  for (int off = 16; off <= 32; off <<= 1) {
    dg.x += __shfl_xor(dg.x, off);
    dg.y += __shfl_xor(dg.y, off);
    cl.x += __shfl_xor(cl.x, off);
    cl.y += __shfl_xor(cl.y, off);
  }
  const double ec = vc < nb ? eps[vc] : 0.0;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    CAcc<true> acc;
    acc.zero();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double2 wv = wl[(16 * t + c16) * 17 + q + 4 * j];  // W[16 t + c16][q + 4 j]
      acc.mac(wv.x, wv.y, pw[j].x, pw[j].y);
      const double2 st = hj[j] < 3 ? sh.sproj[aj[j]][16 * t + c16] : make_double2(0.0, 0.0);
      acc.mac(-st.x, st.y, s1[2][j], s1[3][j]);  // - S_3^dag Y
    }
    const v4d fr = acc.re(), fi = acc.im();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int v = 16 * t + q + 4 * i;
      double2 val;
      if (v == vc) {
        val = make_double2(dg.x + dsum.x, dg.y + dsum.y);
      } else if (v == partner) {
        val = cl;
      } else {
        const double ev = v < nb ? eps[v] : 0.0;
        const double inv = (v < nb && vc < nb) ? 1.0 / (ev - ec) : 0.0;
        val = make_double2(fr[i] * inv, fi[i] * inv);
      }
      sp[((t * T + w) * 4 + i) * 64 + (tid & 63)] = val;
    }
  }
  __syncthreads();  // the W tile is the next k-point's slot tiles
}

template <bool PF = false>
__device__ __forceinline__ void lr_p3_quad_tile(const DysonArgs& a, int ktile, int wtile, LRP3QuadShared& sh,
                                                int tid) {
  constexpr int T = 4;
  const int w = tid >> 6, lane = tid & 63;
  const int q = lane >> 4, c16 = lane & 15;
  const int n0 = wtile * a.wt;
  const int n1 = min(n0 + a.wt, a.nw);
  const int kk0 = ktile * a.kt;
  const int kk1 = min(kk0 + a.kt, a.nklist);
  const double mu = uniform_d(a.mu_ptr ? *a.mu_ptr : a.mu);
  const int nc = a.nc;
  // the dispatchers take this kernel for nc <= 5 only
  __builtin_assume(nc >= 1 && nc <= 5);
  const double beta = a.beta;
  const bool want_s = (a.mode & MODE_S) != 0;
  const bool want_x = (a.mode & MODE_GLOC) != 0;
  const bool hasdiag = c16 >= q && ((c16 - q) & 3) == 0;
  const int idg = (c16 - q) >> 2;
  const int hc = c16 / 5;
  const int ac = c16 - 5 * hc;
  const bool cin = hc < 3 && ac < nc;
  int hj[4], aj[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    hj[j] = (q + 4 * j) / 5;
    aj[j] = q + 4 * j - 5 * hj[j];
  }
  const double edc_c = cin ? a.e_dc[ac] : 0.0;
  const double edc_r = c16 < nc ? a.e_dc[c16] : 0.0;
  int bad = 0, nonfinite = 0;

  for (int kk = kk0; kk < kk1; ++kk) {
    const int k = uniform_i(a.klist ? a.klist[kk] : kk);
    const int nb = uniform_i(a.nb_uniform > 0 ? a.nb_uniform : a.nb[k]);
    // every k of a 64-band bucket has 48 < nb <= 64 (checked on the host)
    __builtin_assume(nb > 48 && nb <= 64);
    const int64_t ob = uniform_l(a.nb_uniform > 0 ? (int64_t)k * nb : a.off_b[k]);
    const double el = lane < nb ? a.eps[ob + lane] : 0.0;
    const double2* P = reinterpret_cast<const double2*>(a.proj) + ob * nc;
    const double wk = uniform_d(a.wk[k]);
    // the projector into LDS: every fragment of the k is read from there, with
    // LDS latency (the previous k, or item, ended with a work-group barrier)
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int e = tid + 256 * m;
      if (e < 5 * 64) {
        const int al = e >> 6, r = e & 63;
        sh.sproj[al][r] = lr_proj(P, al, r, nc, nb);
      }
    }
    __syncthreads();
    // partial-fraction form: the close partner (if any) of the owned column, and
    // whether every column of the work-group has at most one
    int partner = -1;
    bool pfk = false;
    if constexpr (PF) pfk = p3q_pairs(a.eps + ob, nb, 16 * w + c16, beta, partner);
    // one k-point, with the running sum in the direct (PFK false) or the
    // partial-fraction form; the two instantiations keep separate registers
    auto k_body = [&](auto pf_tag) {
    constexpr bool PFK = decltype(pf_tag)::value;
    // direct form: the owned column tile of sum_n G, all four row tiles (three
    // products); partial-fraction form: see p3q_pf_step
    v4d s1[T], s2[T], s3[T];
#pragma unroll
    for (int t = 0; t < T; ++t) s1[t] = s2[t] = s3[t] = (v4d){0.0, 0.0, 0.0, 0.0};
    double2 dsum = make_double2(0.0, 0.0);

    for (int n = n0; n < n1; n += 48) {
      // ---- 0. d table of this wavefront's twelve frequencies (band = lane)
      const int nw0 = n + 12 * w;
#pragma unroll
      for (int f = 0; f < 12; ++f) {
        const int nf = min(nw0 + f, n1 - 1);
        const double wn = (double)(2 * nf + 1) * M_PI / beta;
        sh.dtab[12 * w + f][lane] = lane < nb ? inv_z_minus(mu, wn, el) : make_double2(0.0, 0.0);
      }
      const int g = q, ri = c16;  // row layout: this wavefront's slot g, row ri
      const int sl = 4 * w + g;   // slot in the group
      // Sigma of the wavefront's twelve frequencies (12 x 25 positions, five per
      // lane): loaded now, stored to LDS after the X products hide the latency
      double2 sgl[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const int e = lane + 64 * m;
        const int f = e / 25, rem = e - 25 * f, ra = rem / 5, cb = rem - 5 * ra;
        const int nf = min(nw0 + f, n1 - 1);
        sgl[m] = (ra < nc && cb < nc)
                     ? reinterpret_cast<const double2*>(a.sigma)[(int64_t)nf * nc * nc + ra * nc + cb]
                     : make_double2(0.0, 0.0);
      }
      wave_sync();
      // ---- 1. X of this wavefront's four slots
      {
        double2 pt[T][4], ps[T][4];
#pragma unroll
        for (int t2 = 0; t2 < T; ++t2)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = 16 * t2 + 4 * i + q;
            pt[t2][i] = c16 < 5 ? sh.sproj[c16][r] : make_double2(0.0, 0.0);
            ps[t2][i] = c16 < 15 ? sh.sproj[ac][r] : make_double2(0.0, 0.0);
          }
#pragma unroll 1
        for (int c = 0; c < 4; ++c) {
          const int s = 4 * w + c;
          if (n + 3 * s >= n1) break;
          const int fa = 3 * s + min(hc, 2);
          CAcc<true> x;
          x.zero();
#pragma unroll
          for (int t = 0; t < T; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              if (16 * t + 4 * i >= nb) break;
              const double2 dd = sh.dtab[fa][16 * t + 4 * i + q];
              const double2 a1 = cmul(ps[t][i], dd);
              x.mac_cb(a1.x, a1.y, pt[t][i].x, pt[t][i].y);
            }
          const v4d xr = x.re(), xi = x.im();
#pragma unroll
          for (int i = 0; i < 4; ++i) sh.buf[s][(q + 4 * i) * 17 + c16] = make_double2(xr[i], xi[i]);
        }
      }
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const int e = lane + 64 * m;
        const int f = e / 25, rem = e - 25 * f;
        sh.sgm[12 * w + f][rem] = sgl[m];
      }
      wave_sync();
      // ---- 2. row layout, three sub-sweeps per slot
      {
        const bool rin = ri < nc;
        const bool slot_ok = n + 3 * sl < n1;
#pragma unroll
        for (int h = 0; h < 3; ++h) {
          if (!slot_ok) break;
          const int nf = n + 3 * sl + h;
          double rr[5], rim[5];
#pragma unroll
          for (int j = 0; j < 5; ++j) {
            const double2 v = (rin && j < nc) ? sh.buf[sl][(5 * h + ri) * 17 + j] : make_double2(0.0, 0.0);
            rr[j] = v.x;
            rim[j] = v.y;
          }
          rsweep<0, 5>(rr, rim, ri, nc, bad);
          const bool rmw = want_x && rin && nf < n1;
          double2* prow = reinterpret_cast<double2*>(a.xpart) +
                          ((int64_t)(a.ktile_base + ktile) * a.nw + min(nf, n1 - 1)) * 256 + (ri >> 2) * 64 +
                          16 * (ri & 3);
          double2 prev[5];
#pragma unroll
          for (int j = 0; j < 5; ++j)
            prev[j] = (rmw && kk != kk0 && j < nc) ? prow[j] : make_double2(0.0, 0.0);
#pragma unroll
          for (int j = 0; j < 5; ++j) {
            if (j < nc) {
              double2 v = rin ? sh.sgm[3 * sl + h][ri * 5 + j] : make_double2(0.0, 0.0);
              if (j == ri) v.x -= edc_r;
              rr[j] -= rin ? v.x : 0.0;
              rim[j] -= rin ? v.y : 0.0;
            }
          }
          rsweep<0, 5>(rr, rim, ri, nc, bad);
          if (rmw) {
#pragma unroll
            for (int j = 0; j < 5; ++j)
              if (j < nc) prow[j] = make_double2(wk * rr[j] + prev[j].x, wk * rim[j] + prev[j].y);
          }
          if (ri < 5) {
#pragma unroll
            for (int col = 0; col < 16; ++col) {
              const int j = col - 5 * h;
              const bool in = j >= 0 && j < 5 && rin && j < nc;
              double2 v = make_double2(0.0, 0.0);
#pragma unroll
              for (int jj = 0; jj < 5; ++jj)
                if (jj == j) v = make_double2(rr[jj], rim[jj]);
              sh.buf[sl][(5 * h + ri) * 17 + col] = in ? v : make_double2(0.0, 0.0);
            }
          }
        }
      }
      wave_sync();
      // ---- 2b. R of this wavefront's four slots, in the output layout, in place of Gl
#pragma unroll 1
      for (int c = 0; c < 4; ++c) {
        const int s = 4 * w + c;
        const int fb = n + 3 * s;
        if (fb >= n1) break;
        v4d glr, gli;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double2 v = sh.buf[s][(q + 4 * i) * 17 + c16];
          glr[i] = v.x;
          gli[i] = v.y;
        }
        const double2* sg = sh.sgm[3 * s + min(hc, 2)];  // this lane's frequency of the slot
        double sa_r[4], sa_i[4];
        v4d sbr, sbi;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool in = cin && hj[j] == hc && aj[j] < nc;
          double2 v = in ? sg[ac * 5 + aj[j]] : make_double2(0.0, 0.0);
          double2 u = in ? sg[aj[j] * 5 + ac] : make_double2(0.0, 0.0);
          if (in && aj[j] == ac) {
            v.x -= edc_c;
            u.x -= edc_c;
          }
          sa_r[j] = v.x;
          sa_i[j] = v.y;
          sbr[j] = u.x;
          sbi[j] = u.y;
        }
        CAcc<true> va;
        va.zero();
#pragma unroll
        for (int j = 0; j < 4; ++j) va.mac(glr[j], gli[j], sa_r[j], sa_i[j]);
        const v4d vr = va.re(), vi = va.im();
        CAcc<true> ra;
        ra.set((v4d){sa_r[0], sa_r[1], sa_r[2], sa_r[3]}, (v4d){sa_i[0], sa_i[1], sa_i[2], sa_i[3]});
#pragma unroll
        for (int j = 0; j < 4; ++j) ra.mac(sbr[j], sbi[j], vr[j], vi[j]);
        const v4d rtr = ra.re(), rti = ra.im();
        double chk = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) chk += glr[i] + gli[i] + rtr[i] + rti[i];
        if (!__builtin_isfinite(chk)) nonfinite = 1;
        // each lane overwrites only the elements it has read
#pragma unroll
        for (int i = 0; i < 4; ++i) sh.buf[s][(q + 4 * i) * 17 + c16] = make_double2(rtr[i], rti[i]);
      }
      __syncthreads();
      // ---- 3. all sixteen slots: the owned column tile w of sum_n G
      double2 pk[4][T], pw[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int t2 = 0; t2 < T; ++t2)
          pk[j][t2] = hj[j] < 3 ? sh.sproj[aj[j]][16 * t2 + c16] : make_double2(0.0, 0.0);
        pw[j] = hj[j] < 3 ? sh.sproj[aj[j]][16 * w + c16] : make_double2(0.0, 0.0);
      }
#pragma unroll 1
      for (int s = 0; s < 16; ++s) {
        const int fb = n + 3 * s;
        if (fb >= n1) break;
        v4d rtr, rti;  // R^T of the slot (R[c16][q + 4 i])
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double2 v = sh.buf[s][(q + 4 * i) * 17 + c16];
          rtr[i] = v.x;
          rti[i] = v.y;
        }
        if (!want_s) continue;
        if constexpr (PFK) {
          p3q_pf_step(s1, s2, rtr, rti, sh, pw, hj, s, fb, n1, partner, w, q, c16, dsum);
          continue;
        }
        // d of the slot's frequency of contraction slot j at band 16 t + c16 is
        // read from the table where it is used (zero for frequencies past the
        // tile's end), which keeps it out of the registers
        bool jok[4];
        int jrow[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          jok[j] = hj[j] < 3 && fb + hj[j] < n1;
          jrow[j] = 3 * s + min(hj[j], 2);
        }
        auto dkv = [&](int j, int t) -> double2 {
          return jok[j] ? sh.dtab[jrow[j]][16 * t + c16] : make_double2(0.0, 0.0);
        };
        // the D term of the owned column tile
#pragma unroll
        for (int h = 0; h < 3; ++h) {
          if (fb + h >= n1) break;
          const double2 d = sh.dtab[3 * s + h][16 * w + c16];
          dsum.x += d.x;
          dsum.y += d.y;
        }
        // Q_w = R S_3 for the owned column tile, rows scaled by d of their frequency
        double qr[4], qi[4], qs[4];
        {
          CAcc<true> qa;
          qa.zero();
#pragma unroll
          for (int j = 0; j < 4; ++j) qa.mac(rtr[j], rti[j], pw[j].x, pw[j].y);
          const v4d xr = qa.re(), xi = qa.im();
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double2 v = cmul(make_double2(xr[i], xi[i]), dkv(i, w));
            qr[i] = v.x;
            qi[i] = v.y;
            qs[i] = v.x + v.y;
          }
        }
        // sum_n G[t][w] += [D_h S^dag]_h Q_w, contraction over the packed index
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int t = 0; t < T; ++t) {
            const double2 aa = cmul(dkv(j, t), make_double2(pk[j][t].x, -pk[j][t].y));
            mac3(s1[t], s2[t], s3[t], aa.x, aa.y, aa.x + aa.y, qr[j], qi[j], qs[j]);
          }
      }
      __syncthreads();
    }  // frequency groups

    if (want_s && PFK) {
      double2* sp = reinterpret_cast<double2*>(a.spart) + (int64_t)wtile * a.s_stride + a.off_s[k];
      p3q_pf_finish(s1, s2, dsum, sh, a.eps + ob, nb, partner, sp, w, q, c16, hj, aj, tid);
    } else if (want_s) {
      double2* sp = reinterpret_cast<double2*>(a.spart) + (int64_t)wtile * a.s_stride + a.off_s[k];
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const v4d re = s1[t] - s2[t], im = s3[t] - s1[t] - s2[t];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = (t * T + w) * 4 + i;  // address only: no register indexed by w
          double2 v = make_double2(re[i], im[i]);
          if (t == w && hasdiag && idg == i) {
            v.x += dsum.x;
            v.y += dsum.y;
          }
          sp[e * 64 + lane] = v;
        }
      }
    }
    };
    if (pfk)
      k_body(std::true_type{});
    else
      k_body(std::false_type{});
  }  // k
  if (bad) atomicOr(a.err, ERR_SINGULAR);
  if (nonfinite) atomicOr(a.err, ERR_NONFINITE);
}

}  // namespace dmft
