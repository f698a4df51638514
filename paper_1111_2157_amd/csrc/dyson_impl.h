// Device code of the lattice Dyson kernel (gfx950 / CDNA4), included by the
// per-size instantiation units dyson_16.hip, dyson_32.hip, dyson_48.hip.
//
// One wavefront owns one (k, i w_n) matrix at a time and walks a tile of
// frequencies for each k of its k-tile.  The band-window matrix lives in
// registers in the output layout of the FP64 matrix-core instruction
// v_mfma_f64_16x16x4: for a padded size NBP = 16 T, lane l = 16 q + c16
// holds, in register (t, b, i) of tile (t, b), the element
//
//     row = 16 t + 4 i + q ,   column = 16 b + c16 .
//
// Per frequency:
//   1. embed:  V = (Sigma - V_DC) S          (matrix cores, nc padded to 16)
//              A = (i w + mu) I - diag(E) - S^dag V   (matrix cores; the
//              product lands directly in the register layout above)
//   2. invert: in-place Gauss-Jordan without pivoting on the FP64 vector
//              ALUs.  A is accretive (its anti-Hermitian part is at least
//              w_n I for a causal Sigma), so every leading block is
//              invertible and no row exchange is needed.  Pivot row, column
//              and pivot are broadcast through LDS; the row and column of the
//              next step are updated first and published before the bulk of
//              the current update, so their LDS round trip overlaps it.
//   3. accumulate sum_n G (density) or Re tr G, Re tr G^2 (mu search);
//   4. project: W^T = G^T S^T and X = W S^dag = S G S^dag on the matrix
//              cores, straight from the registers of step 2; w_k X is added
//              to a per-(k tile, n) partial of G_loc.
// Reductions over frequency tiles and k tiles run in fixed order in separate
// kernels, so results are bitwise reproducible.
//
// Variants (template parameters, chosen by the autotuner):
//   PF   = 1: the whole next-step broadcast (pivot column, row, pivot) is read
//             into a second register set during the current update;
//          0: only the pivot row and pivot are read ahead, the pivot column
//             is read at the start of its step (fewer live registers);
//   SLDS = 1: the running frequency sum of G is kept in LDS, 0: in registers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dmft_internal.h"

namespace dmft {

typedef double v4d __attribute__((ext_vector_type(4)));

// D += a*b and D -= a*b on the 16x16x4 FP64 matrix core (a, b: one element per lane).
__device__ __forceinline__ v4d mma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4d mms(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 1);  // neg(a)
}

// Orders LDS traffic between lanes of one wavefront: LDS instructions of a
// wavefront execute in issue order, so only the compiler has to be kept from
// moving accesses across this point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// 1/p for complex p: one hardware reciprocal of |p|^2 refined by two Newton steps.
__device__ __forceinline__ double2 crecip(double2 p) {
  double d = p.x * p.x + p.y * p.y;
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  return make_double2(p.x * r, -p.y * r);
}

template <int NBP>
struct Mat {
  static constexpr int T = NBP / 16;
  v4d re[T][T], im[T][T];
};

template <int NBP>
struct RowB {
  static constexpr int T = NBP / 16;
  double2 rv[T];  // pivot-row entries of this lane's columns
  double2 p;      // pivot
};

template <int NBP>
struct ColB {
  static constexpr int T = NBP / 16;
  double2 cc[T][4];  // pivot-column entries of this lane's rows
};

template <int NBP>
struct GJShared {
  double2 col[2][NBP];
  double2 row[2][NBP];
  double2 piv[2];
};

// g -= cc * rs for the element (register i) of one tile.
__device__ __forceinline__ void upd(v4d& gr, v4d& gi, int i, double2 cc, double2 rs) {
  double r = gr[i], m = gi[i];
  r = __builtin_fma(-cc.x, rs.x, r);
  r = __builtin_fma(cc.y, rs.y, r);
  m = __builtin_fma(-cc.x, rs.y, m);
  m = __builtin_fma(-cc.y, rs.x, m);
  gr[i] = r;
  gi[i] = m;
}

// Publish column K and row K of the current matrix with the in-place
// Gauss-Jordan bookkeeping (column entry at the pivot minus 1, row entry at
// the pivot plus 1, so that one uniform rank-1 update also produces the new
// pivot row and column), and the pivot itself.
template <int NBP, int K>
__device__ __forceinline__ void gj_publish(const Mat<NBP>& g, GJShared<NBP>& sh, int q, int c16) {
  constexpr int T = NBP / 16;
  constexpr int tk = K >> 4, ik = (K >> 2) & 3, qk = K & 3, bk = K >> 4, ck = K & 15, s = K & 1;
  if (c16 == ck) {
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double2 v = make_double2(g.re[t][bk][i], g.im[t][bk][i]);
        if (t == tk && i == ik && q == qk) v.x -= 1.0;
        sh.col[s][16 * t + 4 * i + q] = v;
      }
  }
  if (q == qk) {
#pragma unroll
    for (int b = 0; b < T; ++b) {
      double2 v = make_double2(g.re[tk][b][ik], g.im[tk][b][ik]);
      if (b == bk && c16 == ck) v.x += 1.0;
      sh.row[s][16 * b + c16] = v;
    }
    if (c16 == ck) sh.piv[s] = make_double2(g.re[tk][bk][ik], g.im[tk][bk][ik]);
  }
}

template <int NBP, int K>
__device__ __forceinline__ void fetch_row(RowB<NBP>& rb, const GJShared<NBP>& sh, int c16) {
  constexpr int T = NBP / 16, s = K & 1;
#pragma unroll
  for (int b = 0; b < T; ++b) rb.rv[b] = sh.row[s][16 * b + c16];
  rb.p = sh.piv[s];
}

template <int NBP, int K>
__device__ __forceinline__ void fetch_col(ColB<NBP>& cb, const GJShared<NBP>& sh, int q) {
  constexpr int T = NBP / 16, s = K & 1;
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) cb.cc[t][i] = sh.col[s][16 * t + 4 * i + q];
}

// Gauss-Jordan step K, then (recursively) the remaining steps.  On entry `rb`
// holds step K's pivot row and pivot, and with PF also `cb` its pivot column.
template <int NBP, int PF, int K>
__device__ __forceinline__ void gj_steps(Mat<NBP>& g, RowB<NBP>& rb, ColB<NBP>& cb, GJShared<NBP>& sh, int q,
                                         int c16, int nb, int& bad) {
  if constexpr (K < NBP) {
    if (K >= nb) return;
    constexpr int T = NBP / 16;
    if constexpr (!PF) fetch_col<NBP, K>(cb, sh, q);
    double2 ip = crecip(rb.p);
    bad |= (rb.p.x == 0.0 && rb.p.y == 0.0);
    double2 rs[T];
#pragma unroll
    for (int b = 0; b < T; ++b) rs[b] = cmul(rb.rv[b], ip);
    if constexpr (K + 1 < NBP) {
      constexpr int K1 = K + 1, t1 = K1 >> 4, i1 = (K1 >> 2) & 3, b1 = K1 >> 4;
      // the pivot column and row of step K+1 first, published before the bulk update
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) upd(g.re[t][b1], g.im[t][b1], i, cb.cc[t][i], rs[b1]);
#pragma unroll
      for (int b = 0; b < T; ++b)
        if (b != b1) upd(g.re[t1][b], g.im[t1][b], i1, cb.cc[t1][i1], rs[b]);
      gj_publish<NBP, K1>(g, sh, q, c16);
      wave_sync();
      RowB<NBP> rn;
      fetch_row<NBP, K1>(rn, sh, c16);
      ColB<NBP> cn;
      if constexpr (PF) fetch_col<NBP, K1>(cn, sh, q);
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int b = 0; b < T; ++b) {
          if (b == b1) continue;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (t == t1 && i == i1) continue;
            upd(g.re[t][b], g.im[t][b], i, cb.cc[t][i], rs[b]);
          }
        }
      wave_sync();
      if constexpr (PF)
        gj_steps<NBP, PF, K + 1>(g, rn, cn, sh, q, c16, nb, bad);
      else
        gj_steps<NBP, PF, K + 1>(g, rn, cb, sh, q, c16, nb, bad);
    } else {
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int b = 0; b < T; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) upd(g.re[t][b], g.im[t][b], i, cb.cc[t][i], rs[b]);
    }
  }
}

template <int NBP, int PF>
__device__ __forceinline__ void gauss_jordan(Mat<NBP>& g, GJShared<NBP>& sh, int q, int c16, int nb, int& bad) {
  RowB<NBP> rb;
  ColB<NBP> cb;
  gj_publish<NBP, 0>(g, sh, q, c16);
  wave_sync();
  fetch_row<NBP, 0>(rb, sh, c16);
  if constexpr (PF) fetch_col<NBP, 0>(cb, sh, q);
  gj_steps<NBP, PF, 0>(g, rb, cb, sh, q, c16, nb, bad);
  wave_sync();
}

// Per-k projector fragments (see the layout note at the top of the file).
template <int NBP>
struct Proj {
  static constexpr int T = NBP / 16;
  double pa_r[4][T], pa_i[4][T];  // S[q + 4 i][16 b + c16]
  double pt_r[T][4], pt_i[T][4];  // S[c16][16 t + 4 i + q]
};

// Returns p unchanged but hides its value from the optimizer, so that loads
// through the result stay where they are written: they are neither merged
// with earlier loads of the same address nor hoisted out of a loop.  Unlike
// volatile accesses, such loads are ordinary cached loads that the compiler
// may still issue back to back and wait for together.
template <class T>
__device__ __forceinline__ const T* fresh(const T* p) {
  asm volatile("" : "+v"(p));
  return p;
}

// A value the caller knows to be the same in every lane, moved to scalar
// registers (the compiler cannot prove it for values loaded through a generic
// pointer, and keeps such values in vector registers otherwise).
__device__ __forceinline__ double uniform_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t uniform_l(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Projector fragments are re-read (from L1/L2) where they are used, so that they
// do not occupy registers during the Gauss-Jordan sweep.  The volatile access
// also pins each load to its place in the program order (each one is waited
// for before the next), which keeps the live ranges short in the kernels that
// are tightest on registers.
__device__ __forceinline__ double2 ld_proj(const double2* P, int al, int bd, int nc, int nb) {
  double2 v = make_double2(0.0, 0.0);
  if (al < nc && bd < nb) {
    const volatile double* pv = reinterpret_cast<const volatile double*>(P + al * nb + bd);
    v.x = pv[0];
    v.y = pv[1];
  }
  return v;
}

template <int NBP>
__device__ __forceinline__ void load_pa(Proj<NBP>& pr, const double2* P, int nc, int nb, int q, int c16) {
  constexpr int T = NBP / 16;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int b = 0; b < T; ++b) {
      double2 v = ld_proj(P, q + 4 * i, 16 * b + c16, nc, nb);
      pr.pa_r[i][b] = v.x;
      pr.pa_i[i][b] = v.y;
    }
}

template <int NBP>
__device__ __forceinline__ void load_pt(Proj<NBP>& pr, const double2* P, int nc, int nb, int q, int c16) {
  constexpr int T = NBP / 16;
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double2 v = ld_proj(P, c16, 16 * t + 4 * i + q, nc, nb);
      pr.pt_r[t][i] = v.x;
      pr.pt_i[t][i] = v.y;
    }
}

// KIND_ADJ (fused scalar adjoint of N_tot) and KIND_GEN (general
// vector-Jacobian product) exist in the low-rank form only; the dense form of
// both is adjoint.hip.
enum { KIND_DENSITY = 0, KIND_TRACE = 1, KIND_ADJ = 2, KIND_GEN = 3 };

template <int NBP, int KIND, int SLDS>
struct KernelShared {
  static constexpr int T = NBP / 16;
  GJShared<NBP> gj;
  double2 tr[KIND == KIND_TRACE ? 16 * 17 : 1];  // 16x16 tile transpose
  double2 s[SLDS ? T * T * 4 * 64 : 1];          // running sum of G (lane order)
};

// A = (i w + mu) I - diag(E) - S^dag (Sigma - V_DC) S for frequency n, built on the matrix cores.
template <int NBP>
__device__ __forceinline__ void build_a(Mat<NBP>& g, const DysonArgs& a, const double2* P, int nb, int n, double wn,
                                        const double* dre, const bool* dval, bool hasdiag, int idg, int q,
                                        int c16) {
  constexpr int T = NBP / 16;
  const int nc = a.nc;
  Proj<NBP> pr;
  load_pa<NBP>(pr, P, nc, nb, q, c16);
  // (Sigma - V_DC) fragments: lane holds Sigma'[c16][q + 4 j]
  const double2* sg = reinterpret_cast<const double2*>(a.sigma) + (int64_t)n * nc * nc;
  double sa_r[4], sa_i[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int be = q + 4 * j;
    double2 v = (c16 < nc && be < nc) ? sg[c16 * nc + be] : make_double2(0.0, 0.0);
    if (c16 == be && c16 < nc) v.x -= a.e_dc[c16];
    sa_r[j] = v.x;
    sa_i[j] = v.y;
  }
  // V = Sigma' S  (16 x NBP); chunk j holds orbitals q + 4 j, so chunks with
  // 4 j >= nc are all padding and are skipped (uniform branch)
  const int kc = (nc + 3) >> 2;
  v4d vr[T], vi[T];
#pragma unroll
  for (int b = 0; b < T; ++b) {
    vr[b] = vi[b] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j >= kc) break;
      vr[b] = mma(sa_r[j], pr.pa_r[j][b], vr[b]);
      vr[b] = mms(sa_i[j], pr.pa_i[j][b], vr[b]);
      vi[b] = mma(sa_r[j], pr.pa_i[j][b], vi[b]);
      vi[b] = mma(sa_i[j], pr.pa_r[j][b], vi[b]);
    }
  }
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int b = 0; b < T; ++b) {
      v4d zr = {0.0, 0.0, 0.0, 0.0}, zi = {0.0, 0.0, 0.0, 0.0};
      if (t == b) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          bool on = hasdiag && idg == i;
          zr[i] = on ? dre[t] : 0.0;
          zi[i] = (on && dval[t]) ? wn : 0.0;
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i >= kc) break;
        zr = mms(pr.pa_r[i][t], vr[b][i], zr);
        zr = mms(pr.pa_i[i][t], vi[b][i], zr);
        zi = mms(pr.pa_r[i][t], vi[b][i], zi);
        zi = mma(pr.pa_i[i][t], vr[b][i], zi);
      }
      g.re[t][b] = zr;
      g.im[t][b] = zi;
    }
}

// One (k-tile, frequency-tile) work item on one wavefront (lane = 0..63).
template <int NBP, int KIND, int PF, int SLDS>
__device__ __forceinline__ void dyson_tile(const DysonArgs& a, int ktile, int wtile,
                                           KernelShared<NBP, KIND, SLDS>& sh, int lane) {
  constexpr int T = NBP / 16;
  const int q = lane >> 4, c16 = lane & 15;
  const int n0 = wtile * a.wt;
  const int n1 = min(n0 + a.wt, a.nw);
  const int kk0 = ktile * a.kt;
  const int kk1 = min(kk0 + a.kt, a.nklist);
  const double mu = a.mu_ptr ? *a.mu_ptr : a.mu;
  const int nc = a.nc;
  const double beta = a.beta;
  const bool want_s = (KIND == KIND_DENSITY) && (a.mode & MODE_S);
  const bool want_x = (KIND == KIND_DENSITY) && (a.mode & MODE_GLOC);
  // this lane holds diagonal elements (16 t + c16, 16 t + c16) in register i = idg of tile (t, t)
  const bool hasdiag = c16 >= q && ((c16 - q) & 3) == 0;
  const int idg = (c16 - q) >> 2;
  int bad = 0, nonfinite = 0;

  for (int kk = kk0; kk < kk1; ++kk) {
    const int k = a.klist ? a.klist[kk] : kk;
    const int nb = a.nb_uniform > 0 ? a.nb_uniform : a.nb[k];
    const int64_t ob = a.nb_uniform > 0 ? (int64_t)k * nb : a.off_b[k];
    const double* eps = a.eps + ob;
    const double2* P = reinterpret_cast<const double2*>(a.proj) + ob * nc;
    const double wk = a.wk[k];
    double dre[T];
    bool dval[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      int r = 16 * t + c16;
      dval[t] = r < nb;
      dre[t] = (hasdiag && r < nb) ? mu - eps[r] : 1.0;
    }

    Mat<NBP> sacc;
    if (want_s) {
      if constexpr (SLDS) {
#pragma unroll
        for (int e = 0; e < T * T * 4; ++e) sh.s[e * 64 + lane] = make_double2(0.0, 0.0);
      } else {
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int b = 0; b < T; ++b) sacc.re[t][b] = sacc.im[t][b] = (v4d){0.0, 0.0, 0.0, 0.0};
      }
    }
    double trg = 0.0, trg2 = 0.0;

    for (int n = n0; n < n1; ++n) {
      const double wn = (double)(2 * n + 1) * M_PI / beta;
      Mat<NBP> g;
      build_a<NBP>(g, a, P, nb, n, wn, dre, dval, hasdiag, idg, q, c16);
      gauss_jordan<NBP, PF>(g, sh.gj, q, c16, nb, bad);

      if (want_s) {
        if constexpr (SLDS) {
#pragma unroll
          for (int t = 0; t < T; ++t)
#pragma unroll
            for (int b = 0; b < T; ++b)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                int e = (t * T + b) * 4 + i;
                double2 v = sh.s[e * 64 + lane];
                v.x += g.re[t][b][i];
                v.y += g.im[t][b][i];
                sh.s[e * 64 + lane] = v;
              }
        } else {
#pragma unroll
          for (int t = 0; t < T; ++t)
#pragma unroll
            for (int b = 0; b < T; ++b) {
              sacc.re[t][b] += g.re[t][b];
              sacc.im[t][b] += g.im[t][b];
            }
        }
      }

      double dsum = 0.0;  // this lane's share of Re tr G
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (hasdiag && idg == i && dval[t]) dsum += g.re[t][t][i];
      if (!__builtin_isfinite(dsum)) nonfinite = 1;

      if constexpr (KIND == KIND_TRACE) {
        trg += dsum;
        // Re tr G^2 = sum over tile pairs of G_tb[m][n] G_bt[n][m]
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int b = t; b < T; ++b) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              sh.tr[(4 * i + q) * 17 + c16] = make_double2(g.re[b][t][i], g.im[b][t][i]);
            wave_sync();
            // padded rows/columns hold an identity block: keep them out of the sum
            double acc = 0.0;
            const bool colok = 16 * b + c16 < nb;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              double2 v = sh.tr[c16 * 17 + 4 * i + q];
              double term = g.re[t][b][i] * v.x - g.im[t][b][i] * v.y;
              acc += (colok && 16 * t + 4 * i + q < nb) ? term : 0.0;
            }
            trg2 += (b == t) ? acc : 2.0 * acc;
            wave_sync();
          }
      }

      if (want_x) {
        Proj<NBP> pr;
        load_pt<NBP>(pr, P, nc, nb, q, c16);
        // W^T = G^T S^T  (NBP x 16), then X = W S^dag = S G S^dag (16 x 16)
        v4d wr[T], wi[T];
#pragma unroll
        for (int b = 0; b < T; ++b) {
          wr[b] = wi[b] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int t = 0; t < T; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              wr[b] = mma(g.re[t][b][i], pr.pt_r[t][i], wr[b]);
              wr[b] = mms(g.im[t][b][i], pr.pt_i[t][i], wr[b]);
              wi[b] = mma(g.re[t][b][i], pr.pt_i[t][i], wi[b]);
              wi[b] = mma(g.im[t][b][i], pr.pt_r[t][i], wi[b]);
            }
        }
        v4d xr = {0.0, 0.0, 0.0, 0.0}, xi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < T; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            xr = mma(wr[b][i], pr.pt_r[b][i], xr);
            xr = mma(wi[b][i], pr.pt_i[b][i], xr);
            xi = mma(wi[b][i], pr.pt_r[b][i], xi);
            xi = mms(wr[b][i], pr.pt_i[b][i], xi);
          }
        // lane holds X[q + 4 i][c16]; add w_k X to this k tile's partial
        double2* xp = reinterpret_cast<double2*>(a.xpart) + ((int64_t)(a.ktile_base + ktile) * a.nw + n) * 256;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (q + 4 * i < nc && c16 < nc) {
            double2 v = make_double2(wk * xr[i], wk * xi[i]);
            if (kk != kk0) {
              double2 o = xp[i * 64 + lane];
              v.x += o.x;
              v.y += o.y;
            }
            xp[i * 64 + lane] = v;
          }
        }
      }
    }  // frequencies

    if (want_s) {
      double2* sp = reinterpret_cast<double2*>(a.spart) + (int64_t)wtile * a.s_stride + a.off_s[k];
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int b = 0; b < T; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            int e = (t * T + b) * 4 + i;
            if constexpr (SLDS)
              sp[e * 64 + lane] = sh.s[e * 64 + lane];
            else
              sp[e * 64 + lane] = make_double2(sacc.re[t][b][i], sacc.im[t][b][i]);
          }
    }
    if constexpr (KIND == KIND_TRACE) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        trg += __shfl_xor(trg, off);
        trg2 += __shfl_xor(trg2, off);
      }
      if (lane == 0) {
        a.tpart[((int64_t)wtile * a.nk + k) * 2 + 0] = trg;
        a.tpart[((int64_t)wtile * a.nk + k) * 2 + 1] = trg2;
      }
    }
  }  // k
  if (bad) atomicOr(a.err, ERR_SINGULAR);
  if (nonfinite) atomicOr(a.err, ERR_NONFINITE);
}

template <int NBP, int KIND, int PF, int SLDS, int OCC = 1>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(OCC))) dyson_kernel(DysonArgs a) {
  __shared__ KernelShared<NBP, KIND, SLDS> sh;
  dyson_tile<NBP, KIND, PF, SLDS>(a, blockIdx.x / a.n_wtiles, blockIdx.x % a.n_wtiles, sh, threadIdx.x);
}

// Kernel variants: bit 0 = PF, bit 1 = SLDS (density only), bit 2 = two
// wavefronts per SIMD (register budget 256).  Each size instantiates the
// variants listed in its unit; launch_variant returns hipErrorInvalidValue for
// the others.
template <int NBP, int KIND, int VAR>
hipError_t launch_one(const DysonArgs& a, dim3 grid, hipStream_t s) {
  hipLaunchKernelGGL((dyson_kernel<NBP, KIND, VAR & 1, (VAR >> 1) & 1, (VAR & 4) ? 2 : 1>), grid, dim3(64), 0, s,
                     a);
  return hipGetLastError();
}

template <int NBP, int KIND, int... VARS>
struct VariantSet {
  static hipError_t launch(int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
    hipError_t r = hipErrorInvalidValue;
    bool hit = ((var == VARS ? (r = launch_one<NBP, KIND, VARS>(a, grid, s), true) : false) || ...);
    (void)hit;
    return r;
  }
  static int list(int* out, int max) {
    int n = 0;
    ((n < max ? (out[n++] = VARS, 0) : 0), ...);
    return n;
  }
};

}  // namespace dmft
