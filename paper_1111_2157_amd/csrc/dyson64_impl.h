// Device code of the two-wavefront Dyson kernel for band windows padded to 64
// (included by dyson64.hip and the persistent batched kernel).
//
// The register layout of dyson_impl.h (lane l = 16 q + c16 holds element
// (16 t + 4 i + q, 16 b + c16) in register (t, b, i)) is split by row tiles:
// wavefront w of the work-group owns row tiles t = 2 w and 2 w + 1, all four
// column tiles.  In the Gauss-Jordan sweep the pivot column is needed only
// for a wavefront's own rows, so it travels through wave-private LDS slots;
// the pivot row (and pivot) is published by the wavefront that owns it and
// read by both after one work-group barrier per step.  The running frequency
// sum of G is accumulated on the matrix cores (identity-chunk products) so
// that it can live in accumulation registers, and S G S^dag is formed from
// each wavefront's rows and summed through LDS.
#pragma once

#include "dyson_impl.h"

namespace dmft {

namespace d64 {

constexpr int NBP = 64, T = 4, TL = 2;  // TL row tiles per wavefront

struct LMat {
  v4d re[TL][T], im[TL][T];
};

struct Shared {
  double2 col[2][NBP];
  double2 row[2][NBP];
  double2 piv[2];
  double2 tr[16 * 17];
  double2 x[4 * 64];
};

struct RowB {
  double2 rv[T];
  double2 p;
};
struct ColB {
  double2 cc[TL][4];
};

template <int K>
__device__ __forceinline__ void publish(const LMat& g, Shared& sh, int w, int q, int c16) {
  constexpr int tk = K >> 4, ik = (K >> 2) & 3, qk = K & 3, bk = K >> 4, ck = K & 15, s = K & 1;
  constexpr int wk = tk >> 1, tlk = tk & 1;
  if (c16 == ck) {
#pragma unroll
    for (int tl = 0; tl < TL; ++tl)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double2 v = make_double2(g.re[tl][bk][i], g.im[tl][bk][i]);
        if (w == wk && tl == tlk && i == ik && q == qk) v.x -= 1.0;
        sh.col[s][16 * (2 * w + tl) + 4 * i + q] = v;
      }
  }
  if (w == wk && q == qk) {
#pragma unroll
    for (int b = 0; b < T; ++b) {
      double2 v = make_double2(g.re[tlk][b][ik], g.im[tlk][b][ik]);
      if (b == bk && c16 == ck) v.x += 1.0;
      sh.row[s][16 * b + c16] = v;
    }
    if (c16 == ck) sh.piv[s] = make_double2(g.re[tlk][bk][ik], g.im[tlk][bk][ik]);
  }
}

template <int K>
__device__ __forceinline__ void fetch_row(RowB& rb, const Shared& sh, int c16) {
  constexpr int s = K & 1;
#pragma unroll
  for (int b = 0; b < T; ++b) rb.rv[b] = sh.row[s][16 * b + c16];
  rb.p = sh.piv[s];
}

template <int K>
__device__ __forceinline__ void fetch_col(ColB& cb, const Shared& sh, int w, int q) {
  constexpr int s = K & 1;
#pragma unroll
  for (int tl = 0; tl < TL; ++tl)
#pragma unroll
    for (int i = 0; i < 4; ++i) cb.cc[tl][i] = sh.col[s][16 * (2 * w + tl) + 4 * i + q];
}

// Step K.  On entry rb holds step K's pivot row and pivot; the pivot column is
// read here (it is only needed for this wavefront's rows).
template <int K>
__device__ __forceinline__ void steps(LMat& g, RowB& rb, ColB& cb, Shared& sh, int w, int q, int c16, int nb,
                                      int& bad) {
  if constexpr (K < NBP) {
    if (K >= nb) return;
    fetch_col<K>(cb, sh, w, q);
    double2 ip = crecip(rb.p);
    bad |= (rb.p.x == 0.0 && rb.p.y == 0.0);
    double2 rs[T];
#pragma unroll
    for (int b = 0; b < T; ++b) rs[b] = cmul(rb.rv[b], ip);
    if constexpr (K + 1 < NBP) {
      constexpr int K1 = K + 1, t1 = K1 >> 4, i1 = (K1 >> 2) & 3, b1 = K1 >> 4;
      constexpr int w1 = t1 >> 1, tl1 = t1 & 1;
#pragma unroll
      for (int tl = 0; tl < TL; ++tl)
#pragma unroll
        for (int i = 0; i < 4; ++i) upd(g.re[tl][b1], g.im[tl][b1], i, cb.cc[tl][i], rs[b1]);
      if (w == w1) {
#pragma unroll
        for (int b = 0; b < T; ++b)
          if (b != b1) upd(g.re[tl1][b], g.im[tl1][b], i1, cb.cc[tl1][i1], rs[b]);
      }
      publish<K1>(g, sh, w, q, c16);
      __syncthreads();
      RowB rn;
      fetch_row<K1>(rn, sh, c16);
#pragma unroll
      for (int tl = 0; tl < TL; ++tl)
#pragma unroll
        for (int b = 0; b < T; ++b) {
          if (b == b1) continue;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (tl == tl1 && i == i1) {
              if (w != w1) upd(g.re[tl][b], g.im[tl][b], i, cb.cc[tl][i], rs[b]);
              continue;
            }
            upd(g.re[tl][b], g.im[tl][b], i, cb.cc[tl][i], rs[b]);
          }
        }
      steps<K + 1>(g, rn, cb, sh, w, q, c16, nb, bad);
    } else {
#pragma unroll
      for (int tl = 0; tl < TL; ++tl)
#pragma unroll
        for (int b = 0; b < T; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) upd(g.re[tl][b], g.im[tl][b], i, cb.cc[tl][i], rs[b]);
    }
  }
}

// One (k-tile, frequency-tile) work item on a work-group of two wavefronts (tid = 0..127).
template <int KIND>
__device__ __forceinline__ void tile(const DysonArgs& a, int ktile, int wtile, Shared& sh, int tid) {
  const int w = tid >> 6, lane = tid & 63, q = lane >> 4, c16 = lane & 15;
  const int n0 = wtile * a.wt;
  const int n1 = min(n0 + a.wt, a.nw);
  const int kk0 = ktile * a.kt;
  const int kk1 = min(kk0 + a.kt, a.nklist);
  const double mu = a.mu_ptr ? *a.mu_ptr : a.mu;
  const int nc = a.nc;
  const double beta = a.beta;
  const bool want_s = (KIND == KIND_DENSITY) && (a.mode & MODE_S);
  const bool want_x = (KIND == KIND_DENSITY) && (a.mode & MODE_GLOC);
  const bool hasdiag = c16 >= q && ((c16 - q) & 3) == 0;
  const int idg = (c16 - q) >> 2;
  // identity-chunk operands for accumulating a tile on the matrix cores
  double eye[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) eye[i] = (c16 == 4 * i + q) ? 1.0 : 0.0;
  int bad = 0, nonfinite = 0;

  for (int kk = kk0; kk < kk1; ++kk) {
    const int k = a.klist ? a.klist[kk] : kk;
    const int nb = a.nb_uniform > 0 ? a.nb_uniform : a.nb[k];
    const int64_t ob = a.nb_uniform > 0 ? (int64_t)k * nb : a.off_b[k];
    const double* eps = a.eps + ob;
    const double2* P = reinterpret_cast<const double2*>(a.proj) + ob * nc;
    const double wk = a.wk[k];
    double dre[TL];
    bool dval[TL];
#pragma unroll
    for (int tl = 0; tl < TL; ++tl) {
      int r = 16 * (2 * w + tl) + c16;
      dval[tl] = r < nb;
      dre[tl] = (hasdiag && r < nb) ? mu - eps[r] : 1.0;
    }
    LMat sacc;
#pragma unroll
    for (int tl = 0; tl < TL; ++tl)
#pragma unroll
      for (int b = 0; b < T; ++b) sacc.re[tl][b] = sacc.im[tl][b] = (v4d){0.0, 0.0, 0.0, 0.0};
    double trg = 0.0, trg2 = 0.0;

    for (int n = n0; n < n1; ++n) {
      const double wn = (double)(2 * n + 1) * M_PI / beta;
      LMat g;
      {
        Proj<NBP> pr;
        load_pa<NBP>(pr, P, nc, nb, q, c16);
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
        for (int tl = 0; tl < TL; ++tl) {
          const int t = 2 * w + tl;
#pragma unroll
          for (int b = 0; b < T; ++b) {
            v4d zr = {0.0, 0.0, 0.0, 0.0}, zi = {0.0, 0.0, 0.0, 0.0};
            const bool diag_tile = (t == b);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              bool on = diag_tile && hasdiag && idg == i;
              zr[i] = on ? dre[tl] : 0.0;
              zi[i] = (on && dval[tl]) ? wn : 0.0;
            }
            // the t-th band tile of S^dag: register (i, t) of pa is S[q + 4 i][16 t + c16];
            // t is wave-dependent, so select it from the four tiles
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              if (i >= kc) break;
              double ar = pr.pa_r[i][0], ai = pr.pa_i[i][0];
#pragma unroll
              for (int tt = 1; tt < T; ++tt)
                if (t == tt) {
                  ar = pr.pa_r[i][tt];
                  ai = pr.pa_i[i][tt];
                }
              zr = mms(ar, vr[b][i], zr);
              zr = mms(ai, vi[b][i], zr);
              zi = mms(ar, vi[b][i], zi);
              zi = mma(ai, vr[b][i], zi);
            }
            g.re[tl][b] = zr;
            g.im[tl][b] = zi;
          }
        }
      }

      // Gauss-Jordan sweep
      {
        RowB rb;
        ColB cb;
        publish<0>(g, sh, w, q, c16);
        __syncthreads();
        fetch_row<0>(rb, sh, c16);
        steps<0>(g, rb, cb, sh, w, q, c16, nb, bad);
        __syncthreads();
      }

      if (want_s) {
#pragma unroll
        for (int tl = 0; tl < TL; ++tl)
#pragma unroll
          for (int b = 0; b < T; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              sacc.re[tl][b] = mma(eye[i], g.re[tl][b][i], sacc.re[tl][b]);
              sacc.im[tl][b] = mma(eye[i], g.im[tl][b][i], sacc.im[tl][b]);
            }
      }
      double dsum = 0.0;
#pragma unroll
      for (int tl = 0; tl < TL; ++tl)
#pragma unroll
        for (int b = 0; b < T; ++b)
          if (b == 2 * w + tl) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (hasdiag && idg == i && dval[tl]) dsum += g.re[tl][b][i];
          }
      if (!__builtin_isfinite(dsum)) nonfinite = 1;

      if constexpr (KIND == KIND_TRACE) {
        trg += dsum;
        // Re tr G^2 over tile pairs; tile (b, t) is published by its owner through LDS
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int b = t; b < T; ++b) {
            if (w == (b >> 1)) {
#pragma unroll
              for (int i = 0; i < 4; ++i)
                sh.tr[(4 * i + q) * 17 + c16] = make_double2(g.re[b & 1][t][i], g.im[b & 1][t][i]);
            }
            __syncthreads();
            if (w == (t >> 1)) {
              double acc = 0.0;
              const bool colok = 16 * b + c16 < nb;
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                double2 v = sh.tr[c16 * 17 + 4 * i + q];
                double term = g.re[t & 1][b][i] * v.x - g.im[t & 1][b][i] * v.y;
                acc += (colok && 16 * t + 4 * i + q < nb) ? term : 0.0;
              }
              trg2 += (b == t) ? acc : 2.0 * acc;
            }
            __syncthreads();
          }
      }

      if (want_x) {
        Proj<NBP> pr;
        load_pt<NBP>(pr, P, nc, nb, q, c16);
        // this wavefront's share of W^T = G^T S^T (its rows), then of X = W S^dag
        v4d wr[T], wi[T];
#pragma unroll
        for (int b = 0; b < T; ++b) {
          wr[b] = wi[b] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int tl = 0; tl < TL; ++tl) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              double ptr_ = w ? pr.pt_r[2 + tl][i] : pr.pt_r[tl][i];
              double pti_ = w ? pr.pt_i[2 + tl][i] : pr.pt_i[tl][i];
              wr[b] = mma(g.re[tl][b][i], ptr_, wr[b]);
              wr[b] = mms(g.im[tl][b][i], pti_, wr[b]);
              wi[b] = mma(g.re[tl][b][i], pti_, wi[b]);
              wi[b] = mma(g.im[tl][b][i], ptr_, wi[b]);
            }
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
        if (w == 1) {
#pragma unroll
          for (int i = 0; i < 4; ++i) sh.x[i * 64 + lane] = make_double2(xr[i], xi[i]);
        }
        __syncthreads();
        if (w == 0) {
          double2* xp = reinterpret_cast<double2*>(a.xpart) + ((int64_t)(a.ktile_base + ktile) * a.nw + n) * 256;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (q + 4 * i < nc && c16 < nc) {
              double2 o1 = sh.x[i * 64 + lane];
              double2 v = make_double2(wk * (xr[i] + o1.x), wk * (xi[i] + o1.y));
              if (kk != kk0) {
                double2 o = xp[i * 64 + lane];
                v.x += o.x;
                v.y += o.y;
              }
              xp[i * 64 + lane] = v;
            }
          }
        }
        __syncthreads();
      }
    }  // frequencies

    if (want_s) {
      double2* sp = reinterpret_cast<double2*>(a.spart) + (int64_t)wtile * a.s_stride + a.off_s[k];
#pragma unroll
      for (int tl = 0; tl < TL; ++tl)
#pragma unroll
        for (int b = 0; b < T; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            int e = ((2 * w + tl) * T + b) * 4 + i;
            sp[e * 64 + lane] = make_double2(sacc.re[tl][b][i], sacc.im[tl][b][i]);
          }
    }
    if constexpr (KIND == KIND_TRACE) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        trg += __shfl_xor(trg, off);
        trg2 += __shfl_xor(trg2, off);
      }
      // the two wavefronts' shares are combined in a fixed order through LDS
      if (lane == 0) sh.x[w] = make_double2(trg, trg2);
      __syncthreads();
      if (tid == 0) {
        a.tpart[((int64_t)wtile * a.nk + k) * 2 + 0] = sh.x[0].x + sh.x[1].x;
        a.tpart[((int64_t)wtile * a.nk + k) * 2 + 1] = sh.x[0].y + sh.x[1].y;
      }
      __syncthreads();
    }
  }  // k
  if (bad) atomicOr(a.err, ERR_SINGULAR);
  if (nonfinite) atomicOr(a.err, ERR_NONFINITE);
}

template <int KIND>
__global__ void __launch_bounds__(128) kernel(DysonArgs a) {
  __shared__ Shared sh;
  tile<KIND>(a, blockIdx.x / a.n_wtiles, blockIdx.x % a.n_wtiles, sh, threadIdx.x);
}

}  // namespace d64

}  // namespace dmft
