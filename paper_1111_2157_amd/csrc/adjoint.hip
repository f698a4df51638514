// Adjoint (vector-Jacobian product) of the lattice Dyson and Matsubara-sum
// steps, on the same per-(k, i w_n) register layout as dyson_impl.h.
//
// With G = A^{-1} and dA = -S^dag dSigma S, dG = G S^dag dSigma S G and
// dG/dmu = -G^2.  Per (k, n) the kernel recomputes G (embed + Gauss-Jordan),
// stages it in LDS so that its transpose is available as matrix-core A
// operands, and forms on the matrix cores
//     W = S G          (from registers, as W^T = G^T S^T)
//     Z = G S^dag      (A operand read transposed from LDS)
//     M = W Z = S G^2 S^dag ,
// together with Re tr G and Re tr G^2 (the transposed LDS fragments pair each
// element with its mirror).  That is the fused scalar adjoint of N_tot:
//     dN_tot/dSigma_n = (2/beta) [ sum_k w_k M_kn ]^dag ,
//     dN_tot/dmu      = sum_k w_k [ (beta/4) nb - (2/beta) sum_n (Re tr G^2 + nb/w_n^2) ].
// The general product for upstream (Nbar_k, Gbar_n) in PyTorch's convention,
//     Sigmabar_n = sum_k S G^dag C G^dag S^dag ,  C = (1/beta) Nt + w_k S^dag Gbar_n S ,
// Nt = Nbar + Nbar^dag, is evaluated as Z^dag C W^dag =
//     (1/beta) Z^dag (Nt W^dag) + w_k X^dag Gbar_n X^dag ,   X = S G S^dag = W S^dag ,
// and mubar collects -Re<C, G^2> = -(1/beta) Re tr(Nt G^2) - w_k Re<Gbar_n, M>,
// with tr(Nt G^2) = sum of (Nt G) against the transposed G fragments.
#include "dyson_impl.h"

namespace dmft {

template <int NBP>
struct AdjShared {
  GJShared<NBP> gj;
  double2 g[NBP * NBP];  // G, row-major
  double2 x[16 * 17];    // 16x16 staging for X^dag Gbar X^dag
  double2 u[16 * 17];
};

// Extra arguments of the adjoint launch.
struct AdjArgs {
  const double* nbar;     // complex, N(k) layout, or null
  const int64_t* off_n;   // [nk+1] (ragged) or null (uniform)
  const double* gbar;     // complex [nw][nc][nc] or null
  double* mpart;          // [n_ktiles][nw][256] complex: sum_k w_k M (GEN 0) or Sigmabar (GEN 1)
  double* tpart;          // [n_wtiles][nk][3]: sum_n Re tr G, Re tr G^2, mubar share
};

template <int NBP, int GEN>
__global__ void __launch_bounds__(64) adjoint_kernel(DysonArgs a, AdjArgs ad) {
  constexpr int T = NBP / 16;
  __shared__ AdjShared<NBP> sh;
  const int lane = threadIdx.x, q = lane >> 4, c16 = lane & 15;
  const int wtile = blockIdx.x % a.n_wtiles;
  const int ktile = blockIdx.x / a.n_wtiles;
  const int n0 = wtile * a.wt;
  const int n1 = min(n0 + a.wt, a.nw);
  const int kk0 = ktile * a.kt;
  const int kk1 = min(kk0 + a.kt, a.nklist);
  const double mu = a.mu_ptr ? *a.mu_ptr : a.mu;
  const int nc = a.nc;
  const double beta = a.beta;
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
    const double2* nbar = nullptr;
    if (GEN && ad.nbar) {
      int64_t on = ad.off_n ? ad.off_n[k] : (int64_t)k * nb * nb;
      nbar = reinterpret_cast<const double2*>(ad.nbar) + on;
    }
    double dre[T];
    bool dval[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      int r = 16 * t + c16;
      dval[t] = r < nb;
      dre[t] = (hasdiag && r < nb) ? mu - eps[r] : 1.0;
    }
    double trg = 0.0, trg2 = 0.0, mub = 0.0;

    for (int n = n0; n < n1; ++n) {
      const double wn = (double)(2 * n + 1) * M_PI / beta;
      Mat<NBP> g;
      build_a<NBP>(g, a, P, nb, n, wn, dre, dval, hasdiag, idg, q, c16);
      gauss_jordan<NBP, 0>(g, sh.gj, q, c16, nb, bad);
      // stage G (row-major) for transposed access
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int b = 0; b < T; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            sh.g[(16 * t + 4 * i + q) * NBP + 16 * b + c16] = make_double2(g.re[t][b][i], g.im[t][b][i]);
      wave_sync();

      double dsum = 0.0;
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (hasdiag && idg == i && dval[t]) dsum += g.re[t][t][i];
      if (!__builtin_isfinite(dsum)) nonfinite = 1;
      trg += dsum;

      Proj<NBP> pr;
      load_pt<NBP>(pr, P, nc, nb, q, c16);
      // W^T = G^T S^T: lane holds W[c16][16 b + 4 i + q] in register i of wr[b], wi[b]
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
      // Z = G S^dag: lane holds Z[16 b + 4 i + q][c16] in register i of zr[b], zi[b];
      // the A fragments G[16 b + c16][16 t + 4 i + q] are the mirrors of this lane's
      // own elements, so they also give Re tr G^2 (and tr(Nt G^2) below).
      v4d zr[T], zi[T];
      double g2 = 0.0;
#pragma unroll
      for (int b = 0; b < T; ++b) {
        zr[b] = zi[b] = (v4d){0.0, 0.0, 0.0, 0.0};
        const bool colok = 16 * b + c16 < nb;
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            double2 h = sh.g[(16 * b + c16) * NBP + 16 * t + 4 * i + q];
            zr[b] = mma(h.x, pr.pt_r[t][i], zr[b]);
            zr[b] = mma(h.y, pr.pt_i[t][i], zr[b]);
            zi[b] = mma(h.y, pr.pt_r[t][i], zi[b]);
            zi[b] = mms(h.x, pr.pt_i[t][i], zi[b]);
            double term = g.re[t][b][i] * h.x - g.im[t][b][i] * h.y;
            g2 += (colok && 16 * t + 4 * i + q < nb) ? term : 0.0;
          }
      }
      trg2 += g2;
      // M = W Z = S G^2 S^dag: lane holds M[q + 4 i][c16]
      v4d mr = {0.0, 0.0, 0.0, 0.0}, mi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int b = 0; b < T; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          mr = mma(wr[b][i], zr[b][i], mr);
          mr = mms(wi[b][i], zi[b][i], mr);
          mi = mma(wr[b][i], zi[b][i], mi);
          mi = mma(wi[b][i], zr[b][i], mi);
        }
      v4d outr, outi;
      if constexpr (GEN == 0) {
        outr = mr * wk;
        outi = mi * wk;
      } else {
        outr = outi = (v4d){0.0, 0.0, 0.0, 0.0};
        if (nbar) {
          // Y = Nt W^dag (NBP x 16); lane holds Y[16 t + 4 i + q][c16] in register i of yr[t]
          double tn2 = 0.0;  // this lane's share of Re tr(Nt G^2)
#pragma unroll
          for (int t = 0; t < T; ++t) {
            v4d yr = {0.0, 0.0, 0.0, 0.0}, yi = {0.0, 0.0, 0.0, 0.0};
            const int r = 16 * t + c16;
#pragma unroll
            for (int b = 0; b < T; ++b)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int c = 16 * b + 4 * i + q;
                double2 nt = make_double2(0.0, 0.0);
                if (r < nb && c < nb) {
                  double2 x1 = nbar[r * nb + c], x2 = nbar[c * nb + r];
                  nt = make_double2(x1.x + x2.x, x1.y - x2.y);
                }
                // conj(W)[c16][c]: (wr, -wi)
                yr = mma(nt.x, wr[b][i], yr);
                yr = mma(nt.y, wi[b][i], yr);
                yi = mma(nt.y, wr[b][i], yi);
                yi = mms(nt.x, wi[b][i], yi);
              }
            // Z^dag Y accumulated into out: chunk (t, i): A = conj(Z[16 t + 4 i + q][c16]), B = Y
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              outr = mma(zr[t][i], yr[i], outr);
              outr = mma(zi[t][i], yi[i], outr);
              outi = mma(zr[t][i], yi[i], outi);
              outi = mms(zi[t][i], yr[i], outi);
            }
            // (Nt G)[16 t + 4 i' + q][16 b + c16] paired with G[16 b + c16][16 t + 4 i' + q]
#pragma unroll
            for (int b = 0; b < T; ++b) {
              v4d ur = {0.0, 0.0, 0.0, 0.0}, ui = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
              for (int t2 = 0; t2 < T; ++t2)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const int c = 16 * t2 + 4 * i + q;
                  double2 nt = make_double2(0.0, 0.0);
                  if (r < nb && c < nb) {
                    double2 x1 = nbar[r * nb + c], x2 = nbar[c * nb + r];
                    nt = make_double2(x1.x + x2.x, x1.y - x2.y);
                  }
                  ur = mma(nt.x, g.re[t2][b][i], ur);
                  ur = mms(nt.y, g.im[t2][b][i], ur);
                  ui = mma(nt.x, g.im[t2][b][i], ui);
                  ui = mma(nt.y, g.re[t2][b][i], ui);
                }
              const bool colok = 16 * b + c16 < nb;
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                double2 h = sh.g[(16 * b + c16) * NBP + 16 * t + 4 * i + q];
                double term = ur[i] * h.x - ui[i] * h.y;
                tn2 += (colok && 16 * t + 4 * i + q < nb) ? term : 0.0;
              }
            }
          }
          outr *= 1.0 / beta;
          outi *= 1.0 / beta;
          mub -= tn2 / beta;
        }
        if (ad.gbar) {
          // X = W S^dag: lane holds X[q + 4 i][c16]
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
          const double2* gb = reinterpret_cast<const double2*>(ad.gbar) + (int64_t)n * nc * nc;
          double gm = 0.0;  // Re<Gbar, M> share
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            int al = q + 4 * i;
            sh.x[al * 17 + c16] = make_double2(xr[i], xi[i]);
            if (al < nc && c16 < nc) {
              double2 v = gb[al * nc + c16];
              gm += v.x * mr[i] + v.y * mi[i];
            }
          }
          mub -= wk * gm;
          wave_sync();
          // U = Gbar X^dag: lane computes U[q + 4 i][c16] = sum_d Gbar[q+4i][d] conj(X[c16][d])
          double2 uu[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            int al = q + 4 * i;
            double2 acc = make_double2(0.0, 0.0);
            for (int d = 0; d < nc; ++d) {
              double2 gv = (al < nc) ? gb[al * nc + d] : make_double2(0.0, 0.0);
              double2 xv = sh.x[c16 * 17 + d];
              acc.x += gv.x * xv.x + gv.y * xv.y;
              acc.y += gv.y * xv.x - gv.x * xv.y;
            }
            uu[i] = acc;
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) sh.u[(q + 4 * i) * 17 + c16] = uu[i];
          wave_sync();
          // X^dag U: lane computes [X^dag U][q + 4 i][c16] = sum_g conj(X[g][q+4i]) U[g][c16]
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            int al = q + 4 * i;
            double2 acc = make_double2(0.0, 0.0);
            for (int gg = 0; gg < nc; ++gg) {
              double2 xv = sh.x[gg * 17 + al];
              double2 uv = sh.u[gg * 17 + c16];
              acc.x += xv.x * uv.x + xv.y * uv.y;
              acc.y += xv.x * uv.y - xv.y * uv.x;
            }
            outr[i] += wk * acc.x;
            outi[i] += wk * acc.y;
          }
          wave_sync();
        }
      }
      double2* mp = reinterpret_cast<double2*>(ad.mpart) + ((int64_t)(a.ktile_base + ktile) * a.nw + n) * 256;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (q + 4 * i < nc && c16 < nc) {
          double2 v = make_double2(outr[i], outi[i]);
          if (kk != kk0) {
            double2 o = mp[i * 64 + lane];
            v.x += o.x;
            v.y += o.y;
          }
          mp[i * 64 + lane] = v;
        }
      }
      wave_sync();
    }  // frequencies

#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      trg += __shfl_xor(trg, off);
      trg2 += __shfl_xor(trg2, off);
      mub += __shfl_xor(mub, off);
    }
    if (lane == 0) {
      double* tp = ad.tpart + ((int64_t)wtile * a.nk + k) * 3;
      tp[0] = trg;
      tp[1] = trg2;
      tp[2] = mub;
    }
  }  // k
  if (bad) atomicOr(a.err, ERR_SINGULAR);
  if (nonfinite) atomicOr(a.err, ERR_NONFINITE);
}

template <int NBP>
static hipError_t launch_adj(int gen, const DysonArgs& a, const AdjArgs& ad, dim3 grid, hipStream_t s) {
  if (gen)
    hipLaunchKernelGGL((adjoint_kernel<NBP, 1>), grid, dim3(64), 0, s, a, ad);
  else
    hipLaunchKernelGGL((adjoint_kernel<NBP, 0>), grid, dim3(64), 0, s, a, ad);
  return hipGetLastError();
}

hipError_t launch_adjoint(int nbp, int gen, const DysonArgs& a, const double* nbar, const int64_t* off_n,
                          const double* gbar, double* mpart, double* tpart, int n_ktiles, hipStream_t s) {
  AdjArgs ad{nbar, off_n, gbar, mpart, tpart};
  dim3 grid((unsigned)(n_ktiles * a.n_wtiles));
  switch (nbp) {
    case 16: return launch_adj<16>(gen, a, ad, grid, s);
    case 32: return launch_adj<32>(gen, a, ad, grid, s);
    case 48: return launch_adj<48>(gen, a, ad, grid, s);
    default: return hipErrorInvalidValue;
  }
}

// Sigmabar_n from the k-tile partials: scalar adjoint (gen 0) scale * [sum]^dag,
// general VJP (gen 1) the plain sum.
__global__ void __launch_bounds__(256) sigma_bar_reduce_kernel(int n_ktiles, int nw, int nc, const double* mpart,
                                                               double scale, int dagger, double* out) {
  int n = blockIdx.x;
  int e = threadIdx.x, i = e >> 6, lane = e & 63, q = lane >> 4, c16 = lane & 15;
  int al = q + 4 * i, be = c16;
  if (al >= nc || be >= nc) return;
  const double2* mp = reinterpret_cast<const double2*>(mpart);
  double2 acc = make_double2(0.0, 0.0);
  for (int kt = 0; kt < n_ktiles; ++kt) {
    double2 v = mp[((int64_t)kt * nw + n) * 256 + e];
    acc.x += v.x;
    acc.y += v.y;
  }
  double2* o = reinterpret_cast<double2*>(out) + (int64_t)n * nc * nc;
  if (dagger)
    o[be * nc + al] = make_double2(scale * acc.x, -scale * acc.y);
  else
    o[al * nc + be] = make_double2(scale * acc.x, scale * acc.y);
}

hipError_t launch_sigma_bar_reduce(int n_ktiles, int nw, int nc, const double* mpart, double scale, int dagger,
                                   double* out, hipStream_t s) {
  hipLaunchKernelGGL(sigma_bar_reduce_kernel, dim3(nw), dim3(256), 0, s, n_ktiles, nw, nc, mpart, scale, dagger,
                     out);
  return hipGetLastError();
}

}  // namespace dmft
