// DMFT self-consistency step that consumes G_loc (Sec. 3.2.2 eq. dmftloop2):
//
//     E_imp        = sum_k w_k S_k diag(E_k) S_k^dag - diag(V_DC)
//     Delta(i w_n) = i w_n + mu - E_imp - Sigma(i w_n) - G_loc(i w_n)^-1 .
//
// E_imp: per-block partial sums over strided k (projectors staged in LDS, one
// thread per (alpha, beta)), then a fixed-order sum of the partials.
// Delta: one wavefront per four frequencies; lane 16 g + i holds row i of
// G_loc(i w_{4b+g}) and the inversion is the row-layout Gauss-Jordan sweep of
// the low-rank kernel (no pivoting: the anti-Hermitian part of G_loc(i w_n),
// -sum_k w_k S G (w_n + Im parts) G^dag S^dag, is negative definite for
// w_n > 0, so every leading block is invertible).
#include "lowrank_impl.h"

namespace dmft {

// E_imp partials: block b sums k = b, b + G, ... (G = gridDim.x); each k's
// projector and band energies are staged in LDS and thread (alpha, beta) adds
// w_k sum_r S[alpha][r] E_r conj(S[beta][r]).  One pass over the projectors.
__global__ void __launch_bounds__(256) eimp_partial_kernel(int nk, int nc, int nb_uniform, const int32_t* nb,
                                                           const int64_t* off_b, const double* eps,
                                                           const double* wk, const double* proj, double* part) {
  __shared__ double2 sS[16 * 65];  // rows padded to n + 1: a row stride of n * 16 B puts every row in one bank
  __shared__ double sE[64];
  const int t = threadIdx.x;
  const int al = t / nc, be = t - al * nc;
  const bool owner = t < nc * nc;
  const double2* P = reinterpret_cast<const double2*>(proj);
  double sr = 0.0, si = 0.0;
  for (int k = blockIdx.x; k < nk; k += gridDim.x) {
    const int n = nb_uniform > 0 ? nb_uniform : nb[k];
    const int64_t ob = nb_uniform > 0 ? (int64_t)k * n : off_b[k];
    __syncthreads();
    for (int idx = t; idx < nc * n; idx += 256) {
      const int row = idx / n;
      sS[idx + row] = P[ob * nc + idx];
    }
    for (int r = t; r < n; r += 256) sE[r] = eps[ob + r];
    __syncthreads();
    if (owner) {
      double ar = 0.0, ai = 0.0;
      for (int r = 0; r < n; ++r) {
        const double2 x = sS[al * (n + 1) + r], y = sS[be * (n + 1) + r];
        const double e = sE[r];
        ar += e * (x.x * y.x + x.y * y.y);
        ai += e * (x.y * y.x - x.x * y.y);
      }
      sr += wk[k] * ar;
      si += wk[k] * ai;
    }
  }
  if (owner) reinterpret_cast<double2*>(part)[(int64_t)blockIdx.x * nc * nc + t] = make_double2(sr, si);
}

// E_imp = (fixed-order sum of the partials) - diag(V_DC): one work-group per
// (alpha, beta), thread t sums partials t, t + 256, ... and a tree adds the threads.
__global__ void __launch_bounds__(256) eimp_reduce_kernel(int nc, int nparts, const double* part, const double* e_dc,
                                                          double* e_imp) {
  __shared__ double rr[256], ri[256];
  const int t = threadIdx.x, e = blockIdx.x;
  const double2* q = reinterpret_cast<const double2*>(part);
  double sr = 0.0, si = 0.0;
  for (int b = t; b < nparts; b += 256) {
    const double2 v = q[(int64_t)b * nc * nc + e];
    sr += v.x;
    si += v.y;
  }
  rr[t] = sr;
  ri[t] = si;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      rr[t] += rr[t + h];
      ri[t] += ri[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    const int al = e / nc, be = e - al * nc;
    reinterpret_cast<double2*>(e_imp)[e] = make_double2(al == be ? rr[0] - e_dc[al] : rr[0], ri[0]);
  }
}

// Delta for four frequencies per wavefront.  G_loc and Sigma of the four
// frequencies (contiguous in memory) are staged through LDS so that loads and
// stores are coalesced; lane 16 g + i then works on row i of frequency 4b + g.
__global__ void __launch_bounds__(64) delta_kernel(int nw, int nc, double beta, double mu, const double* gloc,
                                                   const double* sigma, const double* e_imp, double* delta,
                                                   int* err) {
  __shared__ double2 tg[4 * 256], ts[4 * 256];
  const int lane = threadIdx.x, g = lane >> 4, i = lane & 15;
  const int n0 = 4 * blockIdx.x;
  const int nmat = nw - n0 < 4 ? nw - n0 : 4;
  const int nn = nc * nc, cnt = nmat * nn;
  const int64_t base = (int64_t)n0 * nn;
  const double2* G = reinterpret_cast<const double2*>(gloc) + base;
  const double2* S = reinterpret_cast<const double2*>(sigma) + base;
  for (int idx = lane; idx < cnt; idx += 64) {
    tg[idx] = G[idx];
    ts[idx] = S[idx];
  }
  __syncthreads();
  const bool live = g < nmat;
  double rr[16], ri[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    double2 v = (i < nc && j < nc) ? tg[g * nn + i * nc + j] : make_double2(0.0, 0.0);
    if (!live) v = make_double2(i == j ? 1.0 : 0.0, 0.0);  // keeps the idle rows' pivots nonzero
    rr[j] = v.x;
    ri[j] = v.y;
  }
  int bad = 0;
  rsweep<0, 16>(rr, ri, i, nc, bad);
  int nonfinite = 0;
  if (live && i < nc) {
    const int n = n0 + g;
    const double wn = (double)(2 * n + 1) * M_PI / beta;
    const double2* E = reinterpret_cast<const double2*>(e_imp);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (j < nc) {
        const double2 sv = ts[g * nn + i * nc + j], e = E[i * nc + j];
        double2 v = make_double2(-e.x - sv.x - rr[j], -e.y - sv.y - ri[j]);
        if (j == i) {
          v.x += mu;
          v.y += wn;
        }
        if (!__builtin_isfinite(v.x) || !__builtin_isfinite(v.y)) nonfinite = 1;
        ts[g * nn + i * nc + j] = v;  // this lane's own row
      }
    }
  }
  __syncthreads();
  double2* D = reinterpret_cast<double2*>(delta) + base;
  for (int idx = lane; idx < cnt; idx += 64) D[idx] = ts[idx];
  if (live && bad) atomicOr(err, ERR_SINGULAR);
  if (nonfinite) atomicOr(err, ERR_NONFINITE);
}

int self_consistency_parts(int nk) { return nk < kScParts ? nk : kScParts; }

hipError_t launch_self_consistency(int nk, int nc, int nw, int nb_uniform, const int32_t* nb, const int64_t* off_b,
                                   const double* eps, const double* wk, const double* proj, const double* e_dc,
                                   double beta, double mu, const double* gloc, const double* sigma, double* e_imp,
                                   double* delta, double* part, int* err, hipStream_t s) {
  const int np = self_consistency_parts(nk);
  hipLaunchKernelGGL(eimp_partial_kernel, dim3(np), dim3(256), 0, s, nk, nc, nb_uniform, nb, off_b, eps, wk, proj,
                     part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(eimp_reduce_kernel, dim3(nc * nc), dim3(256), 0, s, nc, np, part, e_dc, e_imp);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(delta_kernel, dim3((nw + 3) / 4), dim3(64), 0, s, nw, nc, beta, mu, gloc, sigma, e_imp, delta,
                     err);
  return hipGetLastError();
}

}  // namespace dmft
