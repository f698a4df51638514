// DMFT self-consistency step that consumes G_loc (Sec. 3.2.2 eq. dmftloop2):
//
//     E_imp        = sum_k w_k S_k diag(E_k) S_k^dag - diag(V_DC)
//     Delta(i w_n) = i w_n + mu - E_imp - Sigma(i w_n) - G_loc(i w_n)^-1 .
//
// E_imp: one work-group per (alpha, beta) entry, a fixed-order sum over k.
// Delta: one wavefront per four frequencies; lane 16 g + i holds row i of
// G_loc(i w_{4b+g}) and the inversion is the row-layout Gauss-Jordan sweep of
// the low-rank kernel (no pivoting: the anti-Hermitian part of G_loc(i w_n),
// -sum_k w_k S G (w_n + Im parts) G^dag S^dag, is negative definite for
// w_n > 0, so every leading block is invertible).
#include "lowrank_impl.h"

namespace dmft {

// Fixed-order sum of a block's values (blockDim.x = 256).
__device__ __forceinline__ double sc_block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(256) eimp_kernel(int nk, int nc, int nb_uniform, const int32_t* nb,
                                                   const int64_t* off_b, const double* eps, const double* wk,
                                                   const double* proj, const double* e_dc, double* e_imp) {
  __shared__ double red[256];
  const int al = blockIdx.x / nc, be = blockIdx.x % nc;
  const double2* P = reinterpret_cast<const double2*>(proj);
  double sr = 0.0, si = 0.0;
  for (int k = threadIdx.x; k < nk; k += blockDim.x) {
    const int n = nb_uniform > 0 ? nb_uniform : nb[k];
    const int64_t ob = nb_uniform > 0 ? (int64_t)k * n : off_b[k];
    const double2* pk = P + ob * nc;
    double ar = 0.0, ai = 0.0;
    for (int r = 0; r < n; ++r) {
      const double2 x = pk[al * n + r], y = pk[be * n + r];
      const double e = eps[ob + r];
      // S[al][r] E_r conj(S[be][r])
      ar += e * (x.x * y.x + x.y * y.y);
      ai += e * (x.y * y.x - x.x * y.y);
    }
    sr += wk[k] * ar;
    si += wk[k] * ai;
  }
  sr = sc_block_sum(sr, red);
  si = sc_block_sum(si, red);
  if (threadIdx.x == 0) {
    if (al == be) sr -= e_dc[al];
    reinterpret_cast<double2*>(e_imp)[al * nc + be] = make_double2(sr, si);
  }
}

__global__ void __launch_bounds__(64) delta_kernel(int nw, int nc, double beta, double mu, const double* gloc,
                                                   const double* sigma, const double* e_imp, double* delta,
                                                   int* err) {
  const int lane = threadIdx.x, g = lane >> 4, i = lane & 15;
  const int n = 4 * blockIdx.x + g;
  const bool live = n < nw;
  const double2* G = reinterpret_cast<const double2*>(gloc) + (int64_t)(live ? n : 0) * nc * nc;
  double rr[16], ri[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    double2 v = (i < nc && j < nc) ? G[i * nc + j] : make_double2(0.0, 0.0);
    if (!live) v = make_double2(i == j ? 1.0 : 0.0, 0.0);  // keeps the idle rows' pivots nonzero
    rr[j] = v.x;
    ri[j] = v.y;
  }
  int bad = 0;
  rsweep<0, 16>(rr, ri, i, nc, bad);
  int nonfinite = 0;
  if (live && i < nc) {
    const double wn = (double)(2 * n + 1) * M_PI / beta;
    const double2* S = reinterpret_cast<const double2*>(sigma) + (int64_t)n * nc * nc;
    const double2* E = reinterpret_cast<const double2*>(e_imp);
    double2* D = reinterpret_cast<double2*>(delta) + (int64_t)n * nc * nc;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (j < nc) {
        const double2 s = S[i * nc + j], e = E[i * nc + j];
        double2 v = make_double2(-e.x - s.x - rr[j], -e.y - s.y - ri[j]);
        if (j == i) {
          v.x += mu;
          v.y += wn;
        }
        if (!__builtin_isfinite(v.x) || !__builtin_isfinite(v.y)) nonfinite = 1;
        D[i * nc + j] = v;
      }
    }
  }
  if (live && bad) atomicOr(err, ERR_SINGULAR);
  if (nonfinite) atomicOr(err, ERR_NONFINITE);
}

hipError_t launch_self_consistency(int nk, int nc, int nw, int nb_uniform, const int32_t* nb, const int64_t* off_b,
                                   const double* eps, const double* wk, const double* proj, const double* e_dc,
                                   double beta, double mu, const double* gloc, const double* sigma, double* e_imp,
                                   double* delta, int* err, hipStream_t s) {
  hipLaunchKernelGGL(eimp_kernel, dim3(nc * nc), dim3(256), 0, s, nk, nc, nb_uniform, nb, off_b, eps, wk, proj, e_dc,
                     e_imp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(delta_kernel, dim3((nw + 3) / 4), dim3(64), 0, s, nw, nc, beta, mu, gloc, sigma, e_imp, delta,
                     err);
  return hipGetLastError();
}

}  // namespace dmft
