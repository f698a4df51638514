// HIP kernels of the lattice Dyson step that are not size-specialised: the
// dispatch of the size-specialised Dyson kernel (dyson_impl.h, instantiated in
// dyson_16.hip, dyson_32.hip, dyson_48.hip) and the fixed-order reductions and
// epilogues that turn its partial sums into N(k), G_loc and the scalars.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dmft_internal.h"

namespace dmft {

hipError_t launch_dyson_16(int var, const DysonArgs& a, dim3 grid, hipStream_t s);
hipError_t launch_dyson_32(int var, const DysonArgs& a, dim3 grid, hipStream_t s);
hipError_t launch_dyson_48(int var, const DysonArgs& a, dim3 grid, hipStream_t s);
hipError_t launch_dyson_64(int var, const DysonArgs& a, dim3 grid, hipStream_t s);
int variants_64(int kind, int* out, int max);
int variants_16(int kind, int* out, int max);
int variants_32(int kind, int* out, int max);
int variants_48(int kind, int* out, int max);
hipError_t launch_lowrank(int nbp, int var, const DysonArgs& a, dim3 grid, hipStream_t s);
int lowrank_variants(int nbp, int kind, int* out, int max);
bool dyson_supported(int nbp);

// Dense variants first (the first one is the default), then the low-rank ones.
// Kinds 2 (fused scalar adjoint) and 3 (general vector-Jacobian product): the
// low-rank variants first, then code 0 for the dense adjoint kernel, which
// exists up to 48 bands.
int dyson_variants(int nbp, int kind, int* out, int max) {
  if (kind == 2 || kind == 3) {
    int n = lowrank_variants(nbp, kind, out, max);
    if (nbp <= 48 && dyson_supported(nbp) && n < max) out[n++] = 0;
    return n;
  }
  int n = 0;
  switch (nbp) {
    case 16: n = variants_16(kind, out, max); break;
    case 32: n = variants_32(kind, out, max); break;
    case 48: n = variants_48(kind, out, max); break;
    case 64: n = variants_64(kind, out, max); break;
    default: return 0;
  }
  return n + lowrank_variants(nbp, kind, out + n, max - n);
}

bool dyson_supported(int nbp) { return nbp == 16 || nbp == 32 || nbp == 48 || nbp == 64; }

hipError_t launch_dyson(int nbp, int var, const DysonArgs& a, int n_ktiles, hipStream_t s) {
  dim3 grid((unsigned)(n_ktiles * a.n_wtiles));
  if (var & 8) return launch_lowrank(nbp, var, a, grid, s);
  switch (nbp) {
    case 16: return launch_dyson_16(var, a, grid, s);
    case 32: return launch_dyson_32(var, a, grid, s);
    case 48: return launch_dyson_48(var, a, grid, s);
    case 64: return launch_dyson_64(var, a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

// ----------------------------------------------------------------------------- epilogues

// Fixed-order sum of a block's values (blockDim.x is a power of two, <= 256).
__device__ double block_sum(double v, double* red) {
  int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// N(k) = 1/2 I - (beta/4) M1 + (1/beta)[Ssum + Ssum^dag + 2 s2 M1]  (tail_order 2)
// with Ssum the frequency sum of G, M1 = diag(E) - mu + S^dag (Sigma_inf - V_DC) S.
// Also the per-k scalars tr N, tr(S N S^dag), sum_v E_v N_vv.
__global__ void __launch_bounds__(256) nk_epilogue_kernel(EpilogueArgs a, double* nk_out) {
  __shared__ double2 vinf[16 * 64];  // (Sigma_inf - V_DC) S   (nc x nb)
  __shared__ double2 ps[16 * 64];    // S of the k-point (nc x nb), read nc times per element below
  __shared__ double red[256];
  const int k = blockIdx.x;
  const int nc = a.nc;
  const int nb = a.nb_uniform > 0 ? a.nb_uniform : a.nb[k];
  const int64_t ob = a.nb_uniform > 0 ? (int64_t)k * nb : a.off_b[k];
  const int64_t on = a.nb_uniform > 0 ? (int64_t)k * nb * nb : a.off_n[k];
  const int T = (a.nb_uniform > 0 ? (a.nb_uniform + 15) / 16 * 16 : a.nbp[k]) / 16;
  const double* eps = a.eps + ob;
  const double2* P = reinterpret_cast<const double2*>(a.proj) + ob * nc;
  const double2* sinf = reinterpret_cast<const double2*>(a.sigma_inf);
  const double mu = a.mu_ptr ? *a.mu_ptr : a.mu;
  const double beta = a.beta;
  const bool tail = a.tail_order == 2;
  for (int idx = threadIdx.x; idx < nc * nb; idx += blockDim.x) ps[idx] = P[idx];
  __syncthreads();
  for (int idx = threadIdx.x; idx < nc * nb; idx += blockDim.x) {
    int al = idx / nb, c = idx % nb;
    double2 acc = make_double2(0.0, 0.0);
    for (int be = 0; be < nc; ++be) {
      double2 m = sinf ? sinf[al * nc + be] : make_double2(0.0, 0.0);
      if (al == be) m.x -= a.e_dc[al];
      double2 p = ps[be * nb + c];
      acc.x += m.x * p.x - m.y * p.y;
      acc.y += m.x * p.y + m.y * p.x;
    }
    vinf[al * nb + c] = acc;
  }
  __syncthreads();
  auto ssum = [&](int r, int c) {
    int t = r >> 4, i = (r >> 2) & 3, q = r & 3, b = c >> 4, c16 = c & 15;
    int e = (t * T + b) * 4 + i, lane = q * 16 + c16;
    double2 acc = make_double2(0.0, 0.0);
    const double2* sp = reinterpret_cast<const double2*>(a.spart);
    for (int w = 0; w < a.n_wtiles; ++w) {
      double2 v = sp[(int64_t)w * a.s_stride + a.off_s[k] + e * 64 + lane];
      acc.x += v.x;
      acc.y += v.y;
    }
    return acc;
  };
  double tr = 0.0, hks = 0.0, ncor = 0.0;
  // one thread per pair (r <= c): the two frequency sums it needs, Ssum[r][c]
  // and Ssum[c][r], are read once for both elements
  for (int idx = threadIdx.x; idx < nb * nb; idx += blockDim.x) {
    const int r0 = idx / nb, c0 = idx % nb;
    if (r0 > c0) continue;
    const double2 s_rc = ssum(r0, c0), s_cr = r0 == c0 ? s_rc : ssum(c0, r0);
    for (int e = 0; e < (r0 == c0 ? 1 : 2); ++e) {
      const int r = e ? c0 : r0, c = e ? r0 : c0;
      const double2 s1 = e ? s_cr : s_rc, s2 = e ? s_rc : s_cr;
      double2 m1 = make_double2(r == c ? eps[r] - mu : 0.0, 0.0);
      double2 qcr = make_double2(0.0, 0.0);  // (S^dag S)[c][r]
      for (int al = 0; al < nc; ++al) {
        double2 pr = ps[al * nb + r];
        double2 v = vinf[al * nb + c];
        m1.x += pr.x * v.x + pr.y * v.y;  // conj(S[al][r]) * V[al][c]
        m1.y += pr.x * v.y - pr.y * v.x;
        double2 pc = ps[al * nb + c];
        qcr.x += pc.x * pr.x + pc.y * pr.y;  // conj(S[al][c]) * S[al][r]
        qcr.y += pc.x * pr.y - pc.y * pr.x;
      }
      double2 nv;
      nv.x = (s1.x + s2.x) / beta;
      nv.y = (s1.y - s2.y) / beta;
      if (r == c) nv.x += 0.5;
      if (tail) {
        nv.x += -0.25 * beta * m1.x + 2.0 * a.s2 * m1.x / beta;
        nv.y += -0.25 * beta * m1.y + 2.0 * a.s2 * m1.y / beta;
      }
      if (nk_out) reinterpret_cast<double2*>(nk_out)[on + r * nb + c] = nv;
      if (r == c) {
        tr += nv.x;
        hks += eps[r] * nv.x;
      }
      ncor += nv.x * qcr.x - nv.y * qcr.y;
    }
  }
  tr = block_sum(tr, red);
  ncor = block_sum(ncor, red);
  hks = block_sum(hks, red);
  if (threadIdx.x == 0) {
    a.kscal[k * 3 + 0] = tr;
    a.kscal[k * 3 + 1] = ncor;
    a.kscal[k * 3 + 2] = hks;
  }
}

// Per-k tr N(k) and d tr N(k) / dmu from the frequency sums of Re tr G, Re tr G^2.
__global__ void __launch_bounds__(64) trace_epilogue_kernel(EpilogueArgs a) {
  __shared__ double red[64];
  const int k = blockIdx.x;
  const int nc = a.nc;
  const int nb = a.nb_uniform > 0 ? a.nb_uniform : a.nb[k];
  const int64_t ob = a.nb_uniform > 0 ? (int64_t)k * nb : a.off_b[k];
  const double* eps = a.eps + ob;
  const double2* P = reinterpret_cast<const double2*>(a.proj) + ob * nc;
  const double2* sinf = reinterpret_cast<const double2*>(a.sigma_inf);
  const double mu = a.mu_ptr ? *a.mu_ptr : a.mu;
  const double beta = a.beta;
  // tr M1 = sum_v (E_v - mu) + sum_{al,be} (Sigma_inf - V_DC)[al][be] (S S^dag)[be][al]
  double trm = 0.0;
  for (int v = threadIdx.x; v < nb; v += blockDim.x) {
    trm += eps[v] - mu;
    for (int al = 0; al < nc; ++al)
      for (int be = 0; be < nc; ++be) {
        double2 m = sinf ? sinf[al * nc + be] : make_double2(0.0, 0.0);
        if (al == be) m.x -= a.e_dc[al];
        double2 pb = P[be * nb + v], pa = P[al * nb + v];
        double2 ss = make_double2(pb.x * pa.x + pb.y * pa.y, pb.y * pa.x - pb.x * pa.y);  // S[be][v] conj(S[al][v])
        trm += m.x * ss.x - m.y * ss.y;
      }
  }
  trm = block_sum(trm, red);
  if (threadIdx.x == 0) {
    double trg = 0.0, trg2 = 0.0;
    for (int w = 0; w < a.n_wtiles; ++w) {
      trg += a.tpart[((int64_t)w * a.nk + k) * 2 + 0];
      trg2 += a.tpart[((int64_t)w * a.nk + k) * 2 + 1];
    }
    double tr = 0.5 * nb + 2.0 * trg / beta;
    double d = -2.0 * trg2 / beta;
    if (a.tail_order == 2) {
      tr += -0.25 * beta * trm + 2.0 * a.s2 * trm / beta;
      d += 0.25 * beta * nb - 2.0 * a.s2 * nb / beta;
    }
    a.ktrace[k * 2 + 0] = tr;
    a.ktrace[k * 2 + 1] = d;
  }
}

// Per-k [tr N, d tr N/dmu, mubar_k] from the adjoint kernel's [n_wtiles][nk][3]
// partials; mubar_k gets the tail term (beta/4 - 2 s2/beta) Re tr Nbar_k.
__global__ void __launch_bounds__(64) adj_epilogue_kernel(EpilogueArgs a, const double* nbar) {
  __shared__ double red[64];
  const int k = blockIdx.x;
  const int nc = a.nc;
  const int nb = a.nb_uniform > 0 ? a.nb_uniform : a.nb[k];
  const int64_t ob = a.nb_uniform > 0 ? (int64_t)k * nb : a.off_b[k];
  const int64_t on = a.nb_uniform > 0 ? (int64_t)k * nb * nb : a.off_n[k];
  const double* eps = a.eps + ob;
  const double2* P = reinterpret_cast<const double2*>(a.proj) + ob * nc;
  const double2* sinf = reinterpret_cast<const double2*>(a.sigma_inf);
  const double mu = a.mu_ptr ? *a.mu_ptr : a.mu;
  const double beta = a.beta;
  double trm = 0.0, trn = 0.0;
  for (int v = threadIdx.x; v < nb; v += blockDim.x) {
    trm += eps[v] - mu;
    for (int al = 0; al < nc; ++al)
      for (int be = 0; be < nc; ++be) {
        double2 m = sinf ? sinf[al * nc + be] : make_double2(0.0, 0.0);
        if (al == be) m.x -= a.e_dc[al];
        double2 pb = P[be * nb + v], pa = P[al * nb + v];
        double2 ss = make_double2(pb.x * pa.x + pb.y * pa.y, pb.y * pa.x - pb.x * pa.y);
        trm += m.x * ss.x - m.y * ss.y;
      }
    if (nbar) trn += reinterpret_cast<const double2*>(nbar)[on + (int64_t)v * nb + v].x;
  }
  trm = block_sum(trm, red);
  trn = block_sum(trn, red);
  if (threadIdx.x == 0) {
    double trg = 0.0, trg2 = 0.0, mub = 0.0;
    for (int w = 0; w < a.n_wtiles; ++w) {
      const double* tp = a.tpart + ((int64_t)w * a.nk + k) * 3;
      trg += tp[0];
      trg2 += tp[1];
      mub += tp[2];
    }
    double tr = 0.5 * nb + 2.0 * trg / beta;
    double d = -2.0 * trg2 / beta;
    if (a.tail_order == 2) {
      tr += -0.25 * beta * trm + 2.0 * a.s2 * trm / beta;
      d += 0.25 * beta * nb - 2.0 * a.s2 * nb / beta;
      mub += (0.25 * beta - 2.0 * a.s2 / beta) * trn;
    }
    a.kscal[k * 3 + 0] = tr;
    a.kscal[k * 3 + 1] = d;
    a.kscal[k * 3 + 2] = mub;
  }
}

hipError_t launch_adj_epilogue(const EpilogueArgs& a, const double* nbar, hipStream_t s) {
  hipLaunchKernelGGL(adj_epilogue_kernel, dim3(a.nk), dim3(64), 0, s, a, nbar);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) gloc_reduce_kernel(int n_ktiles, int nw, int nc, const double* xpart,
                                                          double* gloc) {
  int n = blockIdx.x;
  int e = threadIdx.x;  // i * 64 + lane
  int i = e >> 6, lane = e & 63, q = lane >> 4, c16 = lane & 15;
  int al = q + 4 * i, be = c16;
  if (al >= nc || be >= nc) return;
  const double2* xp = reinterpret_cast<const double2*>(xpart);
  double2 acc = make_double2(0.0, 0.0);
  for (int kt = 0; kt < n_ktiles; ++kt) {
    double2 v = xp[((int64_t)kt * nw + n) * 256 + e];
    acc.x += v.x;
    acc.y += v.y;
  }
  reinterpret_cast<double2*>(gloc)[((int64_t)n * nc + al) * nc + be] = acc;
}

__global__ void __launch_bounds__(256) scalar_reduce_kernel(int nk, const double* wk, const double* kvals,
                                                            int nvals, int unit_mask, double* out) {
  __shared__ double red[256];
  for (int j = 0; j < nvals; ++j) {
    double acc = 0.0;
    const bool unit = (unit_mask >> j) & 1;
    for (int k = threadIdx.x; k < nk; k += blockDim.x) acc += (unit ? 1.0 : wk[k]) * kvals[(int64_t)k * nvals + j];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) out[j] = acc;
  }
}

__global__ void fill_zero_kernel(uint32_t* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

hipError_t launch_nk_epilogue(const EpilogueArgs& a, double* nk_out, hipStream_t s) {
  hipLaunchKernelGGL(nk_epilogue_kernel, dim3(a.nk), dim3(256), 0, s, a, nk_out);
  return hipGetLastError();
}

hipError_t launch_trace_epilogue(const EpilogueArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(trace_epilogue_kernel, dim3(a.nk), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gloc_reduce(int n_ktiles, int nw, int nc, const double* xpart, double* gloc, hipStream_t s) {
  hipLaunchKernelGGL(gloc_reduce_kernel, dim3(nw), dim3(256), 0, s, n_ktiles, nw, nc, xpart, gloc);
  return hipGetLastError();
}

hipError_t launch_scalar_reduce(int nk, const double* wk, const double* kvals, int nvals, double* out,
                                hipStream_t s) {
  hipLaunchKernelGGL(scalar_reduce_kernel, dim3(1), dim3(256), 0, s, nk, wk, kvals, nvals, 0, out);
  return hipGetLastError();
}

hipError_t launch_scalar_reduce_mask(int nk, const double* wk, const double* kvals, int nvals, int unit_mask,
                                     double* out, hipStream_t s) {
  hipLaunchKernelGGL(scalar_reduce_kernel, dim3(1), dim3(256), 0, s, nk, wk, kvals, nvals, unit_mask, out);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  size_t n = bytes / 4;
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint32_t*)p, n);
  return hipGetLastError();
}

}  // namespace dmft
