// Hubbard-I atom and the pole form of its self-energy (Sec. 3.2.4 eqs. Dyson
// and G_imp_atom; appendix eq. dyson_pole), batched over atoms, and the
// Matsubara-axis self-energy of a pole form (Sec. 3.2.4 eq. se_pole).
//
// Interaction H_U = (U/2) sum_{a != b} n_a n_b (eq. H_U of Sec. 3.2.3 at J = 0),
// one-body levels e_a, energies from the chemical potential mu:
//     E(Gamma) = sum_{a in Gamma} (e_a - mu) + U N (N - 1) / 2,  X = exp(-beta E) / Z.
// Fock states are eigenstates and f_a connects Gamma to Gamma + a only, so
// G_aa(i w) = sum_N V_N / (i w - P_N) with P_N = e_a - mu + U N and
// V_N = sum_{Gamma: a empty, N electrons} X(Gamma) + X(Gamma + a).
// Appendix: Sigma_inf = mu - e_a + sum V_N P_N; the self-energy poles Q lie one
// between each pair of adjacent G poles, at the zeros of sum V_N / (Q - P_N)
// (bisection: the sum falls from +inf to -inf there), with weights
// W = [sum V_N / (Q - P_N)^2]^-1.  G poles of weight <= wtol are dropped and
// the rest renormalised (a pole of weight V has its self-energy partner within
// about V of it).  Pole positions are returned on the absolute energy axis,
// p = Q + mu, as the pseudo-Hamiltonian of Sec. 3.3 takes them.
#include <math.h>

#include "dmft_internal.h"

namespace dmft {
namespace {

constexpr int kAtomThreads = 256;

template <int NT>
__device__ __forceinline__ double atom_block_reduce(double v, double* red, bool take_min) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = take_min ? fmin(red[t], red[t + s]) : red[t] + red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// One work-group per (atom, orbital a).
__global__ void __launch_bounds__(kAtomThreads) hubbard1_kernel(int nc, const double* eps, const double* Uv,
                                                                const double* muv, double beta, double wtol,
                                                                double* sigma_inf, int32_t* npoles, double* pos,
                                                                double* wgt, double* occ, double* e_u) {
  __shared__ double red[kAtomThreads];
  __shared__ double sP[16], sV[16];
  __shared__ int s_nr;
  const int atom = blockIdx.x / nc, a = blockIdx.x - atom * nc, t = threadIdx.x;
  const double* e = eps + (int64_t)atom * nc;
  const double U = Uv[atom], mu = muv[atom];
  const int nstates = 1 << nc;
  auto energy = [&](int g) {
    double s = 0.0;
    for (int b = 0; b < nc; ++b)
      if ((g >> b) & 1) s += e[b] - mu;
    const int n = __popc(g);
    return s + 0.5 * U * n * (n - 1);
  };
  double emin = INFINITY;
  for (int g = t; g < nstates; g += kAtomThreads) emin = fmin(emin, energy(g));
  emin = atom_block_reduce<kAtomThreads>(emin, red, true);
  const double ea = e[a] - mu;
  double z = 0.0, hu = 0.0, na = 0.0, acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.0;
  for (int g = t; g < nstates; g += kAtomThreads) {
    const double eg = energy(g);
    const int n = __popc(g);
    const double x = exp(-beta * (eg - emin));
    z += x;
    hu += x * 0.5 * U * n * (n - 1);
    if ((g >> a) & 1) {
      na += x;
    } else {
      // Gamma + a has energy E(Gamma) + (e_a - mu) + U N
      const double v = x + exp(-beta * (eg + ea + U * n - emin));
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] += (j == n) ? v : 0.0;
    }
  }
  z = atom_block_reduce<kAtomThreads>(z, red, false);
  hu = atom_block_reduce<kAtomThreads>(hu, red, false);
  na = atom_block_reduce<kAtomThreads>(na, red, false);
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (j < nc) acc[j] = atom_block_reduce<kAtomThreads>(acc[j], red, false);
  const int64_t o = (int64_t)atom * nc + a;
  if (t == 0) {
    // retained G poles in ascending position (equal positions merged: U = 0)
    int nr = 0;
    double vsum = 0.0;
    for (int j = 0; j < nc; ++j) {
      const double v = acc[j] / z;
      if (!(v > wtol)) continue;
      const double p = ea + U * j;
      int at = nr;
      while (at > 0 && sP[at - 1] > p) --at;
      if (at > 0 && sP[at - 1] == p) {
        sV[at - 1] += v;
      } else {
        for (int m = nr; m > at; --m) {
          sP[m] = sP[m - 1];
          sV[m] = sV[m - 1];
        }
        sP[at] = p;
        sV[at] = v;
        ++nr;
      }
      vsum += v;
    }
    double first = 0.0;
    for (int m = 0; m < nr; ++m) {
      sV[m] /= vsum;
      first += sV[m] * sP[m];
    }
    s_nr = nr;
    sigma_inf[o] = mu - e[a] + first;
    npoles[o] = nr > 0 ? nr - 1 : 0;
    if (occ) occ[o] = na / z;
    if (e_u && a == 0) e_u[atom] = hu / z;
  }
  __syncthreads();
  const int nr = s_nr;
  if (t < nr - 1) {
    double lo = sP[t], hi = sP[t + 1];
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (!(mid > lo && mid < hi)) break;
      double gsum = 0.0;
      for (int m = 0; m < nr; ++m) gsum += sV[m] / (mid - sP[m]);
      if (gsum > 0.0) lo = mid;
      else hi = mid;
    }
    const double q = 0.5 * (lo + hi);
    double d = 0.0;
    for (int m = 0; m < nr; ++m) {
      const double r = q - sP[m];
      d += sV[m] / (r * r);
    }
    pos[o * nc + t] = q + mu;
    wgt[o * nc + t] = 1.0 / d;
  }
  for (int j = t; j < nc; j += kAtomThreads)
    if (j >= nr - 1 || nr == 0) {
      pos[o * nc + j] = 0.0;
      wgt[o * nc + j] = 0.0;
    }
}

// Sigma(i w_n)_ab = Sigma_inf_ab + sum_i conj(v_ia) v_ib / (i w_n + mu - p_i), one
// thread per (n, a, b).
__global__ void sigma_from_poles_kernel(int nw, int nc, int np, double beta, double mu, const double* p,
                                        const double* v, const double* sinf, double* sigma) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nw * nc * nc;
  if (idx >= total) return;
  const int n = (int)(idx / (nc * nc));
  const int ab = (int)(idx - (int64_t)n * nc * nc);
  const int a = ab / nc, b = ab - a * nc;
  const double wn = (double)(2 * n + 1) * M_PI / beta;
  const double2* V = reinterpret_cast<const double2*>(v);
  double2 s = sinf ? reinterpret_cast<const double2*>(sinf)[ab] : make_double2(0.0, 0.0);
  for (int i = 0; i < np; ++i) {
    const double2 va = V[i * nc + a], vb = V[i * nc + b];
    // conj(va) vb
    const double nr = va.x * vb.x + va.y * vb.y, ni = va.x * vb.y - va.y * vb.x;
    // 1 / (x + i wn), x = mu - p_i
    const double x = mu - p[i];
    const double den = 1.0 / (x * x + wn * wn);
    const double rr = x * den, ri = -wn * den;
    s.x += nr * rr - ni * ri;
    s.y += nr * ri + ni * rr;
  }
  reinterpret_cast<double2*>(sigma)[idx] = s;
}

// Pole list of one atom in the dmft_poles layout: pole (a, j) of the atom's
// orbital a becomes position pos[a][j] with vector sqrt(wgt[a][j]) e_{a0 + a}
// among nc_lat correlated orbitals; poles are packed orbital after orbital.
__global__ void hubbard1_poles_kernel(int nc, int nc_lat, int a0, const int32_t* npoles, const double* pos,
                                      const double* wgt, double* p, double* v, int32_t* np_out) {
  __shared__ int off[17];
  const int t = threadIdx.x;
  if (t == 0) {
    off[0] = 0;
    for (int a = 0; a < nc; ++a) off[a + 1] = off[a] + min(max(npoles[a], 0), nc - 1);
    *np_out = off[nc];
  }
  __syncthreads();
  double2* V = reinterpret_cast<double2*>(v);
  for (int idx = t; idx < nc * nc; idx += blockDim.x) {
    const int a = idx / nc, j = idx - a * nc;
    if (j >= min(max(npoles[a], 0), nc - 1)) continue;
    const int i = off[a] + j;
    p[i] = pos[a * nc + j];
    for (int b = 0; b < nc_lat; ++b) V[(int64_t)i * nc_lat + b] = make_double2(b == a0 + a ? sqrt(wgt[a * nc + j]) : 0.0, 0.0);
  }
}

}  // namespace

hipError_t launch_hubbard1(int natoms, int nc, const double* eps, const double* U, const double* mu, double beta,
                           double wtol, double* sigma_inf, int32_t* npoles, double* pos, double* wgt, double* occ,
                           double* e_u, hipStream_t s) {
  hipLaunchKernelGGL(hubbard1_kernel, dim3(natoms * nc), dim3(kAtomThreads), 0, s, nc, eps, U, mu, beta, wtol,
                     sigma_inf, npoles, pos, wgt, occ, e_u);
  return hipGetLastError();
}

hipError_t launch_sigma_from_poles(int nw, int nc, int np, double beta, double mu, const double* p, const double* v,
                                   const double* sinf, double* sigma, hipStream_t s) {
  const int64_t total = (int64_t)nw * nc * nc;
  hipLaunchKernelGGL(sigma_from_poles_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, nw, nc, np,
                     beta, mu, p, v, sinf, sigma);
  return hipGetLastError();
}

hipError_t launch_hubbard1_poles(int nc, int nc_lat, int a0, const int32_t* npoles, const double* pos,
                                 const double* wgt, double* p, double* v, int32_t* np_out, hipStream_t s) {
  hipLaunchKernelGGL(hubbard1_poles_kernel, dim3(1), dim3(256), 0, s, nc, nc_lat, a0, npoles, pos, wgt, p, v, np_out);
  return hipGetLastError();
}

}  // namespace dmft
