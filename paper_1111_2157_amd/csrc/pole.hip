// Pole-expansion route of the lattice step (Sec. 3.3 eqs. pseudo_H_k,
// rho_LDA+DMFT_componet_final and fix_mu; Sec. 3.5.2 eqs. DOS and PDOS).
//
// When Sigma has the pole form of Sec. 3.2.4 eq. se_pole,
//     Sigma(i w) = Sigma_inf + sum_i V_i^dag V_i / (i w - p_i),
// the band-window resolvent is the physical block of (i w - H_ps)^-1 with
//     H_ps(k) = [[ diag(E_k) + S^dag (Sigma_inf - V_DC) S,  -(V S)^dag ],
//                [ -(V S),                                  diag(p)    ]]
// (one row of V S per pole), so with H_ps = Psi diag(E^ps) Psi^dag and
// u_l = <phi|psi_l> the physical part of eigenvector l:
//     N(k)   = sum_l u_l u_l^dag n_F(E^ps_l - mu)            (no frequency sum)
//     N_tot  = sum_k w_k sum_l |u_l|^2 n_F(E^ps_l - mu)
//     D(e)   = sum_k w_k sum_l |u_l|^2 L(e + mu - E^ps_l),   L(x) = (eta/pi) / (x^2 + eta^2)
//     D_a(e) = sum_k w_k sum_l |S_a u_l|^2 L(e + mu - E^ps_l).
// The eigensystems do not depend on mu, so once they are known every further
// N(mu) costs O(Nk (Nb + np)).
//
// Eigensolver: one work-group per k, the matrix (upper triangle, packed) and
// the physical rows of the eigenvectors resident in LDS (m = nb + np <= 80),
// cyclic two-sided Jacobi for complex Hermitian matrices in the round-robin
// (tournament) order: in each of the m-1 steps of a sweep the m/2 disjoint
// index pairs rotate at once.  A step is one pass over the 2x2 blocks of the
// matrix, A <- U^dag A U with U block-diagonal in the step's pairing, computed
// for the blocks on and above the diagonal (each stored element belongs to
// exactly one of them), plus the same column rotation of the eigenvector rows.  A pair rotates when
// |a_pq| > 1e-17 ||A||_F; the sweep that rotates nothing ends the iteration.
// The rotation for a pair: with a_pq = r e^{i phi}, zeta = (a_qq - a_pp) / 2r,
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2),
// sigma = t c e^{i phi}, U = [[c, sigma], [-conj(sigma), c]] zeroes a_pq and
// moves the diagonal to a_pp - t r, a_qq + t r (the phase-reduced form of the
// real symmetric 2x2 Jacobi rotation).
#include <math.h>

#include "dmft_internal.h"

namespace dmft {
namespace {

constexpr int kMaxM = 80;         // largest pseudo-Hamiltonian (nb + np)
constexpr int kDosThreads = 256;
constexpr int kDosChunk = 512;    // eigenpairs per slice of the DOS sum
constexpr int kMaxSlices = 128;

__device__ __forceinline__ double2 pz(double r, double i) { return make_double2(r, i); }
__device__ __forceinline__ double2 pconj(double2 a) { return pz(a.x, -a.y); }
__device__ __forceinline__ double2 padd(double2 a, double2 b) { return pz(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 psub(double2 a, double2 b) { return pz(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 pscal(double s, double2 a) { return pz(s * a.x, s * a.y); }
__device__ __forceinline__ double2 pmul(double2 a, double2 b) {
  return pz(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 pfma(double2 a, double2 b, double2 c) {  // c + a b
  return pz(__builtin_fma(a.x, b.x, __builtin_fma(-a.y, b.y, c.x)), __builtin_fma(a.x, b.y, __builtin_fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double pabs2(double2 a) { return a.x * a.x + a.y * a.y; }
// 1/sqrt(x) and 1/x: the hardware estimates refined by two Newton steps
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = x * y;
  y = __builtin_fma(0.5 * y, __builtin_fma(-h, y, 1.0), y);
  h = x * y;
  return __builtin_fma(0.5 * y, __builtin_fma(-h, y, 1.0), y);
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
  return __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
}

// Fixed-order sum over a block of NT threads (NT a power of two).
template <int NT>
__device__ __forceinline__ double pole_block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// n_F(x) = 1 / (exp(beta x) + 1) without overflow.
__device__ __forceinline__ double fermi(double x, double beta) {
  const double y = beta * x;
  if (y > 0.0) {
    const double e = exp(-y);
    return e / (1.0 + e);
  }
  return 1.0 / (1.0 + exp(y));
}

// Weight of one level at x in the positive-frequency Matsubara sum truncated at
// nw frequencies with the analytic 1/(iw) and 1/(iw)^2 tails (the density of the
// frequency-sum route at that nw): 1/2 - beta x / 4 + (2/beta) sum_n x^3 / (w_n^2 (w_n^2 + x^2)).
__device__ double truncated_weight(double x, double beta, int nw) {
  const double x2 = x * x, x3 = x2 * x;
  double s = 0.0;
  for (int n = 0; n < nw; ++n) {
    const double w = (double)(2 * n + 1) * M_PI / beta;
    const double w2 = w * w;
    s += x3 / (w2 * (w2 + x2));
  }
  return 0.5 - beta * x / 4.0 + 2.0 * s / beta;
}

// One pair's rotation of a Jacobi step, read by the update pass as two 16-byte words.
struct __align__(16) JRot {
  double c, sr, si;  // U = [[c, g], [-conj(g), c]], g = sr + i si
  int pq;            // p | q << 16
  int rot;           // 0: identity (the pair is already diagonal)
};

// The Hermitian matrix keeps its upper triangle only, packed by rows: element
// (r, c), r <= c, of an mq x mq matrix sits at r mq - r (r - 1) / 2 + c - r;
// (c, r) is its conjugate.  hget/hput pick the stored element and conjugate by
// select, so lanes reading either triangle do not diverge.
__device__ __forceinline__ int up_idx(int r, int c, int mq) { return r * mq - ((r * (r - 1)) >> 1) + (c - r); }
__device__ __forceinline__ double2 hget(const double2* A, int r, int c, int mq) {
  const double2 v = A[up_idx(min(r, c), max(r, c), mq)];
  return pz(v.x, r <= c ? v.y : -v.y);
}
__device__ __forceinline__ void hput(double2* A, int r, int c, int mq, double2 v) {
  A[up_idx(min(r, c), max(r, c), mq)] = pz(v.x, r <= c ? v.y : -v.y);
}

__device__ __forceinline__ void k_window(const PoleArgs& a, int k, int& nb, int64_t& ob) {
  nb = a.nb_uniform > 0 ? a.nb_uniform : a.nb[k];
  ob = a.nb_uniform > 0 ? (int64_t)k * nb : a.off_b[k];
}

// NT threads per work-group (256, 512 or 1024, chosen at launch from the
// number of update items per step).
template <int NT>
__global__ void __launch_bounds__(NT) pole_eig_kernel(PoleArgs a) {
  constexpr int kEigThreads = NT;
  extern __shared__ double2 lds[];
  __shared__ JRot s_r[kMaxM / 2];
  __shared__ double s_dp[kMaxM / 2], s_dq[kMaxM / 2];
  __shared__ int s_inv[kMaxM], s_any[2];
  __shared__ double s_lam[kMaxM];
  __shared__ double red[kEigThreads];
  const int k = blockIdx.x, t = threadIdx.x;
  int nb;
  int64_t ob;
  k_window(a, k, nb, ob);
  const int nc = a.nc, np = a.np;
  const int m = nb + np, mq = m + (m & 1), P = mq >> 1;
  const int ldv = nb + 1;
  double2* A = lds;                          // packed upper triangle, mq (mq + 1) / 2
  double2* VT = lds + mq * (mq + 1) / 2;     // mq x ldv: row l = physical components of eigenvector l
  const double2* S = reinterpret_cast<const double2*>(a.proj) + ob * nc;
  const double* E = a.eps + ob;
  const double2* SI = reinterpret_cast<const double2*>(a.sigma_inf);
  const double2* V = reinterpret_cast<const double2*>(a.v);

  // T = (Sigma_inf - V_DC) S, nc x nb, staged in the eigenvector area
  for (int idx = t; idx < nc * nb; idx += kEigThreads) {
    const int al = idx / nb, j = idx - al * nb;
    double2 acc = pscal(-a.e_dc[al], S[al * nb + j]);
    if (SI)
      for (int be = 0; be < nc; ++be) acc = pfma(SI[al * nc + be], S[be * nb + j], acc);
    VT[idx] = acc;
  }
  __syncthreads();
  // physical block diag(E) + S^dag T (upper triangle, mirrored)
  for (int idx = t; idx < nb * nb; idx += kEigThreads) {
    const int i = idx / nb, j = idx - i * nb;
    if (i > j) continue;
    double2 acc = pz(0.0, 0.0);
    for (int al = 0; al < nc; ++al) acc = pfma(pconj(S[al * nb + i]), VT[al * nb + j], acc);
    if (i == j) acc = pz(E[i] + acc.x, 0.0);
    A[up_idx(i, j, mq)] = acc;
  }
  // coupling rows -V_i S and the pole block diag(p)
  for (int idx = t; idx < np * nb; idx += kEigThreads) {
    const int i = idx / nb, j = idx - i * nb;
    double2 acc = pz(0.0, 0.0);
    for (int al = 0; al < nc; ++al) acc = pfma(V[i * nc + al], S[al * nb + j], acc);
    A[up_idx(j, nb + i, mq)] = pz(-acc.x, acc.y);  // (j, nb + i) = conj of the coupling row
  }
  for (int idx = t; idx < np * np; idx += kEigThreads) {
    const int i = idx / np, j = idx - i * np;
    if (i <= j) A[up_idx(nb + i, nb + j, mq)] = pz(i == j ? a.p[i] : 0.0, 0.0);
  }
  if (m & 1)  // odd size: one decoupled zero row/column completes the pairing
    for (int j = t; j < mq; j += kEigThreads) A[up_idx(j, m, mq)] = pz(0.0, 0.0);
  __syncthreads();
  for (int idx = t; idx < mq * nb; idx += kEigThreads) {
    const int l = idx / nb, i = idx - l * nb;
    VT[l * ldv + i] = pz(l == i ? 1.0 : 0.0, 0.0);
  }
  double ss = 0.0;
  for (int idx = t; idx < mq * mq; idx += kEigThreads) {
    const int i = idx / mq, j = idx - i * mq;
    if (i <= j) ss += (i == j ? 1.0 : 2.0) * pabs2(A[up_idx(i, j, mq)]);
  }
  const double tol = 1e-17 * sqrt(pole_block_sum<kEigThreads>(ss, red));

  // item walks of the two update passes without divisions: item b = t + 256 j
  // is (b / P, b % P) in the block pass and (b / nb, b % nb) in the vector pass
  const int bI0 = t / P, bJ0 = t - bI0 * P, bdI = kEigThreads / P, bdJ = kEigThreads - bdI * P;
  const int vJ0 = t / nb, vi0 = t - vJ0 * nb, vdJ = kEigThreads / nb, vdi = kEigThreads - vdJ * nb;
  int sweep = 0, converged = 0;
  while (sweep < a.max_sweeps) {
    ++sweep;
    int any = 0;
    for (int s = 0; s < mq - 1; ++s) {
      // rotation parameters: pairs live in wave 0 (P <= 32); its ballot tells
      // every wave whether the step rotates (flag double-buffered by step parity,
      // so a wave still reading step s never sees step s + 1's flag)
      if (t < 64) {
        int rot = 0;
        if (t < P) {
          // round-robin: position 0 holds index 0, position j >= 1 index 1 + (j - 1 + s) mod (mq - 1);
          // pair t joins positions t and mq - 1 - t
          const int p = t == 0 ? 0 : 1 + (t - 1 + s) % (mq - 1);
          const int q = 1 + (mq - 2 - t + s) % (mq - 1);
          const double2 apq = hget(A, p, q, mq);
          const double app = A[up_idx(p, p, mq)].x, aqq = A[up_idx(q, q, mq)].x;
          const double r = sqrt(pabs2(apq));
          JRot R;
          R.c = 1.0;
          R.sr = R.si = 0.0;
          R.pq = p | (q << 16);
          if (r > tol) {
            const double ir = rsq_nr(pabs2(apq));
            const double z = 0.5 * (aqq - app) * ir;
            const double az = fabs(z);
            double tt;
            if (az > 1e100) {
              tt = 0.5 / z;  // 1 + z^2 would overflow; t -> 1 / (2 z)
            } else {
              const double z2p1 = __builtin_fma(z, z, 1.0);
              tt = (z >= 0.0 ? 1.0 : -1.0) * rcp_nr(az + z2p1 * rsq_nr(z2p1));
            }
            R.c = rsq_nr(__builtin_fma(tt, tt, 1.0));
            const double sn = tt * R.c * ir;
            R.sr = sn * apq.x;
            R.si = sn * apq.y;
            s_dp[t] = app - tt * r;
            s_dq[t] = aqq + tt * r;
            rot = 1;
          }
          R.rot = rot;
          s_r[t] = R;
        }
        const unsigned long long bal = __ballot(rot);
        if (t == 0) s_any[s & 1] = bal != 0ull;
      }
      __syncthreads();
      if (!s_any[s & 1]) continue;
      any = 1;
      // A <- U^dag A U, one 2x2 block (pair I rows, pair J columns) per item, I <= J
      for (int I = bI0, J = bJ0; I < P;) {
        if (I <= J) {
          const JRot R1 = s_r[I], R2 = s_r[J];
          if (R1.rot | R2.rot) {
            const int p1 = R1.pq & 0xffff, q1 = R1.pq >> 16;
            if (I == J) {
              A[up_idx(p1, p1, mq)] = pz(s_dp[I], 0.0);
              A[up_idx(q1, q1, mq)] = pz(s_dq[I], 0.0);
              hput(A, p1, q1, mq, pz(0.0, 0.0));
            } else {
              const int p2 = R2.pq & 0xffff, q2 = R2.pq >> 16;
              const double c1 = R1.c, c2 = R2.c;
              const double2 g1 = pz(R1.sr, R1.si), g2 = pz(R2.sr, R2.si);
              const double2 x11 = hget(A, p1, p2, mq), x12 = hget(A, p1, q2, mq);
              const double2 x21 = hget(A, q1, p2, mq), x22 = hget(A, q1, q2, mq);
              // rows: p' = c p - g q, q' = conj(g) p + c q
              const double2 y11 = psub(pscal(c1, x11), pmul(g1, x21));
              const double2 y12 = psub(pscal(c1, x12), pmul(g1, x22));
              const double2 y21 = padd(pmul(pconj(g1), x11), pscal(c1, x21));
              const double2 y22 = padd(pmul(pconj(g1), x12), pscal(c1, x22));
              // columns: p' = c p - conj(g) q, q' = g p + c q
              const double2 z11 = psub(pscal(c2, y11), pmul(pconj(g2), y12));
              const double2 z12 = padd(pmul(g2, y11), pscal(c2, y12));
              const double2 z21 = psub(pscal(c2, y21), pmul(pconj(g2), y22));
              const double2 z22 = padd(pmul(g2, y21), pscal(c2, y22));
              // each mirrored pair has one slot, written by this block only
              hput(A, p1, p2, mq, z11);
              hput(A, p1, q2, mq, z12);
              hput(A, q1, p2, mq, z21);
              hput(A, q1, q2, mq, z22);
            }
          }
        }
        I += bdI;
        J += bdJ;
        if (J >= P) {
          J -= P;
          ++I;
        }
      }
      // eigenvector columns (rows of VT): p' = c p - conj(g) q, q' = g p + c q
      for (int J = vJ0, i = vi0; J < P;) {
        const JRot R = s_r[J];
        if (R.rot) {
          const int p = R.pq & 0xffff, q = R.pq >> 16;
          const double2 g = pz(R.sr, R.si);
          const double2 vp = VT[p * ldv + i], vq = VT[q * ldv + i];
          VT[p * ldv + i] = psub(pscal(R.c, vp), pmul(pconj(g), vq));
          VT[q * ldv + i] = padd(pmul(g, vp), pscal(R.c, vq));
        }
        J += vdJ;
        i += vdi;
        if (i >= nb) {
          i -= nb;
          ++J;
        }
      }
      __syncthreads();
    }
    if (!any) {
      converged = 1;
      break;
    }
  }

  // eigenvalues in ascending order (ties by index)
  if (t < m) s_lam[t] = A[up_idx(t, t, mq)].x;
  if (t < kMaxM) s_inv[t] = t < m ? t : 0;
  __syncthreads();
  if (t < m) {
    const double lt = s_lam[t];
    int r = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = s_lam[j];
      r += (lj < lt) || (lj == lt && j < t);
    }
    s_inv[r] = t;  // r <= m - 1
  }
  __syncthreads();
  const int64_t kb = (int64_t)k * a.mp;
  int nonfinite = !isfinite(tol);
  for (int r = t; r < a.mp; r += kEigThreads) {
    double lam = 0.0, w = 0.0;
    if (r < m) {
      const int l = s_inv[r];
      lam = s_lam[l];
      for (int i = 0; i < nb; ++i) w += pabs2(VT[l * ldv + i]);
      nonfinite |= !isfinite(lam);
    }
    a.evals[kb + r] = lam;
    a.wphys[kb + r] = w;
  }
  double2* U = reinterpret_cast<double2*>(a.evecs) + (int64_t)k * a.nb_max * a.mp;
  for (int idx = t; idx < a.nb_max * a.mp; idx += kEigThreads) {
    const int i = idx / a.mp, r = idx - i * a.mp;
    U[idx] = (i < nb && r < m) ? VT[s_inv[r] * ldv + i] : pz(0.0, 0.0);
  }
  if (a.worb)
    for (int idx = t; idx < a.mp * nc; idx += kEigThreads) {
      const int r = idx / nc, al = idx - r * nc;
      double w = 0.0;
      if (r < m) {
        const int l = s_inv[r];
        double2 acc = pz(0.0, 0.0);
        for (int v = 0; v < nb; ++v) acc = pfma(S[al * nb + v], VT[l * ldv + v], acc);
        w = pabs2(acc);
      }
      a.worb[(kb + r) * nc + al] = w;
    }
  if (t == 0) {
    a.sweeps[k] = sweep;
    if (!converged) atomicOr(a.err, ERR_NOCONV);
  }
  if (nonfinite) atomicOr(a.err, ERR_NONFINITE);
}

__global__ void __launch_bounds__(256) pole_density_kernel(PoleArgs a, double mu, int nw_trunc, double* nk_out,
                                                           double* kscal) {
  extern __shared__ double2 lds[];
  __shared__ double s_f[kMaxM];
  __shared__ double red[256];
  const int k = blockIdx.x, t = threadIdx.x;
  int nb;
  int64_t ob;
  k_window(a, k, nb, ob);
  const int nc = a.nc, m = nb + a.np, ldu = m + 1;
  double2* Us = lds;  // nb x ldu
  const double2* U = reinterpret_cast<const double2*>(a.evecs) + (int64_t)k * a.nb_max * a.mp;
  for (int idx = t; idx < nb * m; idx += 256) {
    const int i = idx / m, l = idx - i * m;
    Us[i * ldu + l] = U[i * a.mp + l];
  }
  if (t < m) {
    const double x = a.evals[(int64_t)k * a.mp + t] - mu;
    s_f[t] = nw_trunc > 0 ? truncated_weight(x, a.beta, nw_trunc) : fermi(x, a.beta);
  }
  __syncthreads();
  const double* E = a.eps + ob;
  const int64_t on = a.nb_uniform > 0 ? (int64_t)k * nb * nb : a.off_n[k];
  double2* N = nk_out ? reinterpret_cast<double2*>(nk_out) + on : nullptr;
  double tr = 0.0, hks = 0.0, ncor = 0.0;
  for (int idx = t; idx < nb * nb; idx += 256) {
    const int i = idx / nb, j = idx - i * nb;
    double2 acc = pz(0.0, 0.0);
    for (int l = 0; l < m; ++l) acc = pfma(pscal(s_f[l], Us[i * ldu + l]), pconj(Us[j * ldu + l]), acc);
    if (N) N[idx] = acc;
    if (i == j) {
      tr += acc.x;
      hks += E[i] * acc.x;
    }
  }
  const double2* S = reinterpret_cast<const double2*>(a.proj) + ob * nc;
  for (int idx = t; idx < nc * m; idx += 256) {
    const int al = idx / m, l = idx - al * m;
    double2 acc = pz(0.0, 0.0);
    for (int v = 0; v < nb; ++v) acc = pfma(S[al * nb + v], Us[v * ldu + l], acc);
    ncor += s_f[l] * pabs2(acc);
  }
  tr = pole_block_sum<256>(tr, red);
  ncor = pole_block_sum<256>(ncor, red);
  hks = pole_block_sum<256>(hks, red);
  if (t == 0) {
    kscal[3 * k + 0] = tr;
    kscal[3 * k + 1] = ncor;
    kscal[3 * k + 2] = hks;
  }
}

__global__ void __launch_bounds__(1024) pole_mu_kernel(PoleArgs a, double n_target, double tol, int method,
                                                       double lo, double hi, double mu0, int max_iter, double* res) {
  __shared__ double red[1024];
  const int64_t total = (int64_t)a.nk * a.mp;
  auto eval = [&](double mu, double& nv, double& dv) {
    double sn = 0.0, sd = 0.0;
    for (int64_t idx = threadIdx.x; idx < total; idx += 1024) {
      const int kk = (int)(idx / a.mp);
      const double w = a.wk[kk] * a.wphys[idx];
      const double f = fermi(a.evals[idx] - mu, a.beta);
      sn += w * f;
      sd += w * a.beta * f * (1.0 - f);
    }
    nv = pole_block_sum<1024>(sn, red);
    dv = pole_block_sum<1024>(sd, red);
  };
  int passes = 0, converged = 0;
  double mu = 0.0, nv = 0.0, dv = 0.0;
  if (method == 1) {
    for (int it = 0; it < max_iter; ++it) {
      mu = 0.5 * (lo + hi);
      eval(mu, nv, dv);
      ++passes;
      if (fabs(nv - n_target) <= tol) {
        converged = 1;
        break;
      }
      if (nv < n_target) lo = mu;
      else hi = mu;
    }
  } else {
    // Newton kept inside the bracket; bisect when the step leaves it or the
    // residual does not fall fast enough
    mu = fmin(fmax(mu0, lo), hi);
    double prev_res = INFINITY, prev_dx = hi - lo;
    for (int it = 0; it < max_iter; ++it) {
      eval(mu, nv, dv);
      ++passes;
      const double r = nv - n_target;
      if (fabs(r) <= tol) {
        converged = 1;
        break;
      }
      if (r < 0) lo = mu;
      else hi = mu;
      double next = 0.0;
      bool ok = dv > 0.0 && isfinite(dv);
      if (ok) {
        next = mu - r / dv;
        if (!(next > lo && next < hi)) ok = false;
        if (fabs(r) > 0.5 * prev_res && fabs(next - mu) > 0.5 * prev_dx) ok = false;
      }
      if (!ok) next = 0.5 * (lo + hi);
      prev_dx = fabs(next - mu);
      prev_res = fabs(r);
      mu = next;
    }
  }
  if (threadIdx.x == 0) {
    res[0] = mu;
    res[1] = nv;
    res[2] = (double)passes;
    res[3] = converged ? 0.0 : 1.0;
  }
}

__global__ void __launch_bounds__(kDosThreads) pole_dos_kernel(PoleArgs a, double mu, double eta, double e_min,
                                                               double de, int ne, int nslices, double* part) {
  __shared__ double s_lam[kDosThreads], s_w[kDosThreads], s_wo[kDosThreads * 16];
  const int t = threadIdx.x, e = blockIdx.x * kDosThreads + t, slice = blockIdx.y;
  const int nc = a.nc;
  const int64_t total = (int64_t)a.nk * a.mp;
  const int64_t per = (total + nslices - 1) / nslices;
  const int64_t s0 = (int64_t)slice * per, s1 = s0 + per < total ? s0 + per : total;
  const double ee = e_min + (double)e * de + mu;
  const double scale = eta / M_PI, eta2 = eta * eta;
  double d = 0.0, pd[16];
#pragma unroll
  for (int al = 0; al < 16; ++al) pd[al] = 0.0;
  for (int64_t c0 = s0; c0 < s1; c0 += kDosThreads) {
    __syncthreads();
    const int64_t idx = c0 + t;
    if (idx < s1) {
      const double w = a.wk[idx / a.mp];
      s_lam[t] = a.evals[idx];
      s_w[t] = w * a.wphys[idx];
      for (int al = 0; al < nc; ++al) s_wo[t * 16 + al] = a.worb ? w * a.worb[idx * nc + al] : 0.0;
    }
    __syncthreads();
    const int cnt = (int)(s1 - c0 < kDosThreads ? s1 - c0 : kDosThreads);
    for (int j = 0; j < cnt; ++j) {
      const double x = ee - s_lam[j];
      const double L = scale / (x * x + eta2);
      d += s_w[j] * L;
#pragma unroll
      for (int al = 0; al < 16; ++al)
        if (al < nc) pd[al] += s_wo[j * 16 + al] * L;
    }
  }
  if (e < ne) {
    double* o = part + ((int64_t)slice * ne + e) * (1 + nc);
    o[0] = d;
#pragma unroll
    for (int al = 0; al < 16; ++al)
      if (al < nc) o[1 + al] = pd[al];
  }
}

__global__ void pole_dos_reduce_kernel(int ne, int nc, int nslices, const double* part, double* dos, double* pdos) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)ne * (1 + nc);
  if (idx >= n) return;
  double s = 0.0;
  for (int sl = 0; sl < nslices; ++sl) s += part[(int64_t)sl * n + idx];
  const int e = (int)(idx / (1 + nc)), c = (int)(idx - (int64_t)e * (1 + nc));
  if (c == 0) dos[e] = s;
  else if (pdos) pdos[(int64_t)e * nc + c - 1] = s;
}

// Energy-functional sums over (k, level m) (Sec. 3.5.1): per block partials of
// B = sum w_k E^ps |u|^2 n_F, N = sum w_k |u|^2 n_F, <H_KS> = sum w_k n_F sum_n E_n |u_nm|^2
// and n_a = sum w_k |S_a u|^2 n_F.
__global__ void __launch_bounds__(256) pole_energy_kernel(PoleArgs a, double mu, double* part) {
  __shared__ double red[256];
  const int t = threadIdx.x, nc = a.nc;
  const int64_t total = (int64_t)a.nk * a.mp;
  double sb = 0.0, sn = 0.0, sh = 0.0, so[16];
#pragma unroll
  for (int al = 0; al < 16; ++al) so[al] = 0.0;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + t; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int k = (int)(idx / a.mp), m = (int)(idx - (int64_t)k * a.mp);
    int nb;
    int64_t ob;
    k_window(a, k, nb, ob);
    if (m >= nb + a.np) continue;
    const double lam = a.evals[idx];
    const double wf = a.wk[k] * fermi(lam - mu, a.beta);
    const double wp = a.wphys[idx];
    sb += wf * lam * wp;
    sn += wf * wp;
    const double2* U = reinterpret_cast<const double2*>(a.evecs) + (int64_t)k * a.nb_max * a.mp + m;
    const double* E = a.eps + ob;
    double hk = 0.0;
    for (int n = 0; n < nb; ++n) hk += E[n] * pabs2(U[(int64_t)n * a.mp]);
    sh += wf * hk;
#pragma unroll
    for (int al = 0; al < 16; ++al)
      if (al < nc) so[al] += wf * a.worb[idx * nc + al];
  }
  double* o = part + (int64_t)blockIdx.x * (3 + nc);
  sb = pole_block_sum<256>(sb, red);
  sn = pole_block_sum<256>(sn, red);
  sh = pole_block_sum<256>(sh, red);
  if (t == 0) {
    o[0] = sb;
    o[1] = sn;
    o[2] = sh;
  }
#pragma unroll
  for (int al = 0; al < 16; ++al)
    if (al < nc) {
      const double v = pole_block_sum<256>(so[al], red);
      if (t == 0) o[3 + al] = v;
    }
}

// Fixed-order sum of partial j over the energy kernel's blocks (one work-group
// per value), written to its slot of out = [B, N_tot, <H_KS>, <V_DC>, <H_U>, n_a ...].
__global__ void __launch_bounds__(256) pole_energy_reduce_kernel(int nparts, int nc, const double* part,
                                                                 double* out) {
  __shared__ double red[256];
  const int t = threadIdx.x, j = blockIdx.x, nv = 3 + nc;
  double s = 0.0;
  for (int b = t; b < nparts; b += 256) s += part[(int64_t)b * nv + j];
  s = pole_block_sum<256>(s, red);
  if (t == 0) out[j < 3 ? j : j + 2] = s;
}

// <V_DC> = sum_a V_DC,a n_a and <H_U> = (B - <H_KS> + <V_DC>) / 2.
__global__ void pole_energy_finish_kernel(int nc, const double* e_dc, double* out) {
  if (threadIdx.x != 0) return;
  double vdc = 0.0;
  for (int al = 0; al < nc; ++al) vdc += e_dc[al] * out[5 + al];
  out[3] = vdc;
  out[4] = 0.5 * (out[0] - out[2] + vdc);
}

hipError_t allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

size_t pole_eig_lds_bytes(int nb, int np) {
  const int m = nb + np, mq = m + (m & 1);
  return (size_t)(mq * (mq + 1) / 2 + mq * (nb + 1)) * 16;
}

template <int NT>
hipError_t launch_pole_eig_nt(const PoleArgs& a, size_t lds_bytes, hipStream_t s) {
  hipError_t e = allow_lds(reinterpret_cast<const void*>(pole_eig_kernel<NT>), lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pole_eig_kernel<NT>, dim3(a.nk), dim3(NT), lds_bytes, s, a);
  return hipGetLastError();
}

hipError_t launch_pole_eig(const PoleArgs& a, size_t lds_bytes, hipStream_t s) {
  // update items of one step at the largest size: 2x2 blocks I <= J and eigenvector pairs
  const int m = a.nb_max + a.np, mq = m + (m & 1), P = mq / 2;
  const int items = P * (P + 1) / 2 + P * a.nb_max;
  if (items <= 512) return launch_pole_eig_nt<256>(a, lds_bytes, s);
  if (items <= 1536) return launch_pole_eig_nt<512>(a, lds_bytes, s);
  return launch_pole_eig_nt<1024>(a, lds_bytes, s);
}

hipError_t launch_pole_density(const PoleArgs& a, double mu, int nw_trunc, double* nk_out, double* kscal,
                               hipStream_t s) {
  const size_t lds = (size_t)a.nb_max * (a.nb_max + a.np + 1) * 16;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(pole_density_kernel), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pole_density_kernel, dim3(a.nk), dim3(256), lds, s, a, mu, nw_trunc, nk_out, kscal);
  return hipGetLastError();
}

hipError_t launch_pole_find_mu(const PoleArgs& a, double n_target, double tol, int method, double lo, double hi,
                               double mu0, int max_iter, double* res, hipStream_t s) {
  hipLaunchKernelGGL(pole_mu_kernel, dim3(1), dim3(1024), 0, s, a, n_target, tol, method, lo, hi, mu0, max_iter,
                     res);
  return hipGetLastError();
}

int pole_dos_kslices(int nk, int mp) {
  const int64_t total = (int64_t)nk * mp;
  int64_t n = (total + kDosChunk - 1) / kDosChunk;
  return (int)(n < 1 ? 1 : n > kMaxSlices ? kMaxSlices : n);
}

hipError_t launch_pole_dos(const PoleArgs& a, double mu, double eta, double e_min, double e_max, int ne,
                           double* part, double* dos, double* pdos, hipStream_t s) {
  const int ns = pole_dos_kslices(a.nk, a.mp);
  const double de = ne > 1 ? (e_max - e_min) / (double)(ne - 1) : 0.0;
  hipLaunchKernelGGL(pole_dos_kernel, dim3((ne + kDosThreads - 1) / kDosThreads, ns), dim3(kDosThreads), 0, s, a,
                     mu, eta, e_min, de, ne, ns, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)ne * (1 + a.nc);
  hipLaunchKernelGGL(pole_dos_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ne, a.nc, ns, part,
                     dos, pdos);
  return hipGetLastError();
}

int pole_energy_parts(int nk, int mp) {
  const int64_t n = ((int64_t)nk * mp + 255) / 256;
  return (int)(n < 1 ? 1 : n > 1024 ? 1024 : n);
}

hipError_t launch_pole_energy(const PoleArgs& a, double mu, double* part, double* out, hipStream_t s) {
  const int np = pole_energy_parts(a.nk, a.mp);
  hipLaunchKernelGGL(pole_energy_kernel, dim3(np), dim3(256), 0, s, a, mu, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pole_energy_reduce_kernel, dim3(3 + a.nc), dim3(256), 0, s, np, a.nc, part, out);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pole_energy_finish_kernel, dim3(1), dim3(64), 0, s, a.nc, a.e_dc, out);
  return hipGetLastError();
}

}  // namespace dmft
