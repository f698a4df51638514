// Low-rank form of the lattice Dyson step (gfx950 / CDNA4).
//
// The self-energy enters the band window only through the nc correlated
// orbitals (the embedding of the DMFT-loop section), so with D = diag(d),
// d_v = 1 / (i w_n + mu - E_v), the band-window matrix is a rank-nc
// correction of a diagonal one:  A = D^-1 - S^dag Sigma' S,  Sigma' = Sigma - V_DC.
// With the nc x nc matrices
//
//     X   = S D S^dag                      (projected bare propagator)
//     K   = X^-1 - Sigma'
//     Gl  = K^-1                            (= S G S^dag)
//     R   = Sigma' + Sigma' Gl Sigma'       (= (I - Sigma' X)^-1 Sigma', since Gl X^-1 = I + Gl Sigma')
//
// the Woodbury identity gives, exactly,
//
//     G           = D + D S^dag R S D
//     tr G        = sum_v d_v + tr(R X2)                            X_j = S D^j S^dag
//     tr G^2      = sum_v d_v^2 + 2 tr(R X3) + tr(R X2 R X2)
//
// so the nb^3 inversion becomes rank-nc products on the matrix cores and two
// nc x nc inversions.  Both are Gauss-Jordan sweeps without pivoting, which is
// safe for the same reason as for A: Im d_v = -w_n / (w_n^2 + (mu - E_v)^2) < 0,
// so for any S of full row rank the anti-Hermitian part of X, S Im(D) S^dag, is
// negative definite; that of X^-1 is then positive definite, that of
// K = X^-1 - Sigma' too for a causal Sigma, and every leading block of either
// matrix is invertible.  (Orthonormal rows, as the projector construction of
// the projection section gives them, are not needed.)
//
// One wavefront walks a (k-tile, frequency-tile) item, four frequencies at a
// time:
//   1. X_f = S D_f S^dag for f = 0..3 on the matrix cores (16x16x4 FP64,
//      contraction over band chunks), staged through LDS;
//   2. lane 16 g + i takes row i of X_g; both inversions run in this row
//      layout for the four matrices at once (see rsweep), and Gl_g goes back
//      through LDS;
//   3. per frequency, in the output layout of the matrix core: R, then either
//      sum_n G += D + (D S^dag)(R S D) and the w_k Gl partial of G_loc
//      (density kind), or the traces (trace kind), or the traces and
//      w_k S G^2 S^dag (adjoint kind: the fused scalar adjoint of N_tot,
//      dN/dSigma_n = (2/beta) [sum_k w_k S G^2 S^dag]^dag), with
//      S G = (I + X R) S D, G S^dag = D S^dag (I + R X) and I + X R = Gl X^-1 = I + Gl Sigma':
//          S G^2 S^dag = (I + Gl Sigma') X2 (I + Sigma' Gl);
//      or (general kind) the vector-Jacobian product for cotangents Nbar_k of
//      N(k) and Gbar_n of G_loc.  With Nt = Nbar + Nbar^dag, Rl = I + Gl Sigma'
//      (= Gl X^-1) and Rr = I + Sigma' Gl (= X^-1 Gl), S G = Rl S D and
//      G S^dag = D S^dag Rr, so the dense kernel's S G^dag C G^dag S^dag becomes
//          Sigmabar_n^dag share = (1/beta) Rl P1 Rr + w_k Gl Gbar_n^dag Gl,   P1 = S D Nt D S^dag,
//      and from G^2 = D^2 + D^2 S^dag R S D + D S^dag R S D^2 + D S^dag R X2 R S D
//          tr(Nt G^2) = sum_v Nt_vv d_v^2 + tr(R P2) + tr(R X2 R P1),
//          P2 = S (D Nt D^2 + D^2 Nt D) S^dag;
//      P1 and P2 come from the two band-window products Nt D S^dag and
//      Nt D^2 S^dag (O(nb^2 nc)), and mubar also takes -w_k Re<Gbar_n, Rl X2 Rr>.
//
// Operand bookkeeping of the 16x16x4 instruction: a matrix M used as the A
// operand comes from registers holding M^T in the output layout (lane
// 16 q + c16, register i: row q + 4 i, column c16), as the B operand from
// registers holding M.  The products are ordered so that their operands are
// already in that form:
//   X   from  A = S[c16][r] d_r,  B = S[c16][r] (conjugated)
//   V   = Gl^T Sigma'^T      (A: Gl,           B: Sigma'[c16][q + 4 j])
//   R^T = Sigma'^T + Sigma'^T V  (A: Sigma'[q + 4 j][c16], B: V)  -> R^T holds R[c16][q + 4 i]
//   Q   = (R S) D            (A: R^T,          B: S[q + 4 j][16 b + c16])
//   sum_n G += (D S^dag) Q   (A: d_r conj(S[q + 4 j][r]), B: Q)
// and tr(E^2), E = R X2, takes one 16x16 transpose through LDS.
#pragma once

#include <type_traits>

#include "dyson_impl.h"

namespace dmft {

// 1 / (zr + i zi - e) for real e.
__device__ __forceinline__ double2 inv_z_minus(double zr, double zi, double e) {
  double x = zr - e;
  double d = x * x + zi * zi;
  double r = __builtin_amdgcn_rcp(d);
  double t = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, t, r);
  t = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, t, r);
  return make_double2(x * r, -zi * r);
}

// Complex products on the 16x16x4 matrix core (real and imaginary parts in
// separate accumulators):  cmma: D += A B,  cmma_cb: D += A conj(B).
__device__ __forceinline__ void cmma(v4d& dr, v4d& di, double ar, double ai, double br, double bi) {
  dr = mma(ar, br, dr);
  dr = mms(ai, bi, dr);
  di = mma(ar, bi, di);
  di = mma(ai, br, di);
}
__device__ __forceinline__ void cmma_cb(v4d& dr, v4d& di, double ar, double ai, double br, double bi) {
  dr = mma(ar, br, dr);
  dr = mma(ai, bi, dr);
  di = mma(ai, br, di);
  di = mms(ar, bi, di);
}

// Complex 16x16 accumulator on the matrix core.  M3 = false: real and
// imaginary parts, four real products per complex product.  M3 = true: the
// three-product form P1 = sum ar br, P2 = sum ai bi, P3 = sum (ar + ai)(br + bi),
// re = P1 - P2, im = P3 - P1 - P2 (a quarter fewer matrix-core products and
// shorter dependent chains; the imaginary part is exact to rounding relative
// to |A| |B|, which is what normwise error bounds need).
template <bool M3>
struct CAcc;

template <>
struct CAcc<false> {
  v4d r, i;
  __device__ __forceinline__ void zero() { r = i = (v4d){0.0, 0.0, 0.0, 0.0}; }
  __device__ __forceinline__ void set(const v4d& re, const v4d& im) {
    r = re;
    i = im;
  }
  __device__ __forceinline__ void mac(double ar, double ai, double br, double bi) { cmma(r, i, ar, ai, br, bi); }
  __device__ __forceinline__ void mac_cb(double ar, double ai, double br, double bi) { cmma_cb(r, i, ar, ai, br, bi); }
  __device__ __forceinline__ v4d re() const { return r; }
  __device__ __forceinline__ v4d im() const { return i; }
  __device__ __forceinline__ void add(int reg, double x, double y) {
    r[reg] += x;
    i[reg] += y;
  }
};

template <>
struct CAcc<true> {
  v4d p1, p2, p3;
  __device__ __forceinline__ void zero() { p1 = p2 = p3 = (v4d){0.0, 0.0, 0.0, 0.0}; }
  __device__ __forceinline__ void set(const v4d& re, const v4d& im) {
    p1 = re;
    p2 = (v4d){0.0, 0.0, 0.0, 0.0};
    p3 = re + im;
  }
  __device__ __forceinline__ void mac(double ar, double ai, double br, double bi) {
    p1 = mma(ar, br, p1);
    p2 = mma(ai, bi, p2);
    p3 = mma(ar + ai, br + bi, p3);
  }
  __device__ __forceinline__ void mac_cb(double ar, double ai, double br, double bi) {
    p1 = mma(ar, br, p1);
    p2 = mms(ai, bi, p2);
    p3 = mma(ar + ai, br - bi, p3);
  }
  __device__ __forceinline__ v4d re() const { return p1 - p2; }
  __device__ __forceinline__ v4d im() const { return p3 - p1 - p2; }
  __device__ __forceinline__ void add(int reg, double x, double y) {
    p1[reg] += x;
    p3[reg] += x + y;
  }
};

// 16x16 output-layout tile transposed through LDS: out register i holds in[c16][q + 4 i].
__device__ __forceinline__ void tile_transpose(const v4d& inr, const v4d& ini, v4d& outr, v4d& outi, double2* buf,
                                               int q, int c16) {
#pragma unroll
  for (int i = 0; i < 4; ++i) buf[(q + 4 * i) * 17 + c16] = make_double2(inr[i], ini[i]);
  wave_sync();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double2 v = buf[c16 * 17 + q + 4 * i];
    outr[i] = v.x;
    outi[i] = v.y;
  }
  wave_sync();
}

// Re sum over this lane's registers of a[i] b[i] (complex).
__device__ __forceinline__ double re_dot4(const v4d& ar, const v4d& ai, const v4d& br, const v4d& bi) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) s += ar[i] * br[i] - ai[i] * bi[i];
  return s;
}

// Projector fragment S[al][bd] (zero outside nc x nb).
__device__ __forceinline__ double2 lr_proj(const double2* P, int al, int bd, int nc, int nb) {
  return (al < nc && bd < nb) ? P[al * nb + bd] : make_double2(0.0, 0.0);
}

// The same fragment, loaded where the call is: the row index is hidden from
// the optimizer, so neither the load nor its address is moved out of the
// enclosing loop (a hoisted address is a 64-bit register pair per load, kept
// or spilled across the loop), and the load is not merged with an earlier one.
__device__ __forceinline__ double2 lr_proj_here(const double2* P, int al, int bd, int nc, int nb) {
  asm volatile("" : "+v"(al));
  return lr_proj(P, al, bd, nc, nb);
}

// The two projector fragment sets of a lane: pa = S[q + 4 j][16 b + c16]
// (B operand of R S, A operand of D S^dag) and pt = S[c16][16 t + 4 i + q]
// (both operands of S D S^dag).
template <int NBP>
__device__ __forceinline__ void lr_load_pa(Proj<NBP>& pr, const double2* P, int nc, int nb, int q, int c16) {
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int b = 0; b < NBP / 16; ++b) {
      double2 v = lr_proj_here(P, q + 4 * j, 16 * b + c16, nc, nb);
      pr.pa_r[j][b] = v.x;
      pr.pa_i[j][b] = v.y;
    }
}
template <int NBP>
__device__ __forceinline__ void lr_load_pt(Proj<NBP>& pr, const double2* P, int nc, int nb, int q, int c16) {
#pragma unroll
  for (int t = 0; t < NBP / 16; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double2 v = lr_proj_here(P, c16, 16 * t + 4 * i + q, nc, nb);
      pr.pt_r[t][i] = v.x;
      pr.pt_i[t][i] = v.y;
    }
}

// Column tiles of sum_n G one work item keeps: all of them, except for 64-band
// windows, whose 64x64 running sum would not fit next to the rest in
// registers; those are split into two items of 32 columns each (the nc x nc
// part of the step is then computed once per item).
template <int NBP, int KIND>
constexpr int lr_col_tiles() {
  return (KIND == KIND_DENSITY && NBP == 64) ? 2 : NBP / 16;
}

// Inversion stage.  One matrix per wavefront with four elements per lane
// would leave each Gauss-Jordan step a serial chain of LDS round trip,
// reciprocal and a few FMAs.  Instead lane 16 g + i holds row i of matrix g
// in registers, the pivot row of step K is broadcast inside each 16-lane row
// by DPP (row_newbcast:K), and each step is one pass of independent FMAs over
// the row.  The update is the in-place Gauss-Jordan step with the pivot row
// scaled through the multiplier 1 - 1/p and the pivot column and pivot set
// directly, which avoids the cancellation of a fully uniform update (whose
// pivot entry p - (p - 1)(p + 1)/p loses about |p|^2 ulps).

struct LRShared {
  double2 buf[4][16 * 17];  // one 16x16 tile per frequency of the group (rows padded to 17)
  double2 dtab[4][64];      // d_r = 1 / (i w + mu - E_r) of the group's frequencies (zero past nb)
};

// Value of lane K of this lane's 16-lane row.  Every lane of a row reads a lane
// of its own row, so no lane is out of bounds; bound_ctrl lets the compiler
// skip initialising the destination (the "old" value is never used).
template <int K>
__device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + K, 0xf, 0xf, true);
}

// Gauss-Jordan steps K .. nc-1 on the row held by this lane (row i of its
// matrix); NC columns are kept (nc <= NC; the others are zero throughout).
template <int K, int NC>
__device__ __forceinline__ void rsweep(double (&rr)[NC], double (&ri)[NC], int i, int nc, int& bad) {
  if constexpr (K < NC) {
    if (K >= nc) return;
    const double2 p = make_double2(row_bcast<K>(rr[K]), row_bcast<K>(ri[K]));
    bad |= (p.x == 0.0 && p.y == 0.0);
    const double2 ip = crecip(p);
    const double2 l = cmul(make_double2(rr[K], ri[K]), ip);
    const bool piv = i == K;
    const double lr = piv ? 1.0 - ip.x : l.x;
    const double li = piv ? -ip.y : l.y;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (j == K) continue;
      const double br = row_bcast<K>(rr[j]), bi = row_bcast<K>(ri[j]);
      rr[j] = __builtin_fma(-lr, br, __builtin_fma(li, bi, rr[j]));
      ri[j] = __builtin_fma(-lr, bi, __builtin_fma(-li, br, ri[j]));
    }
    rr[K] = piv ? ip.x : -l.x;
    ri[K] = piv ? ip.y : -l.y;
    rsweep<K + 1, NC>(rr, ri, i, nc, bad);
  }
}

// S[c16 & 7][r] from the lane's S[c16][r] when nc <= 8: rows 8 .. 15 of S are
// zero, so adding the value eight lanes away along the 16-lane row (row_ror:8)
// moves S[c16 - 8][r] into lanes 8 .. 15 and leaves lanes 0 .. 7 unchanged.
__device__ __forceinline__ double2 lower_rows8(double2 s) {
  return make_double2(s.x + __builtin_amdgcn_update_dpp(0.0, s.x, 0x128, 0xf, 0xf, true),
                      s.y + __builtin_amdgcn_update_dpp(0.0, s.y, 0x128, 0xf, 0xf, true));
}

// Partial-fraction form of the running sum (density kind, nc > 8).  The sum
// needs F[v][v'] = sum_n d_v d_v' M_n[v][v'], M_n = S^dag R_n S,
// d_v = 1 / (z_n - E_v).  Since d_v d_v' = (d_v - d_v') / (E_v - E_v') exactly,
//     F[v][v'] = ((W S)[v][v'] - (S^dag Y)[v][v']) / (E_v - E_v')  (E_v != E_v'),
//     W = sum_n D_n S^dag R_n  (nb x nc),   Y = sum_n R_n S D_n  (nc x nb),
// so a frequency adds two rank-nc products instead of the nb x nb update
// (D S^dag)(R S D), and the nb x nb products are formed once per k-point.  The
// subtraction loses about |d| / |E_v - E_v'| digits, so the diagonal and pairs
// closer than delta = pi / (16 beta) (a sixteenth of the first Matsubara
// frequency) are summed directly per column: sum_n d_v'^2 (R_n S)[.][v'] and,
// for at most one close partner v, sum_n d_v d_v' (R_n S)[.][v'], contracted
// with S^dag at the end of the k-point.  A k-point on which a column has more
// than one close partner takes the direct running sum.  (Normwise relative
// errors on the test and benchmark inputs are below 1e-12.)
//
// Close partners of the columns v' = 16 c + c16 of this lane; returns whether
// the form applies (the same answer in every lane of the wavefront).
template <int T>
__device__ __forceinline__ bool lr_pf_pairs(const double* eps, int nb, int c16, double beta, int (&partner)[T]) {
  const double delta = M_PI / (16.0 * beta);
  int over = 0;
#pragma unroll
  for (int c = 0; c < T; ++c) {
    const int vc = 16 * c + c16;
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
  return !__any(over);
}

// X_f = S D_f S^dag of the four frequencies of a group when nc <= 8: two
// frequencies per matrix-core product, stacked in the A rows (row 8 h + alpha
// holds S[alpha][r] d_{2c + h}[r]); the B columns are S[beta][r]^* as before.
// Output register i holds row 4 i + q, i.e. frequency 2c + (i >> 1), row
// 4 (i & 1) + q: half the products of one frequency per product.
template <int NBP, int RL, bool M3>
__device__ __forceinline__ void lr_x_packed(const Proj<NBP>& pr, const double2* P, int nc, int nb, LRShared& sh,
                                            int q, int c16) {
  constexpr int T = NBP / 16;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int fa = 2 * c + (c16 >> 3);  // frequency of this lane's A row
    CAcc<M3> x;
    x.zero();
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (16 * t + 4 * i >= nb) break;
        const double2 s = RL == 2 ? lr_proj_here(P, c16, 16 * t + 4 * i + q, nc, nb)
                                  : make_double2(pr.pt_r[t][i], pr.pt_i[t][i]);
        const double2 sa = lower_rows8(s);
        const double2 dd = sh.dtab[fa][16 * t + 4 * i + q];
        const double2 a1 = cmul(sa, dd);
        x.mac_cb(a1.x, a1.y, s.x, s.y);
      }
    const v4d xr = x.re(), xi = x.im();
#pragma unroll
    for (int i = 0; i < 4; ++i)
      sh.buf[2 * c + (i >> 1)][(4 * (i & 1) + q) * 17 + c16] = make_double2(xr[i], xi[i]);
  }
}

// PF: the running sum in the partial-fraction form on every k-point where it
// applies (density kind with every column tile in the item); pfc then points
// to the work-group's LDS slots for the close-pair sums (NBP / 16 x 4 x 64).
template <int NBP, int KIND, int RL, bool M3, int NC, int PART, bool PF = false>
__device__ __forceinline__ void lr_tile_part(const DysonArgs& a, int ktile, int wtile, LRShared& sh, int lane,
                                             double2* pfc = nullptr) {
  static_assert(!PF || (KIND == KIND_DENSITY && (NBP / 16) == lr_col_tiles<NBP, KIND>()),
                "the partial-fraction form needs the density kind and every column tile");
  constexpr int T = NBP / 16;
  constexpr int CT = lr_col_tiles<NBP, KIND>();
  constexpr int b0 = PART * CT;
  const int q = lane >> 4, c16 = lane & 15;
  const int g = q, ri_ = c16;  // row-layout coordinates: matrix g, row ri_
  const int n0 = wtile * a.wt;
  const int n1 = min(n0 + a.wt, a.nw);
  const int kk0 = ktile * a.kt;
  const int kk1 = min(kk0 + a.kt, a.nklist);
  const double mu = uniform_d(a.mu_ptr ? *a.mu_ptr : a.mu);
  const int nc = a.nc;
  const int kc = (nc + 3) >> 2;
  // nc >= 1 (and nb >= nc below): the first chunk of every contraction over
  // orbitals or bands is always taken, so its accumulator can start from an
  // inline zero instead of registers cleared beforehand
  __builtin_assume(kc >= 1 && kc <= 4);
  // every dispatcher keeps nc <= NC columns and takes more than 8 only for
  // nc > 8, so the first eight pivot steps and columns need no test
  __builtin_assume(nc >= 1 && nc <= NC);
  if constexpr (NC > 8) __builtin_assume(nc > 8);
  const double beta = a.beta;
  const bool want_s = (KIND == KIND_DENSITY) && (a.mode & MODE_S);
  const bool want_x = (KIND == KIND_DENSITY) && (a.mode & MODE_GLOC) && PART == 0;
  const bool hasdiag = c16 >= q && ((c16 - q) & 3) == 0;
  const int idg = (c16 - q) >> 2;
  // V_DC of orbital c16 (the row-layout row and the output-layout column are
  // both c16): read once, not inside the frequency loop, where each guarded
  // load would be waited for on its own
  const double edc = c16 < nc ? a.e_dc[c16] : 0.0;
  int bad = 0, nonfinite = 0;

  for (int kk = kk0; kk < kk1; ++kk) {
    const int k = uniform_i(a.klist ? a.klist[kk] : kk);
    const int nb = uniform_i(a.nb_uniform > 0 ? a.nb_uniform : a.nb[k]);
    __builtin_assume(nb >= 1 && nb <= NBP);
    // k-points are bucketed by padded size: NBP - 16 < nb, so every chunk but
    // those of the last 16 bands is full.  This is a promise to the compiler,
    // not a hint: were it false, the chunk and fragment tests it removes could
    // let loads run past the k-point's bands, so the host checks it for every
    // bucket before any launch.  The adjoint kinds, whose unrolled bodies
    // would then outgrow the registers, are not told.
    if constexpr (KIND == KIND_DENSITY || KIND == KIND_TRACE) __builtin_assume(nb > NBP - 16);
    const int64_t ob = uniform_l(a.nb_uniform > 0 ? (int64_t)k * nb : a.off_b[k]);
    const double* eps = a.eps + ob;
    // band energies this lane enters into the resolvent table of every
    // frequency group (band (lane + 64 it) mod NBP), read once per k; for
    // 64-band windows (four per lane) they are re-read, which keeps the
    // adjoint kinds spill-free
    constexpr int NDT = (4 * NBP + 63) / 64;
    constexpr bool EPL = NBP <= 48;
    double epl[NDT];
#pragma unroll
    for (int it = 0; it < NDT; ++it) {
      const int r = (lane + 64 * it) % NBP;
      epl[it] = (EPL && r < nb) ? eps[r] : 0.0;
    }
    const double2* P = reinterpret_cast<const double2*>(a.proj) + ob * nc;
    const double wk = uniform_d(a.wk[k]);
    // general product: Nbar_k (row-major) and the real diagonal of Nt = Nbar + Nbar^dag at
    // band 16 t + c16
    const double2* ntb = nullptr;
    double ntd[KIND == KIND_GEN ? T : 1];
    if constexpr (KIND == KIND_GEN) {
      if (a.nbar) ntb = reinterpret_cast<const double2*>(a.nbar) + (a.off_n ? a.off_n[k] : (int64_t)k * nb * nb);
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int v = 16 * t + c16;
        ntd[t] = (ntb && v < nb) ? 2.0 * ntb[(int64_t)v * nb + v].x : 0.0;
      }
    }
    // close partners of the columns, for the partial-fraction form
    int partner[PF ? T : 1];
    bool pfk = false;
    if constexpr (PF) pfk = want_s && lr_pf_pairs<T>(eps, nb, c16, beta, partner);
    // one k-point, with the running sum in the direct (PFK false) or the
    // partial-fraction form; the two instantiations keep separate registers
    auto k_body = [&](auto pf_tag) {
      constexpr bool PFK = decltype(pf_tag)::value;
      // projector fragments: RL = 0 kept in registers for the whole k; RL = 1
      // loaded per group of four frequencies at the start of the stage that
      // uses them, so that they do not occupy registers in the other stages;
      // RL = 2 re-read at every use (fewest live registers)
      Proj<NBP> pr;
      if constexpr (RL == 0) {
        lr_load_pa<NBP>(pr, P, nc, nb, q, c16);
        lr_load_pt<NBP>(pr, P, nc, nb, q, c16);
      }
      // running sum of G, column tiles b0 .. b0 + CT; the three-product form
      // needs three accumulators per tile, so it is used here only up to four tiles
      CAcc<M3 && T * CT <= 4> sacc[T][CT];
      // partial-fraction form (see lr_pf_pairs): W of every row tile (three
      // products up to two tiles), and per column tile Y, the diagonal and the
      // close-pair sums in the output layout of R S (register i: orbital q + 4 i)
      CAcc<M3 && T <= 2> pw[PFK ? T : 1];
      v4d yr[PFK ? T : 1], yi[PFK ? T : 1], gr[PFK ? T : 1], gi[PFK ? T : 1];
      // close-pair sums in LDS (lane-private slots), kept only for column tiles
      // where some lane has a close partner
      bool anyc[PFK ? T : 1];
      if constexpr (PFK) {
#pragma unroll
        for (int t = 0; t < T; ++t) {
          pw[t].zero();
          yr[t] = yi[t] = gr[t] = gi[t] = (v4d){0.0, 0.0, 0.0, 0.0};
          anyc[t] = __any(partner[t] >= 0);
          if (anyc[t]) {
#pragma unroll
            for (int i = 0; i < 4; ++i) pfc[(t * 4 + i) * 64 + lane] = make_double2(0.0, 0.0);
          }
        }
      }
      // sum over frequencies of d at band 16 t + c16: the D term of sum_n G,
      // added to the diagonal once per k so that the running sum above is
      // touched only by the matrix cores inside the frequency loop
      double2 dsum[T];
  #pragma unroll
      for (int t = 0; t < T; ++t) dsum[t] = make_double2(0.0, 0.0);
      if (want_s) {
  #pragma unroll
        for (int t = 0; t < T; ++t)
  #pragma unroll
          for (int c = 0; c < CT; ++c) sacc[t][c].zero();
      }
      double trg = 0.0, trg2 = 0.0, mub = 0.0;

      for (int n = n0; n < n1; n += 4) {
        // 0. d_r of the four frequencies, each computed once and read from LDS by
        //    every lane that needs it (a lane would otherwise redo the complex
        //    reciprocal for each band it touches, the same value 4 to 16 times
        //    across the wavefront)
  #pragma unroll
        for (int it = 0; it < NDT; ++it) {
          const int idx = lane + 64 * it;  // < 4 NBP: NBP is a multiple of 16
          const int f = idx / NBP, r = idx - f * NBP;
          const int nf = min(n + f, n1 - 1);
          const double wn = (double)(2 * nf + 1) * M_PI / beta;
          sh.dtab[f][r] = r < nb ? inv_z_minus(mu, wn, EPL ? epl[it] : eps[r]) : make_double2(0.0, 0.0);
        }
        // row ri_ of Sigma(i w) of frequency n + g, for the subtraction in stage
        // 2 (rows past nc read row nc - 1, in bounds, and discard it there).
        // Up to 14 columns it is loaded here, so that the loads are in flight
        // during stage 1; 16 columns would not fit in the registers of the
        // two-wavefront variants, which load it in stage 2.
        constexpr bool SG_EARLY = NC <= 14;
        const double2* sgp =
            reinterpret_cast<const double2*>(a.sigma) + (int64_t)min(n + g, n1 - 1) * nc * nc + min(ri_, nc - 1) * nc;
        double2 sgrow[NC];
        if constexpr (SG_EARLY) {
  #pragma unroll
          for (int j = 0; j < NC; ++j) sgrow[j] = j < nc ? sgp[j] : make_double2(0.0, 0.0);
        }
        wave_sync();
        // 1. X of the four frequencies n .. n+3 (repeating the last one past n1)
        //    into LDS, in the output layout of the matrix core
        if constexpr (RL == 1) lr_load_pt<NBP>(pr, P, nc, nb, q, c16);
        if constexpr (NC <= 8) {
          lr_x_packed<NBP, RL, M3>(pr, P, nc, nb, sh, q, c16);
        } else {
  #pragma unroll
          for (int f = 0; f < 4; ++f) {
            CAcc<M3> x;
            x.zero();
  #pragma unroll
            for (int t = 0; t < T; ++t)
  #pragma unroll
              for (int i = 0; i < 4; ++i) {
                if (16 * t + 4 * i >= nb) break;
                const double2 s = RL == 2 ? lr_proj_here(P, c16, 16 * t + 4 * i + q, nc, nb)
                                          : make_double2(pr.pt_r[t][i], pr.pt_i[t][i]);
                const double2 dd = sh.dtab[f][16 * t + 4 * i + q];
                double2 a1 = cmul(s, dd);
                x.mac_cb(a1.x, a1.y, s.x, s.y);
              }
            const v4d xr = x.re(), xi = x.im();
  #pragma unroll
            for (int i = 0; i < 4; ++i) sh.buf[f][(q + 4 * i) * 17 + c16] = make_double2(xr[i], xi[i]);
          }
        }
        wave_sync();
        // 2. row layout: invert X, subtract Sigma', invert K -> Gl, back to LDS
        {
          // rows past nc start as zero rows and stay zero through both sweeps (the
          // packed X of nc <= 8 leaves rows 8 .. 15 of the tile unwritten, and LDS
          // keeps whatever an earlier work-group left there)
          const bool rin = ri_ < nc;
          double rr[NC], rim[NC];
  #pragma unroll
          for (int j = 0; j < NC; ++j) {
            const double2 v = rin ? sh.buf[g][ri_ * 17 + j] : make_double2(0.0, 0.0);
            rr[j] = v.x;
            rim[j] = v.y;
          }
          rsweep<0, NC>(rr, rim, ri_, nc, bad);
  #pragma unroll
          for (int j = 0; j < NC; ++j) {
            if (j < nc) {
              double2 v = SG_EARLY ? sgrow[j] : sgp[j];
              if (j == ri_) v.x -= edc;
              rr[j] -= rin ? v.x : 0.0;
              rim[j] -= rin ? v.y : 0.0;
            }
          }
          rsweep<0, NC>(rr, rim, ri_, nc, bad);
  #pragma unroll
          for (int j = 0; j < NC; ++j) sh.buf[g][ri_ * 17 + j] = make_double2(rr[j], rim[j]);
          // the packed X of nc <= 8 leaves rows 8 .. 15 unwritten: complete the
          // tile, so that every element outside Gl's nc x nc corner read later is zero
          if constexpr (NC <= 8) {
  #pragma unroll
            for (int j = NC; j < 16; ++j) sh.buf[g][ri_ * 17 + j] = make_double2(0.0, 0.0);
          }
        }
        wave_sync();
        // 3. per frequency: R, then the running sum / G_loc partial or the traces
        if constexpr (RL == 1) {
          if constexpr (KIND == KIND_DENSITY)
            lr_load_pa<NBP>(pr, P, nc, nb, q, c16);
          else
            lr_load_pt<NBP>(pr, P, nc, nb, q, c16);
        }
  #pragma unroll
        for (int f = 0; f < 4; ++f) {
          const int nf = n + f;
          if (nf >= n1) break;
          const double wn = (double)(2 * nf + 1) * M_PI / beta;
          // the k-tile partial this frequency adds to (G_loc, or S G^2 S^dag for
          // the adjoint kind): read here, so that its latency overlaps the
          // products below (the compiler cannot move it above the previous
          // frequency's stores)
          double2* part = reinterpret_cast<double2*>(a.xpart) + ((int64_t)(a.ktile_base + ktile) * a.nw + nf) * 256;
          const bool part_rmw = kk != kk0 && ((KIND == KIND_DENSITY && want_x) || KIND == KIND_ADJ || KIND == KIND_GEN);
          double2 prev[4];
  #pragma unroll
          for (int i = 0; i < 4; ++i)
            prev[i] = (part_rmw && q + 4 * i < nc && c16 < nc) ? part[i * 64 + lane] : make_double2(0.0, 0.0);
          double2 dcol[T];
  #pragma unroll
          for (int t = 0; t < T; ++t) dcol[t] = sh.dtab[f][16 * t + c16];
          if (want_s) {
  #pragma unroll
            for (int t = 0; t < T; ++t) {
              dsum[t].x += dcol[t].x;
              dsum[t].y += dcol[t].y;
            }
          }
          v4d glr, gli, gltr, glti;  // Gl and (adjoint kinds) Gl^T in the output layout
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
            double2 v = sh.buf[f][(q + 4 * i) * 17 + c16];
            glr[i] = v.x;
            gli[i] = v.y;
            if constexpr (KIND == KIND_ADJ || KIND == KIND_GEN) {
              double2 u = sh.buf[f][c16 * 17 + q + 4 * i];
              gltr[i] = u.x;
              glti[i] = u.y;
            }
          }
          const double2* sg = reinterpret_cast<const double2*>(a.sigma) + (int64_t)nf * nc * nc;
          double sa_r[4], sa_i[4];
          v4d sbr, sbi;
  #pragma unroll
          for (int j = 0; j < 4; ++j) {
            int be = q + 4 * j;
            bool in = c16 < nc && be < nc;
            double2 v = in ? sg[c16 * nc + be] : make_double2(0.0, 0.0);
            double2 u = in ? sg[be * nc + c16] : make_double2(0.0, 0.0);
            if (c16 == be && in) {
              v.x -= edc;
              u.x -= edc;
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
          for (int j = 0; j < 4; ++j) {
            if (j >= kc) break;
            va.mac(glr[j], gli[j], sa_r[j], sa_i[j]);
          }
          const v4d vr = va.re(), vi = va.im();
          CAcc<M3> ra;
          ra.set((v4d){sa_r[0], sa_r[1], sa_r[2], sa_r[3]}, (v4d){sa_i[0], sa_i[1], sa_i[2], sa_i[3]});
  #pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (j >= kc) break;
            ra.mac(sbr[j], sbi[j], vr[j], vi[j]);
          }
          const v4d rtr = ra.re(), rti = ra.im();

          if constexpr (KIND == KIND_DENSITY) {
            double chk = 0.0;
  #pragma unroll
            for (int i = 0; i < 4; ++i) chk += glr[i] + gli[i] + rtr[i] + rti[i];
            if (!__builtin_isfinite(chk)) nonfinite = 1;
            if constexpr (PFK) {
              // R in the output layout (R[q + 4 i][c16]) from R^T through this
              // frequency's LDS tile, which every lane has read Gl from
              v4d rnr, rni;
              wave_sync();
              tile_transpose(rtr, rti, rnr, rni, sh.buf[f], q, c16);
  #pragma unroll
              for (int c = 0; c < T; ++c) {
                // Q = (R S)_c;  Y += Q d_v',  diagonal += Q d_v'^2,  close += Q d_p d_v'
                CAcc<M3> qa;
                qa.zero();
  #pragma unroll
                for (int j = 0; j < 4; ++j) {
                  if (j >= kc) break;
                  const double2 s = RL == 2 ? lr_proj_here(P, q + 4 * j, 16 * c + c16, nc, nb)
                                            : make_double2(pr.pa_r[j][c], pr.pa_i[j][c]);
                  qa.mac(rtr[j], rti[j], s.x, s.y);
                }
                const v4d xr = qa.re(), xi = qa.im();
                const double2 d = dcol[c], d2 = cmul(d, d);
                const double2 dp = partner[c] >= 0 ? cmul(d, sh.dtab[f][partner[c]]) : make_double2(0.0, 0.0);
  #pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const double2 x = make_double2(xr[i], xi[i]);
                  const double2 y = cmul(x, d), g = cmul(x, d2), pp = cmul(x, dp);
                  yr[c][i] += y.x;
                  yi[c][i] += y.y;
                  gr[c][i] += g.x;
                  gi[c][i] += g.y;
                  if (anyc[c]) {
                    double2* slot = &pfc[(c * 4 + i) * 64 + lane];
                    const double2 o = *slot;
                    *slot = make_double2(o.x + pp.x, o.y + pp.y);
                  }
                }
              }
              // W_t += (D S^dag)_t R
  #pragma unroll
              for (int t = 0; t < T; ++t) {
                const double2 dt = dcol[t];
  #pragma unroll
                for (int j = 0; j < 4; ++j) {
                  if (j >= kc) break;
                  const double2 s = RL == 2 ? lr_proj_here(P, q + 4 * j, 16 * t + c16, nc, nb)
                                            : make_double2(pr.pa_r[j][t], pr.pa_i[j][t]);
                  const double2 aa = cmul(dt, make_double2(s.x, -s.y));
                  pw[t].mac(aa.x, aa.y, rnr[j], rni[j]);
                }
              }
            } else if (want_s) {
  #pragma unroll
              for (int c = 0; c < CT; ++c) {
                const int b = b0 + c;
                if (16 * b >= nb) break;
                CAcc<M3> qa;
                qa.zero();
  #pragma unroll
                for (int j = 0; j < 4; ++j) {
                  if (j >= kc) break;
                  const double2 s = RL == 2 ? lr_proj_here(P, q + 4 * j, 16 * b + c16, nc, nb)
                                            : make_double2(pr.pa_r[j][b], pr.pa_i[j][b]);
                  qa.mac(rtr[j], rti[j], s.x, s.y);
                }
                v4d qr = qa.re(), qi = qa.im();
                const double2 db = dcol[b];
  #pragma unroll
                for (int i = 0; i < 4; ++i) {
                  double2 v = cmul(make_double2(qr[i], qi[i]), db);
                  qr[i] = v.x;
                  qi[i] = v.y;
                }
  #pragma unroll
                for (int t = 0; t < T; ++t) {
                  if (16 * t >= nb) break;
                  const double2 dt = dcol[t];
  #pragma unroll
                  for (int j = 0; j < 4; ++j) {
                    if (j >= kc) break;
                    const double2 s = RL == 2 ? lr_proj_here(P, q + 4 * j, 16 * t + c16, nc, nb)
                                              : make_double2(pr.pa_r[j][t], pr.pa_i[j][t]);
                    double2 aa = cmul(dt, make_double2(s.x, -s.y));
                    sacc[t][c].mac(aa.x, aa.y, qr[j], qi[j]);
                  }
                }
              }
            }
            if (want_x) {
  #pragma unroll
              for (int i = 0; i < 4; ++i)
                if (q + 4 * i < nc && c16 < nc)
                  part[i * 64 + lane] = make_double2(wk * glr[i] + prev[i].x, wk * gli[i] + prev[i].y);
            }
          } else if constexpr (KIND == KIND_GEN) {
            double chk = 0.0;
  #pragma unroll
            for (int i = 0; i < 4; ++i) chk += glr[i] + gli[i] + rtr[i] + rti[i];
            if (!__builtin_isfinite(chk)) nonfinite = 1;
            auto ptf = [&](int t, int i) -> double2 {
              return RL == 2 ? lr_proj_here(P, c16, 16 * t + 4 * i + q, nc, nb)
                             : make_double2(pr.pt_r[t][i], pr.pt_i[t][i]);
            };
            // every lane has read Gl of this frequency: its LDS tile is free for transposes
            wave_sync();
            // Rr = I + Sigma' Gl
            CAcc<M3> rra;
            {
              v4d id = {0.0, 0.0, 0.0, 0.0}, z = id;
  #pragma unroll
              for (int i = 0; i < 4; ++i) id[i] = (hasdiag && idg == i) ? 1.0 : 0.0;
              rra.set(id, z);
            }
  #pragma unroll
            for (int j = 0; j < 4; ++j) {
              if (j >= kc) break;
              rra.mac(sa_r[j], sa_i[j], glr[j], gli[j]);
            }
            const v4d rrr = rra.re(), rri = rra.im();
            // X2 = S D^2 S^dag
            CAcc<M3> x2a;
            x2a.zero();
  #pragma unroll
            for (int t = 0; t < T; ++t)
  #pragma unroll
              for (int i = 0; i < 4; ++i) {
                if (16 * t + 4 * i >= nb) break;
                const double2 s = ptf(t, i);
                const double2 dd = sh.dtab[f][16 * t + 4 * i + q];
                const double2 a2 = cmul(cmul(s, dd), dd);
                x2a.mac_cb(a2.x, a2.y, s.x, s.y);
              }
            const v4d x2r = x2a.re(), x2i = x2a.im();
            // this k's share of Sigmabar_n^dag
            CAcc<M3> phi;
            phi.zero();
            if (ntb) {
              // Y1 = Nt D S^dag and Y2 = Nt D^2 S^dag, one 16-row tile at a time, each
              // tile contracted at once into P1 = S D Y1 and P2 = S D Y2 + S D^2 Y1
              const double2* nt = fresh(ntb);
              CAcc<M3> p1a, p2a;
              p1a.zero();
              p2a.zero();
  #pragma unroll
              for (int t = 0; t < T; ++t) {
                if (16 * t >= nb) break;
                const int row = 16 * t + c16;
                CAcc<M3> y1a, y2a;
                y1a.zero();
                y2a.zero();
  #pragma unroll
                for (int b = 0; b < T; ++b)
  #pragma unroll
                  for (int j = 0; j < 4; ++j) {
                    if (16 * b + 4 * j >= nb) break;
                    const int col = 16 * b + 4 * j + q;
                    double2 ntv = make_double2(0.0, 0.0);
                    if (row < nb && col < nb) {
                      const double2 u = nt[row * nb + col], v = nt[col * nb + row];
                      ntv = make_double2(u.x + v.x, u.y - v.y);
                    }
                    const double2 s = ptf(b, j);
                    const double2 dd = sh.dtab[f][col];
                    const double2 b1 = cmul(dd, make_double2(s.x, -s.y));
                    const double2 b2 = cmul(dd, b1);
                    y1a.mac(ntv.x, ntv.y, b1.x, b1.y);
                    y2a.mac(ntv.x, ntv.y, b2.x, b2.y);
                  }
                const v4d y1r = y1a.re(), y1i = y1a.im(), y2r = y2a.re(), y2i = y2a.im();
  #pragma unroll
                for (int i = 0; i < 4; ++i) {
                  if (16 * t + 4 * i >= nb) break;
                  const double2 s = ptf(t, i);
                  const double2 dd = sh.dtab[f][16 * t + 4 * i + q];
                  const double2 a1 = cmul(s, dd), a2 = cmul(a1, dd);
                  p1a.mac(a1.x, a1.y, y1r[i], y1i[i]);
                  p2a.mac(a1.x, a1.y, y2r[i], y2i[i]);
                  p2a.mac(a2.x, a2.y, y1r[i], y1i[i]);
                }
              }
              const v4d p1r = p1a.re(), p1i = p1a.im(), p2r = p2a.re(), p2i = p2a.im();
              // Re tr(Nt G^2) = sum_v Nt_vv Re d_v^2 + Re tr(R P2) + Re tr(E F),
              // E = R X2, F = R P1 (formed transposed: F^T = P1^T R^T)
              CAcc<M3> ea, fta;
              ea.zero();
              fta.zero();
  #pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (j >= kc) break;
                ea.mac(rtr[j], rti[j], x2r[j], x2i[j]);
                fta.mac(p1r[j], p1i[j], rtr[j], rti[j]);
              }
              double tn = re_dot4(rtr, rti, p2r, p2i) + re_dot4(ea.re(), ea.im(), fta.re(), fta.im());
              if (q == 0) {
  #pragma unroll
                for (int t = 0; t < T; ++t) tn += ntd[t] * (dcol[t].x * dcol[t].x - dcol[t].y * dcol[t].y);
              }
              mub -= tn / beta;
              // Rl (P1 / beta) Rr = Y + Gl (Sigma' Y),  Y = (P1 / beta) Rr
              const double ib = 1.0 / beta;
              v4d p1tr, p1ti;
              tile_transpose(p1r * ib, p1i * ib, p1tr, p1ti, sh.buf[f], q, c16);
              CAcc<M3> ya;
              ya.zero();
  #pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (j >= kc) break;
                ya.mac(p1tr[j], p1ti[j], rrr[j], rri[j]);
              }
              const v4d yr = ya.re(), yi = ya.im();
              CAcc<M3> za;
              za.zero();
  #pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (j >= kc) break;
                za.mac(sa_r[j], sa_i[j], yr[j], yi[j]);
              }
              const v4d zr = za.re(), zi = za.im();
              phi.set(yr, yi);
  #pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (j >= kc) break;
                phi.mac(gltr[j], glti[j], zr[j], zi[j]);
              }
            }
            if (a.gbar) {
              const double2* gb = reinterpret_cast<const double2*>(a.gbar) + (int64_t)nf * nc * nc;
              // M = S G^2 S^dag = Rl X2 Rr = Y + Gl (Sigma' Y),  Y = X2 Rr; mubar takes -w_k Re<Gbar, M>
              v4d x2tr, x2ti;
              tile_transpose(x2r, x2i, x2tr, x2ti, sh.buf[f], q, c16);
              CAcc<M3> ya;
              ya.zero();
  #pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (j >= kc) break;
                ya.mac(x2tr[j], x2ti[j], rrr[j], rri[j]);
              }
              const v4d yr = ya.re(), yi = ya.im();
              CAcc<M3> za;
              za.zero();
  #pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (j >= kc) break;
                za.mac(sa_r[j], sa_i[j], yr[j], yi[j]);
              }
              const v4d zr = za.re(), zi = za.im();
              CAcc<M3> ma;
              ma.set(yr, yi);
  #pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (j >= kc) break;
                ma.mac(gltr[j], glti[j], zr[j], zi[j]);
              }
              const v4d mr = ma.re(), mi = ma.im();
              double gm = 0.0;
              double hb_r[4], hb_i[4];
  #pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int al = q + 4 * i;
                const bool in = al < nc && c16 < nc;
                const double2 v = in ? gb[al * nc + c16] : make_double2(0.0, 0.0);
                gm += v.x * mr[i] + v.y * mi[i];
                // w_k conj(Gbar)[c16][q + 4 i]: registers of (w_k conj(Gbar))^T
                const double2 u = in ? gb[c16 * nc + al] : make_double2(0.0, 0.0);
                hb_r[i] = wk * u.x;
                hb_i[i] = -wk * u.y;
              }
              mub -= wk * gm;
              // + w_k Gl Gbar^dag Gl = H Gl,  H^T = w_k conj(Gbar) Gl^T
              CAcc<M3> ha;
              ha.zero();
  #pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (j >= kc) break;
                ha.mac(hb_r[j], hb_i[j], gltr[j], glti[j]);
              }
              const v4d htr = ha.re(), hti = ha.im();
  #pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (j >= kc) break;
                phi.mac(htr[j], hti[j], glr[j], gli[j]);
              }
            }
            // stored as Sigmabar_n = (share)^dag, the dense adjoint's partial layout
            v4d ftr, fti;
            tile_transpose(phi.re(), phi.im(), ftr, fti, sh.buf[f], q, c16);
  #pragma unroll
            for (int i = 0; i < 4; ++i)
              if (q + 4 * i < nc && c16 < nc) part[i * 64 + lane] = make_double2(ftr[i] + prev[i].x, prev[i].y - fti[i]);
          } else {
            // X2 = S D^2 S^dag, X3 = S D^3 S^dag of this frequency
            CAcc<M3> x2a, x3a;
            x2a.zero();
            x3a.zero();
  #pragma unroll
            for (int t = 0; t < T; ++t)
  #pragma unroll
              for (int i = 0; i < 4; ++i) {
                if (16 * t + 4 * i >= nb) break;
                const double2 s = RL == 2 ? lr_proj_here(P, c16, 16 * t + 4 * i + q, nc, nb)
                                        : make_double2(pr.pt_r[t][i], pr.pt_i[t][i]);
                const double2 dd = sh.dtab[f][16 * t + 4 * i + q];
                double2 a2 = cmul(cmul(s, dd), dd);
                x2a.mac_cb(a2.x, a2.y, s.x, s.y);
                double2 a3 = cmul(a2, dd);
                x3a.mac_cb(a3.x, a3.y, s.x, s.y);
              }
            const v4d x2r = x2a.re(), x2i = x2a.im(), x3r = x3a.re(), x3i = x3a.im();
            CAcc<M3> ea_;
            ea_.zero();
  #pragma unroll
            for (int j = 0; j < 4; ++j) {
              if (j >= kc) break;
              ea_.mac(rtr[j], rti[j], x2r[j], x2i[j]);
            }
            const v4d er = ea_.re(), ei = ea_.im();
            v4d etr, eti;
            wave_sync();
            tile_transpose(er, ei, etr, eti, sh.buf[f], q, c16);
            double t2 = re_dot4(rtr, rti, x2r, x2i);
            double t3 = re_dot4(rtr, rti, x3r, x3i);
            double ee = re_dot4(er, ei, etr, eti);
            double sd = 0.0, sd2 = 0.0;
            if (q == 0) {
  #pragma unroll
              for (int t = 0; t < T; ++t) {
                sd += dcol[t].x;
                sd2 += dcol[t].x * dcol[t].x - dcol[t].y * dcol[t].y;
              }
            }
            trg += sd + t2;
            trg2 += sd2 + 2.0 * t3 + ee;
            if constexpr (KIND == KIND_ADJ) {
              // M = S G^2 S^dag = (I + Gl Sigma') X2 (I + Sigma' Gl), as
              // Rr = I + Sigma' Gl, Y = X2 Rr, M = Y + Gl (Sigma' Y)
              CAcc<M3> rra;
              {
                v4d id = {0.0, 0.0, 0.0, 0.0}, z = id;
  #pragma unroll
                for (int i = 0; i < 4; ++i) id[i] = (hasdiag && idg == i) ? 1.0 : 0.0;
                rra.set(id, z);
              }
  #pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (j >= kc) break;
                rra.mac(sa_r[j], sa_i[j], glr[j], gli[j]);
              }
              const v4d rrr = rra.re(), rri = rra.im();
              v4d x2tr, x2ti;
              tile_transpose(x2r, x2i, x2tr, x2ti, sh.buf[f], q, c16);
              CAcc<M3> ya;
              ya.zero();
  #pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (j >= kc) break;
                ya.mac(x2tr[j], x2ti[j], rrr[j], rri[j]);
              }
              const v4d yr = ya.re(), yi = ya.im();
              CAcc<M3> za;
              za.zero();
  #pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (j >= kc) break;
                za.mac(sa_r[j], sa_i[j], yr[j], yi[j]);
              }
              const v4d zr = za.re(), zi = za.im();
              CAcc<M3> ma;
              ma.set(yr, yi);
  #pragma unroll
              for (int j = 0; j < 4; ++j) {
                if (j >= kc) break;
                ma.mac(gltr[j], glti[j], zr[j], zi[j]);
              }
              const v4d mr = ma.re(), mi = ma.im();
  #pragma unroll
              for (int i = 0; i < 4; ++i)
                if (q + 4 * i < nc && c16 < nc)
                  part[i * 64 + lane] = make_double2(wk * mr[i] + prev[i].x, wk * mi[i] + prev[i].y);
            }
          }
        }
        wave_sync();
      }  // frequency groups

      if constexpr (PFK) {
        double2* sp = reinterpret_cast<double2*>(a.spart) + (int64_t)wtile * a.s_stride + a.off_s[k];
        // W through LDS (row v, column beta at v * 17 + beta; the tiles are free
        // after the last group), read back as the A operand of W S
        double2* wl = &sh.buf[0][0];
  #pragma unroll
        for (int t = 0; t < T; ++t) {
          const v4d re = pw[t].re(), im = pw[t].im();
  #pragma unroll
          for (int i = 0; i < 4; ++i) wl[(16 * t + q + 4 * i) * 17 + c16] = make_double2(re[i], im[i]);
        }
        wave_sync();
        double2 srow[4][T];  // S[q + 4 j][16 t + c16]
  #pragma unroll
        for (int j = 0; j < 4; ++j)
  #pragma unroll
          for (int t = 0; t < T; ++t) srow[j][t] = lr_proj(P, q + 4 * j, 16 * t + c16, nc, nb);
  #pragma unroll
        for (int c = 0; c < T; ++c) {
          const int vc = 16 * c + c16;
          const double ec = vc < nb ? eps[vc] : 0.0;
          // the diagonal and the close pair: over the orbitals q + 4 i (this lane's
          // registers, then the four lanes of the column)
          double2 dg = make_double2(0.0, 0.0), cl = make_double2(0.0, 0.0);
          const int pv = partner[c];
  #pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double2 sc = make_double2(srow[i][c].x, -srow[i][c].y);
            const double2 gd = cmul(sc, make_double2(gr[c][i], gi[c][i]));
            dg.x += gd.x;
            dg.y += gd.y;
            const double2 spv = pv >= 0 ? lr_proj(P, q + 4 * i, pv, nc, nb) : make_double2(0.0, 0.0);
            const double2 cv = anyc[c] ? pfc[(c * 4 + i) * 64 + lane] : make_double2(0.0, 0.0);
            const double2 cd = cmul(make_double2(spv.x, -spv.y), cv);
            cl.x += cd.x;
            cl.y += cd.y;
          }
  #pragma unroll
          for (int off = 16; off <= 32; off <<= 1) {
            dg.x += __shfl_xor(dg.x, off);
            dg.y += __shfl_xor(dg.y, off);
            cl.x += __shfl_xor(cl.x, off);
            cl.y += __shfl_xor(cl.y, off);
          }
  #pragma unroll
          for (int t = 0; t < T; ++t) {
            // W S - S^dag Y for tile (t, c)
            CAcc<M3 && T <= 2> acc;
            acc.zero();
  #pragma unroll
            for (int j = 0; j < 4; ++j) {
              if (j >= kc) break;
              const double2 wv = wl[(16 * t + c16) * 17 + q + 4 * j];
              acc.mac(wv.x, wv.y, srow[j][c].x, srow[j][c].y);
              acc.mac(-srow[j][t].x, srow[j][t].y, yr[c][j], yi[c][j]);
            }
            const v4d fr = acc.re(), fi = acc.im();
  #pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int v = 16 * t + q + 4 * i;
              const double ev = v < nb ? eps[v] : 0.0;
              double2 val;
              if (t == c && v == vc) {
                val = make_double2(dg.x + dsum[c].x, dg.y + dsum[c].y);
              } else if (v == pv) {
                val = cl;
              } else {
                const double inv = (v < nb && vc < nb) ? 1.0 / (ev - ec) : 0.0;
                val = make_double2(fr[i] * inv, fi[i] * inv);
              }
              sp[((t * T + c) * 4 + i) * 64 + lane] = val;
            }
          }
        }
        wave_sync();  // W's LDS is the next k-point's X tiles
      } else if (want_s) {
        double2* sp = reinterpret_cast<double2*>(a.spart) + (int64_t)wtile * a.s_stride + a.off_s[k];
  #pragma unroll
        for (int t = 0; t < T; ++t)
  #pragma unroll
          for (int c = 0; c < CT; ++c)
  #pragma unroll
            for (int i = 0; i < 4; ++i) {
              int e = (t * T + b0 + c) * 4 + i;
              double2 v = make_double2(sacc[t][c].re()[i], sacc[t][c].im()[i]);
              if (t == b0 + c && hasdiag && idg == i) {
                v.x += dsum[t].x;
                v.y += dsum[t].y;
              }
              sp[e * 64 + lane] = v;
            }
      }
      if constexpr (KIND == KIND_GEN) {
  #pragma unroll
        for (int off = 32; off >= 1; off >>= 1) mub += __shfl_xor(mub, off);
        if (!__builtin_isfinite(mub)) nonfinite = 1;
        if (lane == 0) {
          // [unused, unused, mubar share] in the adjoint layout
          double* tp = a.tpart + ((int64_t)wtile * a.nk + k) * 3;
          tp[0] = 0.0;
          tp[1] = 0.0;
          tp[2] = mub;
        }
      } else if constexpr (KIND != KIND_DENSITY) {
  #pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          trg += __shfl_xor(trg, off);
          trg2 += __shfl_xor(trg2, off);
        }
        if (!__builtin_isfinite(trg) || !__builtin_isfinite(trg2)) nonfinite = 1;
        if (lane == 0) {
          // trace kind: [Re tr G, Re tr G^2]; adjoint kind: the same and a zero mubar share
          constexpr int stride = KIND == KIND_ADJ ? 3 : 2;
          double* tp = a.tpart + ((int64_t)wtile * a.nk + k) * stride;
          tp[0] = trg;
          tp[1] = trg2;
          if constexpr (KIND == KIND_ADJ) tp[2] = 0.0;
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

// NC: columns kept in the row-layout inversions, nc rounded up to 4, 8, 12 or 16.
template <int NBP, int KIND, int RL, bool M3, int NC, bool PF = false>
__device__ __forceinline__ void lr_tile(const DysonArgs& a, int ktile, int wtile, int part, LRShared& sh, int lane,
                                        double2* pfc = nullptr) {
  constexpr int NP = (NBP / 16) / lr_col_tiles<NBP, KIND>();
  if constexpr (NP > 1) {
    if (part) {
      lr_tile_part<NBP, KIND, RL, M3, NC, 1>(a, ktile, wtile, sh, lane);
      return;
    }
  }
  lr_tile_part<NBP, KIND, RL, M3, NC, 0, PF>(a, ktile, wtile, sh, lane, pfc);
}

// Grid: (k tiles x frequency tiles) x column parts, the column part fastest.
template <int NBP, int KIND, int RL, bool M3, int NC, int OCC, bool PF = false>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(OCC))) lr_kernel(DysonArgs a) {
  __shared__ LRShared sh;
  __shared__ double2 pfc[PF ? NBP / 16 * 4 * 64 : 1];
  constexpr int NP = (NBP / 16) / lr_col_tiles<NBP, KIND>();
  const int item = blockIdx.x / NP, part = blockIdx.x % NP;
  lr_tile<NBP, KIND, RL, M3, NC, PF>(a, item / a.n_wtiles, item % a.n_wtiles, part, sh, threadIdx.x, pfc);
}

// Variant id of the low-rank kernel: bit 3 set; projector fragments kept in
// registers for the whole k-point (bits 0 and 4 clear), re-read at every use
// (bit 0) or loaded once per four-frequency group at the start of each stage
// (bit 4); bit 1 = three-product complex arithmetic on the matrix cores;
// bit 2 = two wavefronts per SIMD; bit 6 = the running sum in the
// partial-fraction form (density kind, nc > 8; the other column counts run
// the direct form).  An LRSet lists the variants one instantiation unit
// compiles for one size and kind.
template <int NBP, int KIND, int... VARS>
struct LRSet {
  template <int VAR>
  static hipError_t one(const DysonArgs& a, dim3 grid, hipStream_t s) {
    constexpr int parts = (NBP / 16) / lr_col_tiles<NBP, KIND>();
    constexpr int rl = (VAR & 16) ? 1 : (VAR & 1) ? 2 : 0;
    constexpr bool m3 = (VAR & 2) != 0;
    constexpr int occ = (VAR & 4) ? 2 : 1;
    constexpr bool pf = (VAR & 64) != 0;
    static_assert(!pf || (KIND == KIND_DENSITY && occ == 1 && parts == 1), "partial fractions: density, one part");
    grid.x *= parts;
    // columns of the row-layout inversions: nc rounded up to 8, 12 or 16, with
    // exact 10 (32-band windows) and 14 (48-band windows) for the
    // d-shell and f-shell orbital counts: every column costs a broadcast and
    // four FMAs in each of the nc pivot steps
    if (a.nc <= 8) {
      hipLaunchKernelGGL((lr_kernel<NBP, KIND, rl, m3, 8, occ>), grid, dim3(64), 0, s, a);
      return hipGetLastError();
    }
    if constexpr (NBP == 32) {
      if (a.nc <= 10) {
        hipLaunchKernelGGL((lr_kernel<NBP, KIND, rl, m3, 10, occ, pf>), grid, dim3(64), 0, s, a);
        return hipGetLastError();
      }
    }
    if (a.nc <= 12) {
      hipLaunchKernelGGL((lr_kernel<NBP, KIND, rl, m3, 12, occ, pf>), grid, dim3(64), 0, s, a);
      return hipGetLastError();
    }
    if constexpr (NBP == 48) {
      if (a.nc <= 14) {
        hipLaunchKernelGGL((lr_kernel<NBP, KIND, rl, m3, 14, occ, pf>), grid, dim3(64), 0, s, a);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((lr_kernel<NBP, KIND, rl, m3, 16, occ, pf>), grid, dim3(64), 0, s, a);
    return hipGetLastError();
  }
  static hipError_t launch(int var, const DysonArgs& a, dim3 grid, hipStream_t s) {
    hipError_t r = hipErrorInvalidValue;
    bool hit = ((var == VARS ? (r = one<VARS>(a, grid, s), true) : false) || ...);
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
