// Host side of libdmft: argument checks, workspace layout, tiling plans, kernel
// launches, the chemical-potential search, the batched pass and its hipGraph,
// and the autotuner.  See include/dmft.h for the public contract.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "dmft.h"
#include "dmft_internal.h"

using namespace dmft;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxQueues = 32;  // queue counters of a batched plan
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr int kNbpSizes[] = {16, 32, 48, 64};

int nbp_of(int nb) {
  for (int s : kNbpSizes)
    if (nb <= s) return s;
  return -1;
}

// Tiling of one launch: kt k-points per k-tile, wt frequencies per frequency tile.
struct Tile {
  int kt = 1, wt = 1;
};

enum { KIND_DENSITY = 0, KIND_TRACE = 1, KIND_ADJOINT = 2, KIND_GENERAL = 3 };

// One padded-size bucket of k-points.
struct Bucket {
  int nbp = 0;
  std::vector<int32_t> klist;
  int n_ktiles = 0;
  int ktile_base = 0;
};

// Workspace layout of a single-lattice call.
struct Layout {
  size_t err = 0, out2 = 0, meta_nb = 0, meta_offb = 0, meta_offn = 0, meta_nbp = 0, meta_klist = 0;
  size_t meta_offs = 0;
  size_t spart = 0, xpart = 0, tpart = 0, kscal = 0, ktrace = 0, total = 0;
  int64_t s_stride = 0;
  int n_wtiles = 0, n_ktiles_total = 0;
  std::vector<Bucket> buckets;
  std::vector<int32_t> nb, nbp;
  std::vector<int64_t> off_b, off_n, off_s;
  bool ragged = false;
  int nbp_max = 0;
  int kind = KIND_DENSITY;
  Tile tile;
  size_t tune_a = 0, tune_b = 0;  // autotuner scratch: two result copies
  size_t sc_part = 0;             // partial sums of the impurity level
};

}  // namespace

struct dmft_handle_s {
  int device = 0;
  std::string last_error;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  void* readback = nullptr;         // pinned 64 B: error word and scalars of a mu-search pass
  hipEvent_t staged = nullptr;      // recorded after the last upload from `pinned`
  std::map<std::string, Tile> tune;  // autotuned tiles keyed by kind/size/nk/nw
  std::map<std::string, int> tvar;   // autotuned kernel variant keyed by kind/size
  // batched plan
  struct Iter {
    dmft_lattice lat;
    dmft_sigma sig;
    Layout lay;
    size_t base = 0;  // offset of this iterate's region inside ws
  };
  std::vector<Iter> iters;
  std::vector<std::vector<int32_t>> iter_nb;  // host copies of the ragged window sizes
  int b_tail = 2;
  size_t b_total = 0, b_args = 0, b_items = 0, b_counters = 0, b_mu = 0;
  int b_nbig = 0, b_nsmall = 0, b_nargs = 0, b_wgs = 0;
  bool b_lowrank = false;                // batched items use the low-rank form
  // low-rank form: one persistent launch per item class, in this order
  struct LRClassPlan {
    int nbp, ncls, off, count, grid;
  };
  std::vector<LRClassPlan> b_cls;
  // the class kernels of a pass run concurrently on side streams (fork/join,
  // also inside a captured graph), so that the tail of one class overlaps the
  // next class instead of idling the chip; all streams have the default priority
  std::vector<hipStream_t> b_side;
  bool b_concurrent = true;  // else the classes run one after another on the pass's stream (plan's choice)
  int b_conc_pref = -1;      // -1: the plan times both; 0 / 1: fixed
  int b_tile_pref = -1;      // -1: the plan times every tile candidate; k >= 0: only candidate k
  int b_tile_chosen = -1;    // candidate of the current plan's tiles (-1: the default, untimed)
  hipEvent_t b_fork = nullptr;
  std::vector<hipEvent_t> b_join;
  // kernel timing of the batched pass: one event pair around the whole Dyson
  // section and one per class, recorded by every timed pass and read before
  // the next one; a graph replay is timed by a pair around hipGraphLaunch
  // (events recorded inside a captured graph carry no usable timestamps here),
  // which then also covers the pass's epilogue reductions
  std::pair<hipEvent_t, hipEvent_t> b_tspan{nullptr, nullptr};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> b_tcls;
  bool b_tpending = false;   // span events of a pass not yet read
  bool b_tcls_pending = false;  // per-class events of that pass recorded too
  bool b_capturing = false;  // batched_pass_impl runs under stream capture
  std::vector<double> b_cls_ms;
  int b_form_pref = DMFT_FORM_AUTO;      // form requested for later plans
  void* b_ws = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // kernel timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tev;  // recorded, not yet read
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tfree;
  double t_ms = 0.0;
  int64_t t_count = 0;
};

namespace {

int batched_harvest(dmft_handle h);

int fail(dmft_handle h, int code, const char* fmt, ...) {
  if (h) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    h->last_error = buf;
  }
  return code;
}

// Every HIP call of an entry point goes through HIPCHK, which first refuses a
// planning handle (created without a device): such a handle validates
// arguments and sizes workspaces but never reaches the runtime.
#define HIPCHK(h, expr)                                                                    \
  do {                                                                                     \
    if (!(h) || (h)->device < 0) return fail(h, DMFT_EINVAL, "handle has no device (planning handle)"); \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(h, DMFT_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int check_lattice(dmft_handle h, const dmft_lattice* lat) {
  if (!h) return DMFT_EINVAL;
  if (!lat) return fail(h, DMFT_EINVAL, "lattice is NULL");
  if (lat->nk < 1) return fail(h, DMFT_EINVAL, "nk must be >= 1 (got %d)", lat->nk);
  if (lat->nc < 1 || lat->nc > 16) return fail(h, DMFT_EINVAL, "nc must be in 1..16 (got %d)", lat->nc);
  if (lat->nb_max < lat->nc || lat->nb_max > 64)
    return fail(h, DMFT_EINVAL, "nb_max must be in nc..64 (got %d)", lat->nb_max);
  if (!lat->eps || !lat->wk || !lat->proj) return fail(h, DMFT_EINVAL, "eps, wk and proj must be set");
  if (lat->nb) {
    for (int k = 0; k < lat->nk; ++k)
      if (lat->nb[k] < lat->nc || lat->nb[k] > lat->nb_max)
        return fail(h, DMFT_EINVAL, "nb[%d] = %d outside nc..nb_max", k, lat->nb[k]);
  }
  return DMFT_OK;
}

int check_shapes(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig) {
  int r = check_lattice(h, lat);
  if (r) return r;
  if (!sig) return fail(h, DMFT_EINVAL, "sigma is NULL");
  if (sig->nw < 1) return fail(h, DMFT_EINVAL, "nw must be >= 1 (got %d)", sig->nw);
  if (!(sig->beta > 0) || !std::isfinite(sig->beta))
    return fail(h, DMFT_EINVAL, "beta must be positive and finite");
  if (!sig->sigma || !sig->e_dc) return fail(h, DMFT_EINVAL, "sigma and e_dc must be set");
  return DMFT_OK;
}

std::string tile_key(int kind, int nbp, int nk, int nw) {
  char key[96];
  snprintf(key, sizeof key, "%d/%d/%d/%d", kind, nbp, nk, nw);
  return key;
}

Tile heuristic_tile(int nk, int nw) {
  Tile t;
  // k-tile: keep the G_loc partials (nk/kt x nw x 4 KiB) near 1 GiB at most.
  double xbytes = (double)nk * nw * 4096.0;
  t.kt = std::max(1, (int)std::ceil(xbytes / (1u << 30)));
  t.kt = std::min(t.kt, std::max(1, nk / 4));
  // frequency tile: aim at >= 4096 work-groups in total (>= 2 per wavefront slot).
  int n_ktiles = (nk + t.kt - 1) / t.kt;
  int want_wtiles = std::max(1, (4096 + n_ktiles - 1) / n_ktiles);
  t.wt = std::max(4, (nw + want_wtiles - 1) / want_wtiles);
  t.wt = std::min(t.wt, nw);
  return t;
}

Tile choose_tile(const dmft_handle h, int kind, int nk, int nw, int nbp) {
  auto it = h->tune.find(tile_key(kind, nbp, nk, nw));
  return it != h->tune.end() ? it->second : heuristic_tile(nk, nw);
}

const char* kind_name(int kind) {
  return kind == KIND_DENSITY ? "density" : kind == KIND_TRACE ? "trace" : kind == KIND_ADJOINT ? "adjoint" : "general";
}

int choose_var(const dmft_handle h, int kind, int nbp) {
  char key[32];
  snprintf(key, sizeof key, "%d/%d", kind, nbp);
  auto it = h->tvar.find(key);
  if (it != h->tvar.end()) return it->second;
  int v[16];
  return dyson_variants(nbp, kind, v, 16) > 0 ? v[0] : -1;
}

// Build the workspace layout for one lattice.
int make_layout(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, Layout& L, int kind,
                const Tile* force = nullptr) {
  int nk = lat->nk, nw = sig->nw;
  L.ragged = lat->nb != nullptr;
  L.nb.assign(nk, lat->nb_max);
  if (lat->nb)
    for (int k = 0; k < nk; ++k) L.nb[k] = lat->nb[k];
  L.off_b.assign(nk + 1, 0);
  L.off_n.assign(nk + 1, 0);
  L.off_s.assign(nk + 1, 0);
  L.nbp.assign(nk, 0);
  for (int k = 0; k < nk; ++k) {
    L.off_b[k + 1] = L.off_b[k] + L.nb[k];
    L.off_n[k + 1] = L.off_n[k] + (int64_t)L.nb[k] * L.nb[k];
    L.nbp[k] = nbp_of(L.nb[k]);
    if (!dyson_supported(L.nbp[k]))
      return fail(h, DMFT_EUNSUPPORTED, "no kernel variant for nb = %d", L.nb[k]);
    L.off_s[k + 1] = L.off_s[k] + (int64_t)L.nbp[k] * L.nbp[k];
  }
  L.nbp_max = *std::max_element(L.nbp.begin(), L.nbp.end());
  L.kind = kind;
  L.tile = force ? *force : choose_tile(h, kind, nk, nw, L.nbp_max);
  L.tile.wt = std::max(1, std::min(L.tile.wt, nw));
  L.tile.kt = std::max(1, std::min(L.tile.kt, nk));
  L.n_wtiles = (nw + L.tile.wt - 1) / L.tile.wt;
  L.buckets.clear();
  int base = 0;
  for (int s : kNbpSizes) {
    Bucket b;
    b.nbp = s;
    for (int k = 0; k < nk; ++k)
      if (L.nbp[k] == s) b.klist.push_back(k);
    if (b.klist.empty()) continue;
    b.n_ktiles = ((int)b.klist.size() + L.tile.kt - 1) / L.tile.kt;
    b.ktile_base = base;
    base += b.n_ktiles;
    L.buckets.push_back(b);
  }
  L.n_ktiles_total = base;
  // the kernels are compiled for one padded size each and take nb_k within
  // (NBP - 16, NBP] as given (they skip the chunk tests of all but the last
  // 16 bands); every k of a bucket must satisfy that
  for (const Bucket& b : L.buckets)
    for (int32_t k : b.klist)
      if (!(L.nb[k] > b.nbp - 16 && L.nb[k] <= b.nbp))
        return fail(h, DMFT_EUNSUPPORTED, "internal: nb[%d] = %d outside the bucket of padded size %d", k, L.nb[k],
                    b.nbp);
  L.s_stride = L.off_s[nk];
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  // error word (int at offset 0) followed, 16 bytes on, by the small device
  // results (N_tot and dN/dmu of a trace pass, the adjoint scalars), so the mu
  // search reads both back with one copy
  L.err = take(16 + 16 * sizeof(double));
  L.out2 = L.err + 16;
  L.meta_nb = take(sizeof(int32_t) * nk);
  L.meta_offb = take(sizeof(int64_t) * (nk + 1));
  L.meta_offn = take(sizeof(int64_t) * (nk + 1));
  L.meta_nbp = take(sizeof(int32_t) * nk);
  L.meta_klist = take(sizeof(int32_t) * nk);
  L.meta_offs = take(sizeof(int64_t) * (nk + 1));
  L.spart = take((size_t)L.n_wtiles * L.s_stride * 16);
  L.xpart = take((size_t)L.n_ktiles_total * nw * 256 * 16);
  L.tpart = take((size_t)L.n_wtiles * nk * 3 * sizeof(double));
  L.kscal = take((size_t)nk * 3 * sizeof(double));
  L.ktrace = take((size_t)nk * 2 * sizeof(double));
  L.tune_a = take((size_t)nw * lat->nc * lat->nc * 16 + 64);
  L.tune_b = take((size_t)nw * lat->nc * lat->nc * 16 + 64);
  L.sc_part = take((size_t)kScParts * lat->nc * lat->nc * 16);
  L.total = o;
  return DMFT_OK;
}

int check_ws(dmft_handle h, const Layout& L, void* ws, size_t ws_bytes) {
  if (!ws) return fail(h, DMFT_EWORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % kAlign) return fail(h, DMFT_EWORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(h, DMFT_EWORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  return DMFT_OK;
}

// Upload the per-k metadata (sizes, offsets, bucket k lists) into ws.
int upload_meta(dmft_handle h, const Layout& L, char* ws, hipStream_t s, bool sync) {
  size_t nk = L.nb.size();
  size_t need = sizeof(int32_t) * nk * 3 + sizeof(int64_t) * (nk + 1) * 3;
  if (h->staged) HIPCHK(h, hipEventSynchronize(h->staged));
  if (need > h->pinned_bytes) {
    if (h->pinned) HIPCHK(h, hipHostFree(h->pinned));
    h->pinned = nullptr;
    HIPCHK(h, hipHostMalloc(&h->pinned, need, hipHostMallocDefault));
    h->pinned_bytes = need;
  }
  char* p = (char*)h->pinned;
  int32_t* nbv = (int32_t*)p;
  int64_t* offb = (int64_t*)(nbv + nk);
  int64_t* offn = offb + nk + 1;
  int32_t* nbpv = (int32_t*)(offn + nk + 1);
  int32_t* kl = nbpv + nk;
  int64_t* offs = (int64_t*)(kl + nk);
  std::copy(L.nb.begin(), L.nb.end(), nbv);
  std::copy(L.off_b.begin(), L.off_b.end(), offb);
  std::copy(L.off_n.begin(), L.off_n.end(), offn);
  std::copy(L.nbp.begin(), L.nbp.end(), nbpv);
  std::copy(L.off_s.begin(), L.off_s.end(), offs);
  size_t at = 0;
  for (const Bucket& b : L.buckets) {
    std::copy(b.klist.begin(), b.klist.end(), kl + at);
    at += b.klist.size();
  }
  HIPCHK(h, hipMemcpyAsync(ws + L.meta_nb, nbv, sizeof(int32_t) * nk, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(ws + L.meta_offb, offb, sizeof(int64_t) * (nk + 1), hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(ws + L.meta_offn, offn, sizeof(int64_t) * (nk + 1), hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(ws + L.meta_nbp, nbpv, sizeof(int32_t) * nk, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(ws + L.meta_klist, kl, sizeof(int32_t) * nk, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(ws + L.meta_offs, offs, sizeof(int64_t) * (nk + 1), hipMemcpyHostToDevice, s));
  if (!h->staged) HIPCHK(h, hipEventCreateWithFlags(&h->staged, hipEventDisableTiming));
  HIPCHK(h, hipEventRecord(h->staged, s));
  if (sync) HIPCHK(h, hipEventSynchronize(h->staged));
  return DMFT_OK;
}

double sum_inv_w2(int nw, double beta) {
  double s2 = 0.0;
  for (int n = 0; n < nw; ++n) {
    double w = (2.0 * n + 1.0) * M_PI / beta;
    s2 += 1.0 / (w * w);
  }
  return s2;
}

// Enqueue the Dyson kernel(s) for all buckets with the given mode.
struct AdjReq {
  int gen = -1;  // -1: Dyson kernel; 0/1: adjoint kernel generation
  const double* nbar = nullptr;
  const double* gbar = nullptr;
};

int run_dyson(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, const Layout& L,
              char* ws, double mu, const double* mu_ptr, int mode, hipStream_t s, const AdjReq& adj = AdjReq()) {
  DysonArgs a{};
  a.nk = lat->nk;
  a.nc = lat->nc;
  a.nw = sig->nw;
  a.nb_uniform = L.ragged ? 0 : lat->nb_max;
  a.nb = (const int32_t*)(ws + L.meta_nb);
  a.off_b = (const int64_t*)(ws + L.meta_offb);
  a.eps = lat->eps;
  a.wk = lat->wk;
  a.proj = lat->proj;
  a.beta = sig->beta;
  a.sigma = sig->sigma;
  a.e_dc = sig->e_dc;
  a.mu = mu;
  a.mu_ptr = mu_ptr;
  a.kt = L.tile.kt;
  a.wt = L.tile.wt;
  a.n_wtiles = L.n_wtiles;
  a.mode = mode;
  a.spart = (double*)(ws + L.spart);
  a.s_stride = L.s_stride;
  a.off_s = (const int64_t*)(ws + L.meta_offs);
  a.xpart = (double*)(ws + L.xpart);
  a.tpart = (double*)(ws + L.tpart);
  a.err = (int*)(ws + L.err);
  size_t at = 0;
  for (const Bucket& b : L.buckets) {
    a.klist = L.ragged || L.buckets.size() > 1 ? (const int32_t*)(ws + L.meta_klist) + at : nullptr;
    a.nklist = (int)b.klist.size();
    a.ktile_base = b.ktile_base;
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (h->timing) {
      if (!h->tfree.empty()) {
        ev = h->tfree.back();
        h->tfree.pop_back();
      } else {
        HIPCHK(h, hipEventCreate(&ev.first));
        HIPCHK(h, hipEventCreate(&ev.second));
      }
      HIPCHK(h, hipEventRecord(ev.first, s));
    }
    if (adj.gen == 0 && (choose_var(h, KIND_ADJOINT, b.nbp) & 8)) {
      // fused scalar adjoint in the low-rank form (same partials as the dense kernel)
      DysonArgs aa = a;
      aa.mode = MODE_ADJ;
      HIPCHK(h, launch_dyson(b.nbp, choose_var(h, KIND_ADJOINT, b.nbp), aa, b.n_ktiles, s));
    } else if (adj.gen == 1 && (choose_var(h, KIND_GENERAL, b.nbp) & 8)) {
      // general vector-Jacobian product in the low-rank form (same partials as the dense kernel)
      DysonArgs aa = a;
      aa.mode = MODE_GEN;
      aa.nbar = adj.nbar;
      aa.off_n = L.ragged ? (const int64_t*)(ws + L.meta_offn) : nullptr;
      aa.gbar = adj.gbar;
      HIPCHK(h, launch_dyson(b.nbp, choose_var(h, KIND_GENERAL, b.nbp), aa, b.n_ktiles, s));
    } else if (adj.gen >= 0) {
      if (b.nbp > 48) return fail(h, DMFT_EUNSUPPORTED, "the dense adjoint supports band windows up to 48");
      HIPCHK(h, launch_adjoint(b.nbp, adj.gen, a, adj.nbar, L.ragged ? (const int64_t*)(ws + L.meta_offn) : nullptr,
                               adj.gbar, (double*)(ws + L.xpart), (double*)(ws + L.tpart), b.n_ktiles, s));
    } else {
      const int kind = (mode & MODE_TRACE) ? KIND_TRACE : KIND_DENSITY;
      int var = choose_var(h, kind, b.nbp);
      // the three-frequency packing serves nc <= 5 only; the variant chosen for
      // this size (by the autotuner on another shape, or by the caller) falls
      // back to the size's default elsewhere
      if (var == kLowrankP3Variant && !lowrank_p3_fits(b.nbp, lat->nc)) {
        int v[16];
        var = dyson_variants(b.nbp, kind, v, 16) > 0 ? v[0] : var;
      }
      HIPCHK(h, launch_dyson(b.nbp, var, a, b.n_ktiles, s));
    }
    if (h->timing) {
      HIPCHK(h, hipEventRecord(ev.second, s));
      h->tev.push_back(ev);
    }
    at += b.klist.size();
  }
  return DMFT_OK;
}

EpilogueArgs epilogue_args(const dmft_lattice* lat, const dmft_sigma* sig, const Layout& L,
                           char* ws, double mu, const double* mu_ptr, int tail_order) {
  EpilogueArgs e{};
  e.nk = lat->nk;
  e.nc = lat->nc;
  e.nw = sig->nw;
  e.nb_uniform = L.ragged ? 0 : lat->nb_max;
  e.nb = (const int32_t*)(ws + L.meta_nb);
  e.off_b = (const int64_t*)(ws + L.meta_offb);
  e.off_n = (const int64_t*)(ws + L.meta_offn);
  e.nbp = (const int32_t*)(ws + L.meta_nbp);
  e.eps = lat->eps;
  e.wk = lat->wk;
  e.proj = lat->proj;
  e.beta = sig->beta;
  e.sigma_inf = sig->sigma_inf;
  e.e_dc = sig->e_dc;
  e.mu = mu;
  e.mu_ptr = mu_ptr;
  e.tail_order = tail_order;
  e.n_wtiles = L.n_wtiles;
  e.spart = (const double*)(ws + L.spart);
  e.s_stride = L.s_stride;
  e.off_s = (const int64_t*)(ws + L.meta_offs);
  e.tpart = (const double*)(ws + L.tpart);
  e.kscal = (double*)(ws + L.kscal);
  e.ktrace = (double*)(ws + L.ktrace);
  e.s2 = sum_inv_w2(sig->nw, sig->beta);
  return e;
}

int prepare(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, void* ws, size_t ws_bytes,
            Layout& L, int kind, hipStream_t s) {
  int r = check_shapes(h, lat, sig);
  if (r) return r;
  r = make_layout(h, lat, sig, L, kind);
  if (r) return r;
  r = check_ws(h, L, ws, ws_bytes);
  if (r) return r;
  HIPCHK(h, hipSetDevice(h->device));
  return upload_meta(h, L, (char*)ws, s, false);
}

int density_impl(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, const Layout& L,
                 char* ws, double mu, const double* mu_ptr, int tail_order, double* nk, double* gloc,
                 double* scalars, hipStream_t s) {
  int mode = 0;
  if (nk || scalars) mode |= MODE_S;
  if (gloc) mode |= MODE_GLOC;
  int r = run_dyson(h, lat, sig, L, ws, mu, mu_ptr, mode, s);
  if (r) return r;
  EpilogueArgs e = epilogue_args(lat, sig, L, ws, mu, mu_ptr, tail_order);
  if (mode & MODE_S) {
    HIPCHK(h, launch_nk_epilogue(e, nk, s));
    if (scalars) HIPCHK(h, launch_scalar_reduce(lat->nk, lat->wk, e.kscal, 3, scalars, s));
  }
  if (gloc) HIPCHK(h, launch_gloc_reduce(L.n_ktiles_total, sig->nw, lat->nc,
                                         (const double*)(ws + L.xpart), gloc, s));
  return DMFT_OK;
}

int ntot_impl(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, const Layout& L,
              char* ws, double mu, const double* mu_ptr, int tail_order, double* out, hipStream_t s) {
  int r = run_dyson(h, lat, sig, L, ws, mu, mu_ptr, MODE_TRACE, s);
  if (r) return r;
  EpilogueArgs e = epilogue_args(lat, sig, L, ws, mu, mu_ptr, tail_order);
  HIPCHK(h, launch_trace_epilogue(e, s));
  HIPCHK(h, launch_scalar_reduce(lat->nk, lat->wk, e.ktrace, 2, out, s));
  return DMFT_OK;
}

}  // namespace

// ============================================================ allocation-free density pass

namespace dmft {

// density_matrix on a caller-independent scratch buffer (the library's
// file-scope device array, see noalloc.hip): uniform band windows only, so the
// per-k metadata is generated on the device instead of staged through pinned
// host memory, and tiles coarsened until the layout fits `cap` bytes.  Makes
// no allocating call: no device or pinned allocation, no event creation.
int density_noalloc_impl(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu, int tail_order,
                         double* nk, double* gloc, double* scalars, int32_t* status, hipStream_t s) {
  if (!h) return DMFT_EINVAL;
  if (tail_order != 0 && tail_order != 2) return fail(h, DMFT_EINVAL, "tail_order must be 0 or 2");
  if (!nk && !gloc && !scalars) return fail(h, DMFT_EINVAL, "no output requested");
  if (!std::isfinite(mu)) return fail(h, DMFT_EINVAL, "mu is not finite");
  int r = check_shapes(h, lat, sig);
  if (r) return r;
  if (lat->nb)
    for (int k = 0; k < lat->nk; ++k)
      if (lat->nb[k] != lat->nb_max)
        return fail(h, DMFT_EINVAL, "the allocation-free pass takes uniform band windows (nb[%d] = %d, nb_max = %d)",
                    k, lat->nb[k], lat->nb_max);
  dmft_lattice u = *lat;
  u.nb = nullptr;
  const size_t cap = noalloc_scratch_bytes();
  Layout L;
  Tile t = choose_tile(h, KIND_DENSITY, u.nk, sig->nw, nbp_of(u.nb_max));
  for (;;) {
    r = make_layout(h, &u, sig, L, KIND_DENSITY, &t);
    if (r) return r;
    if (L.total <= cap) break;
    // fewer k tiles shrink the G_loc partials, fewer frequency tiles those of sum_n G
    if (t.kt < u.nk) {
      t.kt = std::min(u.nk, 2 * t.kt);
    } else if (t.wt < sig->nw) {
      t.wt = std::min(sig->nw, 2 * t.wt);
    } else {
      return fail(h, DMFT_EWORKSPACE, "this shape needs %zu bytes of scratch; the allocation-free scratch holds %zu",
                  L.total, cap);
    }
  }
  if (h->device < 0) return fail(h, DMFT_EINVAL, "handle has no device (planning handle)");
  char* w = (char*)noalloc_scratch(h->device);
  if (!w) return fail(h, DMFT_EHIP, "no scratch address for device %d", h->device);
  HIPCHK(h, hipSetDevice(h->device));
  // metadata and a cleared error word (a kernel: the scratch keeps the last call's contents)
  HIPCHK(h, launch_uniform_meta(u.nk, u.nb_max, nbp_of(u.nb_max), (int32_t*)(w + L.meta_nb),
                                (int64_t*)(w + L.meta_offb), (int64_t*)(w + L.meta_offn), (int32_t*)(w + L.meta_nbp),
                                (int32_t*)(w + L.meta_klist), (int64_t*)(w + L.meta_offs), (int*)(w + L.err), s));
  const bool timing = h->timing;
  h->timing = false;  // timing would create events
  r = density_impl(h, &u, sig, L, w, mu, nullptr, tail_order, nk, gloc, scalars, s);
  h->timing = timing;
  if (r) return r;
  if (status) HIPCHK(h, launch_status_code((const int*)(w + L.err), status, s));
  return DMFT_OK;
}

}  // namespace dmft

// ============================================================================ C ABI

extern "C" {

int density_matrix_noalloc(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu, int tail_order,
                           double* nk, double* gloc, double* scalars, int32_t* status, hipStream_t stream) {
  return dmft::density_noalloc_impl(h, lat, sig, mu, tail_order, nk, gloc, scalars, status, stream);
}

const char* dmft_strerror(int status) {
  switch (status) {
    case DMFT_OK: return "ok";
    case DMFT_EINVAL: return "invalid argument";
    case DMFT_EHIP: return "HIP runtime error";
    case DMFT_ENONFINITE: return "non-finite value on the device";
    case DMFT_ESINGULAR: return "vanishing pivot (singular Dyson matrix)";
    case DMFT_ENOCONV: return "chemical-potential search did not converge";
    case DMFT_EWORKSPACE: return "workspace missing, misaligned or too small";
    case DMFT_EUNSUPPORTED: return "shape not supported by the compiled kernels";
    default: return "unknown status";
  }
}

int dmft_create(dmft_handle* out, int device) {
  if (!out) return DMFT_EINVAL;
  *out = nullptr;
  if (device == DMFT_NO_DEVICE) {
    // planning handle: no HIP call now or later (HIPCHK refuses it)
    dmft_handle h = new dmft_handle_s;
    h->device = DMFT_NO_DEVICE;
    *out = h;
    return DMFT_OK;
  }
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DMFT_EHIP;
  if (hipSetDevice(device) != hipSuccess) return DMFT_EHIP;
  // the allocation-free entry point's scratch address on this device (once per device)
  if (noalloc_setup(device) != hipSuccess) return DMFT_EHIP;
  dmft_handle h = new dmft_handle_s;
  h->device = device;
  *out = h;
  return DMFT_OK;
}

int dmft_destroy(dmft_handle h) {
  if (!h) return DMFT_EINVAL;
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->cap_stream) (void)hipStreamSynchronize(h->cap_stream);
  for (hipStream_t st : h->b_side) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (hipEvent_t e : h->b_join) (void)hipEventDestroy(e);
  if (h->b_fork) (void)hipEventDestroy(h->b_fork);
  if (h->b_tspan.first) (void)hipEventDestroy(h->b_tspan.first);
  if (h->b_tspan.second) (void)hipEventDestroy(h->b_tspan.second);
  for (auto& ev : h->b_tcls) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->staged) {
    (void)hipEventSynchronize(h->staged);
    (void)hipEventDestroy(h->staged);
  }
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->readback) (void)hipHostFree(h->readback);
  for (auto& ev : h->tev) {
    (void)hipEventSynchronize(ev.second);
    h->tfree.push_back(ev);
  }
  for (auto& ev : h->tfree) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  delete h;
  return DMFT_OK;
}

const char* dmft_last_error(dmft_handle h) { return h ? h->last_error.c_str() : ""; }

int dmft_workspace_size(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, size_t* bytes) {
  if (!bytes) return fail(h, DMFT_EINVAL, "bytes is NULL");
  int r = check_shapes(h, lat, sig);
  if (r) return r;
  Layout L, L2;
  r = make_layout(h, lat, sig, L, KIND_DENSITY);
  if (r) return r;
  r = make_layout(h, lat, sig, L2, KIND_TRACE);
  if (r) return r;
  Layout L3;
  r = make_layout(h, lat, sig, L3, KIND_ADJOINT);
  if (r) return r;
  *bytes = std::max(std::max(L.total, L2.total), L3.total);
  return DMFT_OK;
}

int gloc_compute(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu, double* gloc,
                 void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!gloc) return fail(h, DMFT_EINVAL, "gloc is NULL");
  Layout L;
  int r = prepare(h, lat, sig, ws, ws_bytes, L, KIND_DENSITY, stream);
  if (r) return r;
  return density_impl(h, lat, sig, L, (char*)ws, mu, nullptr, 2, nullptr, gloc, nullptr, stream);
}

int dmft_hybridization(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu, const double* gloc,
                       double* delta, double* e_imp, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!gloc || !delta) return fail(h, DMFT_EINVAL, "gloc and delta are required");
  if (!std::isfinite(mu)) return fail(h, DMFT_EINVAL, "mu is not finite");
  Layout L;
  int r = check_shapes(h, lat, sig);
  if (r) return r;
  r = make_layout(h, lat, sig, L, KIND_DENSITY);
  if (r) return r;
  r = check_ws(h, L, ws, ws_bytes);
  if (r) return r;
  HIPCHK(h, hipSetDevice(h->device));
  // uniform windows: the kernels take nb from the argument and read no per-k metadata
  if (L.ragged) {
    r = upload_meta(h, L, (char*)ws, stream, false);
    if (r) return r;
  }
  char* w = (char*)ws;
  double* eimp = e_imp ? e_imp : (double*)(w + L.tune_a);  // scratch when not requested
  HIPCHK(h, launch_self_consistency(lat->nk, lat->nc, sig->nw, L.ragged ? 0 : lat->nb_max,
                                    (const int32_t*)(w + L.meta_nb), (const int64_t*)(w + L.meta_offb), lat->eps,
                                    lat->wk, lat->proj, sig->e_dc, sig->beta, mu, gloc, sig->sigma, eimp, delta,
                                    (double*)(w + L.sc_part), (int*)(w + L.err), stream));
  return DMFT_OK;
}

int density_matrix(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu, int tail_order,
                   double* nk, double* gloc, double* scalars, void* ws, size_t ws_bytes,
                   hipStream_t stream) {
  if (tail_order != 0 && tail_order != 2) return fail(h, DMFT_EINVAL, "tail_order must be 0 or 2");
  if (!nk && !gloc && !scalars) return fail(h, DMFT_EINVAL, "no output requested");
  if (!std::isfinite(mu)) return fail(h, DMFT_EINVAL, "mu is not finite");
  Layout L;
  int r = prepare(h, lat, sig, ws, ws_bytes, L, KIND_DENSITY, stream);
  if (r) return r;
  return density_impl(h, lat, sig, L, (char*)ws, mu, nullptr, tail_order, nk, gloc, scalars, stream);
}

int dmft_ntot(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu, int tail_order,
              double* out, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (tail_order != 0 && tail_order != 2) return fail(h, DMFT_EINVAL, "tail_order must be 0 or 2");
  if (!out) return fail(h, DMFT_EINVAL, "out is NULL");
  if (!std::isfinite(mu)) return fail(h, DMFT_EINVAL, "mu is not finite");
  Layout L;
  int r = prepare(h, lat, sig, ws, ws_bytes, L, KIND_TRACE, stream);
  if (r) return r;
  return ntot_impl(h, lat, sig, L, (char*)ws, mu, nullptr, tail_order, out, stream);
}

}  // extern "C"

namespace {

// Fused scalar adjoint of N_tot on a prepared layout: out = [N_tot, dN/dmu]
// (device, may be NULL), sigma_bar = dN/dSigma (device [nw][nc][nc], may be NULL).
int ntot_vjp_impl(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, const Layout& L, char* w, double mu,
                  int tail_order, double* sigma_bar, double* out, hipStream_t stream) {
  AdjReq adj;
  adj.gen = 0;
  int r = run_dyson(h, lat, sig, L, w, mu, nullptr, 0, stream, adj);
  if (r) return r;
  EpilogueArgs e = epilogue_args(lat, sig, L, w, mu, nullptr, tail_order);
  if (out) {
    HIPCHK(h, launch_adj_epilogue(e, nullptr, stream));
    // per-k values are [tr N, d tr N/dmu, mubar_k]: reduce all three, return the first two
    HIPCHK(h, launch_scalar_reduce_mask(lat->nk, lat->wk, e.kscal, 3, 4, (double*)(w + L.out2), stream));
    HIPCHK(h, hipMemcpyAsync(out, w + L.out2, 2 * sizeof(double), hipMemcpyDeviceToDevice, stream));
  }
  if (sigma_bar)
    HIPCHK(h, launch_sigma_bar_reduce(L.n_ktiles_total, sig->nw, lat->nc, (const double*)(w + L.xpart),
                                      2.0 / sig->beta, 1, sigma_bar, stream));
  return DMFT_OK;
}

}  // namespace

extern "C" {

int dmft_variants(int kind, int nbp, int* out, int max) {
  if (kind < 0 || kind > 3) return 0;
  int v[16];
  int n = dyson_variants(nbp, kind, v, 16);
  for (int i = 0; i < n && i < max && out; ++i) out[i] = v[i];
  return n;
}

int dmft_get_variant(dmft_handle h, int kind, int nbp) {
  if (!h || kind < 0 || kind > 3) return -1;
  return choose_var(h, kind, nbp);
}

int dmft_set_variant(dmft_handle h, int kind, int nbp, int var) {
  if (!h) return DMFT_EINVAL;
  char key[32];
  snprintf(key, sizeof key, "%d/%d", kind, nbp);
  if (var < 0) {
    h->tvar.erase(key);
    return DMFT_OK;
  }
  int v[16];
  int n = dyson_variants(nbp, kind, v, 16);
  for (int i = 0; i < n; ++i)
    if (v[i] == var) {
      h->tvar[key] = var;
      return DMFT_OK;
    }
  return fail(h, DMFT_EINVAL, "variant %d not instantiated for kind %d, nbp %d", var, kind, nbp);
}

int dmft_timing(dmft_handle h, int enable, double* kernel_ms, int64_t* launches) {
  if (!h) return DMFT_EINVAL;
  int rb = batched_harvest(h);
  if (rb) return rb;
  for (auto& ev : h->tev) {
    HIPCHK(h, hipEventSynchronize(ev.second));
    float ms = 0.f;
    HIPCHK(h, hipEventElapsedTime(&ms, ev.first, ev.second));
    h->t_ms += ms;
    h->t_count += 1;
    h->tfree.push_back(ev);
  }
  h->tev.clear();
  if (kernel_ms) *kernel_ms = h->t_ms;
  if (launches) *launches = h->t_count;
  if (enable) {
    h->t_ms = 0.0;
    h->t_count = 0;
    std::fill(h->b_cls_ms.begin(), h->b_cls_ms.end(), 0.0);
  }
  h->timing = enable != 0;
  return DMFT_OK;
}

int dmft_ntot_vjp(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu, int tail_order,
                  double* sigma_bar, double* out, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (tail_order != 0 && tail_order != 2) return fail(h, DMFT_EINVAL, "tail_order must be 0 or 2");
  if (!sigma_bar && !out) return fail(h, DMFT_EINVAL, "no output requested");
  if (!std::isfinite(mu)) return fail(h, DMFT_EINVAL, "mu is not finite");
  Layout L;
  int r = prepare(h, lat, sig, ws, ws_bytes, L, KIND_ADJOINT, stream);
  if (r) return r;
  return ntot_vjp_impl(h, lat, sig, L, (char*)ws, mu, tail_order, sigma_bar, out, stream);
}

int density_matrix_vjp(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu, int tail_order,
                       const double* nk_bar, const double* gloc_bar, double* sigma_bar, double* mu_bar, void* ws,
                       size_t ws_bytes, hipStream_t stream) {
  if (tail_order != 0 && tail_order != 2) return fail(h, DMFT_EINVAL, "tail_order must be 0 or 2");
  if (!sigma_bar) return fail(h, DMFT_EINVAL, "sigma_bar is NULL");
  if (!std::isfinite(mu)) return fail(h, DMFT_EINVAL, "mu is not finite");
  Layout L;
  int r = prepare(h, lat, sig, ws, ws_bytes, L, KIND_ADJOINT, stream);
  if (r) return r;
  char* w = (char*)ws;
  AdjReq adj;
  adj.gen = 1;
  adj.nbar = nk_bar;
  adj.gbar = gloc_bar;
  r = run_dyson(h, lat, sig, L, w, mu, nullptr, 0, stream, adj);
  if (r) return r;
  HIPCHK(h, launch_sigma_bar_reduce(L.n_ktiles_total, sig->nw, lat->nc, (const double*)(w + L.xpart), 1.0, 0,
                                    sigma_bar, stream));
  if (mu_bar) {
    EpilogueArgs e = epilogue_args(lat, sig, L, w, mu, nullptr, tail_order);
    HIPCHK(h, launch_adj_epilogue(e, nk_bar, stream));
    // mubar = sum_k mubar_k (unweighted: the k weights are inside C)
    HIPCHK(h, launch_scalar_reduce_mask(lat->nk, lat->wk, e.kscal, 3, 4, (double*)(w + L.out2), stream));
    HIPCHK(h, hipMemcpyAsync(mu_bar, w + L.out2 + 2 * sizeof(double), sizeof(double), hipMemcpyDeviceToDevice,
                             stream));
  }
  return DMFT_OK;
}

int dmft_sync_status(dmft_handle h, void* ws, hipStream_t stream) {
  if (!h || !ws) return fail(h, DMFT_EINVAL, "handle or workspace is NULL");
  HIPCHK(h, hipStreamSynchronize(stream));
  int err = 0;
  HIPCHK(h, hipMemcpy(&err, ws, sizeof(int), hipMemcpyDeviceToHost));
  int zero = 0;
  HIPCHK(h, hipMemcpy(ws, &zero, sizeof(int), hipMemcpyHostToDevice));
  // a vanishing pivot is reported first: the reciprocal taken after it is what
  // makes the later values non-finite
  if (err & ERR_SINGULAR) return fail(h, DMFT_ESINGULAR, "device flagged a vanishing pivot");
  if (err & ERR_NONFINITE) return fail(h, DMFT_ENONFINITE, "device flagged a non-finite value");
  if (err & ERR_NOCONV) return fail(h, DMFT_ENOCONV, "an eigensolver did not converge");
  return DMFT_OK;
}

int find_mu(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, int tail_order, double n_target,
            double tol_n, int method, double mu_lo, double mu_hi, double mu0, int max_iter, double* mu_out,
            int* passes_out, double* n_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (tail_order != 0 && tail_order != 2) return fail(h, DMFT_EINVAL, "tail_order must be 0 or 2");
  if (method != DMFT_NEWTON && method != DMFT_BISECT) return fail(h, DMFT_EINVAL, "unknown method");
  if (!(mu_lo < mu_hi) || !std::isfinite(mu_lo) || !std::isfinite(mu_hi))
    return fail(h, DMFT_EINVAL, "need finite mu_lo < mu_hi");
  if (!(tol_n > 0) || max_iter < 1) return fail(h, DMFT_EINVAL, "need tol_n > 0 and max_iter >= 1");
  Layout L;
  int r = prepare(h, lat, sig, ws, ws_bytes, L, KIND_TRACE, stream);
  if (r) return r;
  char* w = (char*)ws;
  double* dout = (double*)(w + L.out2);
  int passes = 0;
  // pinned readback slot: the error word and N, dN/dmu come back in one copy
  if (!h->readback) HIPCHK(h, hipHostMalloc(&h->readback, 64, hipHostMallocDefault));
  char* rb = (char*)h->readback;
  auto eval = [&](double mu, double* nv, double* dv) -> int {
    int rr = ntot_impl(h, lat, sig, L, w, mu, nullptr, tail_order, dout, stream);
    if (rr) return rr;
    HIPCHK(h, hipMemcpyAsync(rb, w + L.err, 16 + 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(h, hipStreamSynchronize(stream));
    ++passes;
    int err = 0;
    std::memcpy(&err, rb, sizeof(int));
    if (err) {
      int zero = 0;
      HIPCHK(h, hipMemcpy(w + L.err, &zero, sizeof(int), hipMemcpyHostToDevice));
      return fail(h, (err & ERR_SINGULAR) ? DMFT_ESINGULAR : DMFT_ENONFINITE, "device error at mu=%g", mu);
    }
    double nd[2];
    std::memcpy(nd, rb + 16, sizeof nd);
    *nv = nd[0];
    if (dv) *dv = nd[1];
    return DMFT_OK;
  };
  double lo = mu_lo, hi = mu_hi, mu = 0.0, nv = 0.0, dv = 0.0;
  int converged = 0;
  // N(mu) increases with mu.  When [lo, hi] does not contain the target, the
  // iterates run into one end of the bracket until no double lies strictly
  // between lo and hi; the search stops there instead of spending max_iter passes.
  auto collapsed = [&](double next) { return !(next > lo && next < hi); };
  auto no_bracket = [&]() {
    if (mu_out) *mu_out = mu;
    if (passes_out) *passes_out = passes;
    if (n_out) *n_out = nv;
    return fail(h, DMFT_ENOCONV, "[%.17g, %.17g] does not bracket n_target = %.17g (N = %.17g after %d passes)",
                mu_lo, mu_hi, n_target, nv, passes);
  };
  if (method == DMFT_BISECT) {
    for (int it = 0; it < max_iter; ++it) {
      mu = 0.5 * (lo + hi);
      if (it > 0 && collapsed(mu)) return no_bracket();
      r = eval(mu, &nv, nullptr);
      if (r) return r;
      if (std::fabs(nv - n_target) <= tol_n) { converged = 1; break; }
      if (nv < n_target) lo = mu; else hi = mu;
    }
  } else {
    // Newton inside the bracket (safeguarded as in Numerical Recipes' rtsafe):
    // take the Newton step when it stays strictly inside [lo, hi] and shrinks
    // the residual fast enough, otherwise bisect.
    mu = std::min(std::max(mu0, lo), hi);
    double prev_res = INFINITY, prev_dx = hi - lo;
    for (int it = 0; it < max_iter; ++it) {
      r = eval(mu, &nv, &dv);
      if (r) return r;
      double res = nv - n_target;
      if (std::fabs(res) <= tol_n) { converged = 1; break; }
      if (res < 0) lo = mu; else hi = mu;
      double next;
      bool newton_ok = dv > 0 && std::isfinite(dv);
      if (newton_ok) {
        next = mu - res / dv;
        if (!(next > lo && next < hi)) newton_ok = false;
        if (std::fabs(res) > 0.5 * prev_res && std::fabs(next - mu) > 0.5 * prev_dx) newton_ok = false;
      }
      if (!newton_ok) {
        next = 0.5 * (lo + hi);
        if (collapsed(next)) return no_bracket();
      }
      prev_dx = std::fabs(next - mu);
      prev_res = std::fabs(res);
      mu = next;
    }
  }
  if (mu_out) *mu_out = mu;
  if (passes_out) *passes_out = passes;
  if (n_out) *n_out = nv;
  if (!converged) return fail(h, DMFT_ENOCONV, "no convergence after %d passes (N=%g)", passes, nv);
  return DMFT_OK;
}











// Autotuner: for each kind (density pass, trace pass) time every instantiated
// kernel variant of the shape's largest padded size on a few frequency-tile
// sizes, after checking that each candidate reproduces the default candidate
// (G_loc and the scalars, or N and dN/dmu, to 1e-11 relative); keep the fastest.
int dmft_autotune(dmft_handle h, const dmft_lattice* lat, const dmft_sigma* sig, double mu, void* ws,
                  size_t ws_bytes, hipStream_t stream, char* best_out, size_t best_len) {
  int r = check_shapes(h, lat, sig);
  if (r) return r;
  if (!std::isfinite(mu)) return fail(h, DMFT_EINVAL, "mu is not finite");
  HIPCHK(h, hipSetDevice(h->device));
  char* w = (char*)ws;
  std::string report;
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  for (int kind : {KIND_DENSITY, KIND_TRACE, KIND_ADJOINT}) {
    Layout L0;
    r = make_layout(h, lat, sig, L0, kind);
    if (r) return r;
    r = check_ws(h, L0, ws, ws_bytes);
    if (r) return r;
    int nbp = L0.nbp_max, nk = lat->nk, nw = sig->nw, nc = lat->nc;
    int vars[16];
    int nv = dyson_variants(nbp, kind, vars, 16);
    Tile base = heuristic_tile(nk, nw);
    std::vector<Tile> tiles;
    // frequency tiles around the default, then the k-tile halved and doubled
    // with the frequency tile scaled the other way (the same number of items;
    // fewer G_loc partial read-backs against fewer partials of the running sum)
    for (int f : {1, 2, 4, 8}) {
      Tile t = base;
      t.wt = std::max(4, std::min(nw, base.wt * f / 2));
      bool dup = false;
      for (auto& u : tiles) dup |= (u.wt == t.wt && u.kt == t.kt);
      if (!dup) tiles.push_back(t);
    }
    for (int g : {-1, 1}) {
      Tile t = base;
      t.kt = g < 0 ? base.kt / 2 : std::min(nk, base.kt * 2);
      t.wt = g < 0 ? std::min(nw, base.wt * 2) : std::max(4, base.wt / 2);
      if (t.kt < 1 || t.kt == base.kt) continue;
      bool dup = false;
      for (auto& u : tiles) dup |= (u.wt == t.wt && u.kt == t.kt);
      if (!dup) tiles.push_back(t);
    }
    size_t nres = kind == KIND_DENSITY ? (size_t)nw * nc * nc * 2 + 3
                  : kind == KIND_ADJOINT ? (size_t)nw * nc * nc * 2 + 2 : 2;
    std::vector<double> ref(nres), got(nres);
    bool have_ref = false;
    double best_ms = 1e300;
    Tile best_tile = base;
    int best_var = vars[0];
    char key[32];
    snprintf(key, sizeof key, "%d/%d", kind, nbp);
    for (int vi = 0; vi < nv; ++vi) {
      if (vars[vi] == kLowrankP3Variant && !lowrank_p3_fits(nbp, nc)) continue;
      h->tvar[key] = vars[vi];
      for (const Tile& t : tiles) {
        Layout L;
        r = make_layout(h, lat, sig, L, kind, &t);
        if (r) return r;
        if (check_ws(h, L, ws, ws_bytes)) continue;
        r = upload_meta(h, L, w, stream, true);
        if (r) return r;
        double* out = (double*)(w + (have_ref ? L.tune_b : L.tune_a));
        auto run = [&]() -> int {
          if (kind == KIND_DENSITY)
            return density_impl(h, lat, sig, L, w, mu, nullptr, 2, nullptr, out, out + (size_t)nw * nc * nc * 2,
                                stream);
          if (kind == KIND_ADJOINT) return ntot_vjp_impl(h, lat, sig, L, w, mu, 2, out + 2, out, stream);
          return ntot_impl(h, lat, sig, L, w, mu, nullptr, 2, out, stream);
        };
        r = run();
        if (r) return r;
        float ms = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
          HIPCHK(h, hipEventRecord(e0, stream));
          r = run();
          if (r) return r;
          HIPCHK(h, hipEventRecord(e1, stream));
          HIPCHK(h, hipEventSynchronize(e1));
          float m = 0.f;
          HIPCHK(h, hipEventElapsedTime(&m, e0, e1));
          ms = std::min(ms, m);
        }
        HIPCHK(h, hipMemcpy(have_ref ? got.data() : ref.data(), out, nres * sizeof(double), hipMemcpyDeviceToHost));
        bool ok = true;
        if (have_ref) {
          double dn = 0.0, rn = 0.0;
          for (size_t i = 0; i < nres; ++i) {
            dn = std::max(dn, std::fabs(got[i] - ref[i]));
            rn = std::max(rn, std::fabs(ref[i]));
          }
          ok = std::isfinite(dn) && dn <= 1e-11 * std::max(rn, 1e-300);
        }
        have_ref = true;
        char line[160];
        snprintf(line, sizeof line, "%s nbp=%d var=%d kt=%d wt=%d: %.3f ms%s\n", kind_name(kind), nbp, vars[vi], t.kt,
                 t.wt, ms, ok ? "" : " (rejected)");
        report += line;
        if (ok && ms < best_ms) {
          best_ms = ms;
          best_tile = t;
          best_var = vars[vi];
        }
      }
    }
    h->tvar[key] = best_var;
    h->tune[tile_key(kind, nbp, nk, nw)] = best_tile;
    char line[160];
    snprintf(line, sizeof line, "best %s: var=%d kt=%d wt=%d %.3f ms\n", kind_name(kind), best_var, best_tile.kt,
             best_tile.wt, best_ms);
    report += line;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_out && best_len) {
    strncpy(best_out, report.c_str(), best_len - 1);
    best_out[best_len - 1] = 0;
  }
  return DMFT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batched pass

namespace {

// Layouts of all iterates inside one workspace, plus the argument array, the
// work queue, the queue counters and per-iterate mu slots.
int batched_layout(dmft_handle h, int n_iter, const dmft_lattice* const* lat, const dmft_sigma* const* sig,
                   std::vector<Layout>& Ls, std::vector<size_t>& base, const std::vector<Tile>* tiles,
                   size_t* total, size_t* o_args, size_t* o_items, size_t* o_cnt, size_t* o_mu, int* n_args,
                   int* n_items) {
  if (n_iter < 1 || !lat || !sig) return fail(h, DMFT_EINVAL, "need n_iter >= 1 and lattice/sigma arrays");
  Ls.assign(n_iter, Layout());
  base.assign(n_iter, 0);
  size_t o = 0;
  int na = 0, ni = 0;
  for (int s = 0; s < n_iter; ++s) {
    int r = check_shapes(h, lat[s], sig[s]);
    if (r) return r;
    Tile t;
    if (tiles) {
      t = (*tiles)[s];
    } else {
      // few, large frequency tiles: the queue is drained dynamically, and the
      // partial sums over frequency tiles stay a few GiB even for big batches
      t = heuristic_tile(lat[s]->nk, sig[s]->nw);
      t.wt = std::max(t.wt, (sig[s]->nw + 7) / 8);
    }
    r = make_layout(h, lat[s], sig[s], Ls[s], KIND_DENSITY, &t);
    if (r) return r;
    base[s] = o;
    o = align_up(o + Ls[s].total);
    for (const Bucket& b : Ls[s].buckets) {
      ++na;
      ni += b.n_ktiles * Ls[s].n_wtiles;
    }
  }
  *o_args = o;
  o = align_up(o + sizeof(DysonArgs) * na);
  *o_items = o;
  o = align_up(o + sizeof(BatchItemHost) * ni);
  *o_cnt = o;
  o = align_up(o + kMaxQueues * sizeof(int));
  *o_mu = o;
  o = align_up(o + sizeof(double) * n_iter);
  *total = o;
  *n_args = na;
  *n_items = ni;
  return DMFT_OK;
}

// Side streams and fork/join events of the concurrent class launches.
int batched_streams(dmft_handle h, int nside) {
  while ((int)h->b_side.size() < nside) {
    hipStream_t st = nullptr;
    HIPCHK(h, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    h->b_side.push_back(st);
    hipEvent_t e = nullptr;
    HIPCHK(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->b_join.push_back(e);
  }
  if (!h->b_fork) HIPCHK(h, hipEventCreateWithFlags(&h->b_fork, hipEventDisableTiming));
  return DMFT_OK;
}

// Timing events of the current plan (one pair per class and one for the span).
int batched_events(dmft_handle h) {
  if (!h->b_tspan.first) {
    HIPCHK(h, hipEventCreate(&h->b_tspan.first));
    HIPCHK(h, hipEventCreate(&h->b_tspan.second));
  }
  while (h->b_tcls.size() < h->b_cls.size()) {
    std::pair<hipEvent_t, hipEvent_t> ev;
    HIPCHK(h, hipEventCreate(&ev.first));
    HIPCHK(h, hipEventCreate(&ev.second));
    h->b_tcls.push_back(ev);
  }
  if (h->b_cls_ms.size() < h->b_cls.size()) h->b_cls_ms.resize(h->b_cls.size(), 0.0);
  return DMFT_OK;
}

// Reads the timing events of the last timed batched pass (waits for it) and
// adds them to the handle's kernel time: the span counts as one launch.
int batched_harvest(dmft_handle h) {
  if (!h->b_tpending) return DMFT_OK;
  h->b_tpending = false;
  HIPCHK(h, hipEventSynchronize(h->b_tspan.second));
  float ms = 0.f;
  HIPCHK(h, hipEventElapsedTime(&ms, h->b_tspan.first, h->b_tspan.second));
  h->t_ms += ms;
  h->t_count += 1;
  if (h->b_tcls_pending) {
    h->b_tcls_pending = false;
    for (size_t c = 0; c < h->b_cls.size() && c < h->b_tcls.size(); ++c) {
      HIPCHK(h, hipEventElapsedTime(&ms, h->b_tcls[c].first, h->b_tcls[c].second));
      h->b_cls_ms[c] += ms;
    }
  }
  return DMFT_OK;
}

int batched_pass_impl(dmft_handle h, const double* mu_dev, double* const* nk_out, double* const* gloc_out,
                      void* ws, size_t ws_bytes, hipStream_t stream, bool kernel_only) {
  if (h->iters.empty()) return fail(h, DMFT_EINVAL, "no batched plan (call dmft_batched_plan first)");
  if (ws != h->b_ws || ws_bytes < h->b_total) return fail(h, DMFT_EWORKSPACE, "workspace differs from the plan's");
  if (!mu_dev) return fail(h, DMFT_EINVAL, "mu_dev is NULL");
  char* w = (char*)ws;
  int n_iter = (int)h->iters.size();
  const bool timed = h->timing && !kernel_only && !h->b_capturing;
  if (timed) {
    int r = batched_harvest(h);  // the previous pass's events are re-recorded below
    if (r) return r;
    r = batched_events(h);
    if (r) return r;
  }
  HIPCHK(h, launch_copy_doubles(mu_dev, (double*)(w + h->b_mu), n_iter, stream));
  HIPCHK(h, launch_fill_zero(w + h->b_counters, kMaxQueues * sizeof(int), stream));
  if (timed) HIPCHK(h, hipEventRecord(h->b_tspan.first, stream));
  if (h->b_lowrank && !h->b_concurrent) {
    for (size_t c = 0; c < h->b_cls.size(); ++c) {
      const auto& k = h->b_cls[c];
      if (timed) HIPCHK(h, hipEventRecord(h->b_tcls[c].first, stream));
      HIPCHK(h, launch_lr_class(k.nbp, k.ncls, w + h->b_items + sizeof(BatchItemHost) * k.off, k.count,
                                (const DysonArgs*)(w + h->b_args), (int*)(w + h->b_counters) + c, k.grid, stream));
      if (timed) HIPCHK(h, hipEventRecord(h->b_tcls[c].second, stream));
    }
  } else if (h->b_lowrank) {
    const int nside = (int)h->b_side.size();
    HIPCHK(h, hipEventRecord(h->b_fork, stream));
    for (hipStream_t st : h->b_side) HIPCHK(h, hipStreamWaitEvent(st, h->b_fork, 0));
    for (size_t c = 0; c < h->b_cls.size(); ++c) {
      const auto& k = h->b_cls[c];
      hipStream_t st = h->b_side[c % nside];
      if (timed) HIPCHK(h, hipEventRecord(h->b_tcls[c].first, st));
      HIPCHK(h, launch_lr_class(k.nbp, k.ncls, w + h->b_items + sizeof(BatchItemHost) * k.off, k.count,
                                (const DysonArgs*)(w + h->b_args), (int*)(w + h->b_counters) + c, k.grid, st));
      if (timed) HIPCHK(h, hipEventRecord(h->b_tcls[c].second, st));
    }
    for (int i = 0; i < nside; ++i) {
      HIPCHK(h, hipEventRecord(h->b_join[i], h->b_side[i]));
      HIPCHK(h, hipStreamWaitEvent(stream, h->b_join[i], 0));
    }
  } else
    HIPCHK(h, launch_batched(w + h->b_items, h->b_nbig, h->b_nsmall, (const DysonArgs*)(w + h->b_args),
                             (int*)(w + h->b_counters), h->b_wgs, stream));
  if (timed) {
    HIPCHK(h, hipEventRecord(h->b_tspan.second, stream));
    h->b_tpending = true;
    h->b_tcls_pending = h->b_lowrank;
  }
  if (kernel_only) return DMFT_OK;
  for (int s = 0; s < n_iter; ++s) {
    const auto& it = h->iters[s];
    char* wb = w + it.base;
    const double* mup = (const double*)(w + h->b_mu) + s;
    EpilogueArgs e = epilogue_args(&it.lat, &it.sig, it.lay, wb, 0.0, mup, h->b_tail);
    if (nk_out && nk_out[s]) HIPCHK(h, launch_nk_epilogue(e, nk_out[s], stream));
    if (gloc_out && gloc_out[s])
      HIPCHK(h, launch_gloc_reduce(it.lay.n_ktiles_total, it.sig.nw, it.lat.nc, (const double*)(wb + it.lay.xpart),
                                   gloc_out[s], stream));
  }
  return DMFT_OK;
}

int batched_build(dmft_handle h, int n_iter, const dmft_lattice* const* lat, const dmft_sigma* const* sig,
                  int tail_order, void* ws, size_t ws_bytes, hipStream_t stream, const std::vector<Tile>* tiles,
                  bool lowrank) {
  std::vector<Layout> Ls;
  std::vector<size_t> base;
  size_t total, o_args, o_items, o_cnt, o_mu;
  int na, ni;
  int r = batched_layout(h, n_iter, lat, sig, Ls, base, tiles, &total, &o_args, &o_items, &o_cnt, &o_mu, &na, &ni);
  if (r) return r;
  if (!ws || (uintptr_t)ws % kAlign) return fail(h, DMFT_EWORKSPACE, "workspace NULL or misaligned");
  if (ws_bytes < total) return fail(h, DMFT_EWORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, total);
  HIPCHK(h, hipSetDevice(h->device));
  char* w = (char*)ws;
  h->iters.clear();
  h->iter_nb.assign(n_iter, {});
  std::vector<DysonArgs> args;
  struct Q {
    BatchItemHost it;
    double cost;
  };
  std::vector<Q> big, small;
  std::map<std::pair<int, int>, std::vector<Q>> lrq;  // low-rank queues by (nbp, column class)
  for (int s = 0; s < n_iter; ++s) {
    Layout& L = Ls[s];
    r = upload_meta(h, L, w + base[s], stream, true);
    if (r) return r;
    dmft_handle_s::Iter itr;
    itr.lat = *lat[s];
    if (lat[s]->nb) {
      h->iter_nb[s].assign(lat[s]->nb, lat[s]->nb + lat[s]->nk);
      itr.lat.nb = h->iter_nb[s].data();
    }
    itr.sig = *sig[s];
    itr.lay = L;
    itr.base = base[s];
    h->iters.push_back(itr);
    char* wb = w + base[s];
    const double* mup = (const double*)(w + o_mu) + s;
    size_t at = 0;
    for (const Bucket& b : L.buckets) {
      DysonArgs a{};
      a.nk = lat[s]->nk;
      a.nc = lat[s]->nc;
      a.nw = sig[s]->nw;
      a.nb_uniform = L.ragged ? 0 : lat[s]->nb_max;
      a.nb = (const int32_t*)(wb + L.meta_nb);
      a.off_b = (const int64_t*)(wb + L.meta_offb);
      a.eps = lat[s]->eps;
      a.wk = lat[s]->wk;
      a.proj = lat[s]->proj;
      a.beta = sig[s]->beta;
      a.sigma = sig[s]->sigma;
      a.e_dc = sig[s]->e_dc;
      a.mu_ptr = mup;
      a.klist = (const int32_t*)(wb + L.meta_klist) + at;
      a.nklist = (int)b.klist.size();
      a.kt = L.tile.kt;
      a.wt = L.tile.wt;
      a.n_wtiles = L.n_wtiles;
      a.ktile_base = b.ktile_base;
      a.mode = MODE_S | MODE_GLOC;
      a.spart = (double*)(wb + L.spart);
      a.s_stride = L.s_stride;
      a.off_s = (const int64_t*)(wb + L.meta_offs);
      a.xpart = (double*)(wb + L.xpart);
      a.tpart = (double*)(wb + L.tpart);
      a.err = (int*)(w + base[0] + Ls[0].err);
      int ai = (int)args.size();
      args.push_back(a);
      at += b.klist.size();
      const double nbp = b.nbp, nc = lat[s]->nc;
      for (int kt = 0; kt < b.n_ktiles; ++kt) {
        int nkt = std::min(L.tile.kt, (int)b.klist.size() - kt * L.tile.kt);
        for (int wt = 0; wt < L.n_wtiles; ++wt) {
          int nwt = std::min(L.tile.wt, sig[s]->nw - wt * L.tile.wt);
          if (lowrank) {
            // one queue per class (padded size, columns of the inversions)
            double c = (nbp * nbp * nc + 2.0 * nbp * nc * nc + 4.0 * nc * nc * nc) * nkt * nwt;
            lrq[{b.nbp, lr_nc_class(b.nbp, lat[s]->nc)}].push_back(Q{{ai, b.nbp, kt, wt}, c});
          } else {
            double c = nbp * nbp * (nbp + 2.0 * nc) * nkt * nwt;
            Q qq{{ai, b.nbp, kt, wt}, c};
            (b.nbp == 64 ? big : small).push_back(qq);
          }
        }
      }
    }
  }
  auto by_cost = [](const Q& x, const Q& y) { return x.cost > y.cost; };
  std::stable_sort(big.begin(), big.end(), by_cost);
  std::stable_sort(small.begin(), small.end(), by_cost);
  std::vector<BatchItemHost> items;
  for (auto& x : big) items.push_back(x.it);
  for (auto& x : small) items.push_back(x.it);
  int ncu = 0;
  HIPCHK(h, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device));
  ncu = std::max(ncu, 1);
  h->b_cls.clear();
  if (lowrank) {
    // largest padded size first, so that the longest items start earliest
    for (auto it = lrq.rbegin(); it != lrq.rend(); ++it) {
      auto& qv = it->second;
      std::stable_sort(qv.begin(), qv.end(), by_cost);
      dmft_handle_s::LRClassPlan c;
      c.nbp = it->first.first;
      c.ncls = it->first.second;
      c.off = (int)items.size();
      c.count = (int)qv.size();
      // one wavefront per SIMD: four single-wavefront, two pair or one four-wavefront
      // work-group per CU
      c.grid = std::min(c.count, lr_class_wgs_per_cu(c.nbp, c.ncls) * ncu);
      for (auto& x : qv) items.push_back(x.it);
      h->b_cls.push_back(c);
    }
    if ((int)h->b_cls.size() > kMaxQueues) return fail(h, DMFT_EUNSUPPORTED, "too many item classes");
    int rs = batched_streams(h, std::min<int>(3, (int)h->b_cls.size()));
    if (rs) return rs;
    h->b_cls_ms.assign(h->b_cls.size(), 0.0);
  }
  HIPCHK(h, hipMemcpy(w + o_args, args.data(), sizeof(DysonArgs) * args.size(), hipMemcpyHostToDevice));
  if (!items.empty())
    HIPCHK(h, hipMemcpy(w + o_items, items.data(), sizeof(BatchItemHost) * items.size(), hipMemcpyHostToDevice));
  int zero = 0;
  HIPCHK(h, hipMemcpy(w + base[0] + Ls[0].err, &zero, sizeof(int), hipMemcpyHostToDevice));
  h->b_tail = tail_order;
  h->b_total = total;
  h->b_args = o_args;
  h->b_items = o_items;
  h->b_counters = o_cnt;
  h->b_mu = o_mu;
  h->b_nbig = (int)big.size();
  h->b_nsmall = (int)small.size();
  h->b_nargs = (int)args.size();
  h->b_lowrank = lowrank;
  // dense: two-wavefront work-groups, one per SIMD pair (the low-rank classes
  // size their own grids above)
  h->b_wgs = 2 * ncu;
  h->b_ws = ws;
  return DMFT_OK;
}

}  // namespace

extern "C" {

// Tiles the batched plan times: the default tile of every iterate and the same
// with the k-tile halved and quartered (more, smaller items balance the class
// kernels' last round better, at the price of more G_loc partials), then the
// frequency tile halved, and the k-tile quartered with the frequency tile
// rounded down to whole groups of 48 frequencies.
std::vector<std::vector<Tile>> batched_tile_candidates(const std::vector<Tile>& base) {
  std::vector<std::vector<Tile>> out;
  for (int f : {1, 2, 4}) {
    std::vector<Tile> c = base;
    bool changed = f == 1;
    for (auto& t : c) {
      const int kt = std::max(1, t.kt / f);
      changed |= kt != t.kt;
      t.kt = kt;
    }
    if (changed) out.push_back(c);
  }
  std::vector<Tile> c = base;
  bool changed = false;
  for (auto& t : c) {
    const int wt = std::max(4, t.wt / 2);
    changed |= wt != t.wt;
    t.wt = wt;
  }
  if (changed) out.push_back(c);
  // the quarter k-tile with the frequency tile rounded down to a multiple of 48
  // (whole groups of the four-wavefront packed kernel, and of the 12, 8 and 4
  // frequencies of the others)
  c = base;
  changed = false;
  for (auto& t : c) {
    const int kt = std::max(1, t.kt / 4), wt = t.wt >= 96 ? t.wt / 48 * 48 : t.wt;
    changed |= kt != t.kt && wt != t.wt;
    t.kt = kt;
    t.wt = wt;
  }
  if (changed) out.push_back(c);
  return out;
}

int dmft_batched_workspace_size(dmft_handle h, int n_iter, const dmft_lattice* const* lat, const dmft_sigma* const* sig,
                                size_t* bytes) {
  if (!bytes) return fail(h, DMFT_EINVAL, "bytes is NULL");
  std::vector<Layout> Ls;
  std::vector<size_t> base;
  size_t total, a, b, c, d;
  int na, ni;
  int r = batched_layout(h, n_iter, lat, sig, Ls, base, nullptr, &total, &a, &b, &c, &d, &na, &ni);
  if (r) return r;
  // room for every tile the plan times
  std::vector<Tile> tiles;
  for (auto& L : Ls) tiles.push_back(L.tile);
  size_t most = total;
  for (const auto& cand : batched_tile_candidates(tiles)) {
    r = batched_layout(h, n_iter, lat, sig, Ls, base, &cand, &total, &a, &b, &c, &d, &na, &ni);
    if (r) return r;
    most = std::max(most, total);
  }
  *bytes = most;
  return DMFT_OK;
}

int dmft_batched_plan(dmft_handle h, int n_iter, const dmft_lattice* const* lat, const dmft_sigma* const* sig,
                      int tail_order, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!h) return DMFT_EINVAL;
  if (tail_order != 0 && tail_order != 2) return fail(h, DMFT_EINVAL, "tail_order must be 0 or 2");
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  if (h->graph) {
    (void)hipGraphDestroy(h->graph);
    h->graph = nullptr;
  }
  h->b_tile_chosen = -1;
  int r = batched_build(h, n_iter, lat, sig, tail_order, ws, ws_bytes, stream, nullptr, false);
  if (r) return r;
  // Autotune the form of the step (dense inversion or low-rank) and the k- and
  // frequency-tile sizes of the persistent launches: time the kernels for each
  // candidate that fits the workspace, keep the fastest plan.
  std::vector<Tile> base_tiles;
  for (auto& it : h->iters) base_tiles.push_back(it.lay.tile);
  std::vector<double> mu0(n_iter, 0.0);
  char* w = (char*)ws;
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  double best = 1e300, best_lowrank = 1e300;
  std::vector<Tile> best_tiles = base_tiles;
  bool best_lr = true;
  // low-rank form first; the dense form's other tiles are timed only when its
  // first one comes within 1.5x of the best low-rank plan
  const std::vector<std::vector<Tile>> cands = batched_tile_candidates(base_tiles);
  int best_ci = -1;
  for (bool lr : {true, false}) {
    if (h->b_form_pref != DMFT_FORM_AUTO && lr != (h->b_form_pref == DMFT_FORM_LOWRANK)) continue;
    double first = -1.0;
    for (int ci = 0; ci < (int)cands.size(); ++ci) {
      const std::vector<Tile>& cand = cands[ci];
      if (h->b_tile_pref >= 0 && ci != h->b_tile_pref && h->b_tile_pref < (int)cands.size()) continue;
      if (!lr && first > 1.5 * best_lowrank) break;
      std::vector<Layout> Ls;
      std::vector<size_t> bs;
      size_t total, a, b, c, d;
      int na, ni;
      r = batched_layout(h, n_iter, lat, sig, Ls, bs, &cand, &total, &a, &b, &c, &d, &na, &ni);
      if (r) return r;
      if (total > ws_bytes) continue;
      r = batched_build(h, n_iter, lat, sig, tail_order, ws, ws_bytes, stream, &cand, lr);
      if (r) return r;
      HIPCHK(h, hipMemcpy(w + h->b_mu, mu0.data(), sizeof(double) * n_iter, hipMemcpyHostToDevice));
      // low-rank candidates run twice and keep the faster pass (their times
      // differ by a few percent, about the spread of one pass)
      float ms = 1e30f;
      for (int rep = 0; rep < (lr ? 2 : 1); ++rep) {
        HIPCHK(h, hipEventRecord(e0, stream));
        r = batched_pass_impl(h, (const double*)(w + h->b_mu), nullptr, nullptr, ws, ws_bytes, stream, true);
        if (r) return r;
        HIPCHK(h, hipEventRecord(e1, stream));
        HIPCHK(h, hipEventSynchronize(e1));
        float t = 0.f;
        HIPCHK(h, hipEventElapsedTime(&t, e0, e1));
        ms = std::min(ms, t);
      }
      if (first < 0) first = ms;
      if (lr) best_lowrank = std::min(best_lowrank, (double)ms);
      if (ms < best) {
        best = ms;
        best_tiles = cand;
        best_lr = lr;
        best_ci = ci;
      }
    }
  }
  r = batched_build(h, n_iter, lat, sig, tail_order, ws, ws_bytes, stream, &best_tiles, best_lr);
  h->b_tile_chosen = r ? -1 : best_ci;
  if (r) return r;
  // class kernels concurrently on side streams or one after another: the
  // overlap fills each class's tail but makes the classes share the CUs, so
  // time both and keep the faster (the later of two timings of each, the first
  // pass after a rebuild warming the caches)
  h->b_concurrent = h->b_conc_pref != 0;
  if (best_lr && h->b_cls.size() > 1) {
    // launch orders: by cost (as built), or the widest work-groups first, so
    // that a class whose work-group takes a whole CU is not starved by the
    // narrower ones filling every CU partly; with the concurrency fixed by
    // the caller only the orders are timed
    std::vector<dmft_handle_s::LRClassPlan> orders[2];
    orders[0] = h->b_cls;
    orders[1] = h->b_cls;
    auto width = [](const dmft_handle_s::LRClassPlan& c) { return 64 * (4 / lr_class_wgs_per_cu(c.nbp, c.ncls)); };
    std::stable_sort(orders[1].begin(), orders[1].end(),
                     [&](const auto& x, const auto& y) { return width(x) > width(y); });
    HIPCHK(h, hipMemcpy(w + h->b_mu, mu0.data(), sizeof(double) * n_iter, hipMemcpyHostToDevice));
    double t[2][2] = {{1e300, 1e300}, {1e300, 1e300}};
    for (int rep = 0; rep < 2; ++rep)
      for (int o = 0; o < 2; ++o)
        for (int conc = 0; conc < 2; ++conc) {
          if (h->b_conc_pref >= 0 && conc != h->b_conc_pref) continue;
          h->b_cls = orders[o];
          h->b_concurrent = conc != 0;
          HIPCHK(h, hipEventRecord(e0, stream));
          r = batched_pass_impl(h, (const double*)(w + h->b_mu), nullptr, nullptr, ws, ws_bytes, stream, true);
          if (r) return r;
          HIPCHK(h, hipEventRecord(e1, stream));
          HIPCHK(h, hipEventSynchronize(e1));
          float ms = 0.f;
          HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
          t[o][conc] = ms;  // the second repetition's time is kept
        }
    int bo = 0, bc = h->b_conc_pref >= 0 ? h->b_conc_pref : 1;
    for (int o = 0; o < 2; ++o)
      for (int conc = 0; conc < 2; ++conc)
        if (t[o][conc] < t[bo][bc]) {
          bo = o;
          bc = conc;
        }
    h->b_cls = orders[bo];
    h->b_concurrent = bc != 0;
    // the timing passes may have flagged the error word (mu = 0 need not suit
    // the inputs): the plan starts clean, as batched_build leaves it
    int zero = 0;
    HIPCHK(h, hipMemcpy(w + h->iters[0].base + h->iters[0].lay.err, &zero, sizeof(int), hipMemcpyHostToDevice));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return DMFT_OK;
}

int dmft_batched_pass(dmft_handle h, const double* mu_dev, double* const* nk_out, double* const* gloc_out, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
  if (!h) return DMFT_EINVAL;
  return batched_pass_impl(h, mu_dev, nk_out, gloc_out, ws, ws_bytes, stream, false);
}

int dmft_batched_graph_capture(dmft_handle h, const double* mu_dev, double* const* nk_out, double* const* gloc_out,
                               void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!h) return DMFT_EINVAL;
  if (h->iters.empty()) return fail(h, DMFT_EINVAL, "no batched plan (call dmft_batched_plan first)");
  if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  if (h->graph) {
    (void)hipGraphDestroy(h->graph);
    h->graph = nullptr;
  }
  HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  h->b_capturing = true;  // no timing events inside the graph
  int r = batched_pass_impl(h, mu_dev, nk_out, gloc_out, ws, ws_bytes, h->cap_stream, false);
  h->b_capturing = false;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (r) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (e != hipSuccess) return fail(h, DMFT_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  h->graph = g;
  HIPCHK(h, hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
  return dmft_batched_graph_launch(h, stream);
}

int dmft_batched_set_form(dmft_handle h, int form) {
  if (!h) return DMFT_EINVAL;
  if (form != DMFT_FORM_AUTO && form != DMFT_FORM_DENSE && form != DMFT_FORM_LOWRANK)
    return fail(h, DMFT_EINVAL, "unknown batched form %d", form);
  h->b_form_pref = form;
  return DMFT_OK;
}

int dmft_batched_classes(dmft_handle h, int max, int32_t* nbp, int32_t* ncls, int32_t* items, double* kernel_ms) {
  if (!h) return DMFT_EINVAL;
  if (h->iters.empty() || !h->b_lowrank) return 0;
  int rb = batched_harvest(h);
  if (rb) return rb;
  const int n = (int)h->b_cls.size();
  for (int c = 0; c < n && c < max; ++c) {
    if (nbp) nbp[c] = h->b_cls[c].nbp;
    if (ncls) ncls[c] = h->b_cls[c].ncls;
    if (items) items[c] = h->b_cls[c].count;
    if (kernel_ms) kernel_ms[c] = c < (int)h->b_cls_ms.size() ? h->b_cls_ms[c] : 0.0;
  }
  return n;
}

int dmft_batched_set_concurrent(dmft_handle h, int mode) {
  if (!h) return DMFT_EINVAL;
  if (mode < -1 || mode > 1) return fail(h, DMFT_EINVAL, "unknown concurrency mode %d", mode);
  h->b_conc_pref = mode;
  return DMFT_OK;
}

int dmft_batched_concurrent(dmft_handle h) {
  if (!h || h->iters.empty() || !h->b_lowrank) return -1;
  return h->b_concurrent ? 1 : 0;
}

int dmft_batched_set_tile_candidate(dmft_handle h, int index) {
  if (!h) return DMFT_EINVAL;
  if (index < -1) return fail(h, DMFT_EINVAL, "tile candidate %d", index);
  h->b_tile_pref = index;
  return DMFT_OK;
}

int dmft_batched_tile_candidate(dmft_handle h) {
  if (!h || h->iters.empty()) return -1;
  return h->b_tile_chosen;
}

int dmft_batched_form(dmft_handle h) {
  if (!h || h->iters.empty()) return -1;
  return h->b_lowrank ? DMFT_FORM_LOWRANK : DMFT_FORM_DENSE;
}

int dmft_batched_graph_launch(dmft_handle h, hipStream_t stream) {
  if (!h) return DMFT_EINVAL;
  if (!h->gexec) return fail(h, DMFT_EINVAL, "no captured graph");
  if (h->timing) {
    int r = batched_harvest(h);  // the previous pass's or replay's events
    if (r) return r;
    r = batched_events(h);
    if (r) return r;
    HIPCHK(h, hipEventRecord(h->b_tspan.first, stream));
  }
  HIPCHK(h, hipGraphLaunch(h->gexec, stream));
  if (h->timing) {
    HIPCHK(h, hipEventRecord(h->b_tspan.second, stream));
    h->b_tpending = true;
  }
  return DMFT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Pole-expansion route (Sec. 3.3 eqs. pseudo_H_k, rho_LDA+DMFT_componet_final,
// fix_mu; Sec. 3.5.2 eqs. DOS, PDOS).

namespace {

struct PoleLayout {
  size_t err = 0, res = 0, meta_nb = 0, meta_offb = 0, meta_offn = 0, kscal = 0, sweeps = 0, part = 0, epart = 0;
  size_t total = 0;
  int mp = 0;
  bool ragged = false;
};

int check_poles(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol) {
  int r = check_lattice(h, lat);
  if (r) return r;
  if (!pol) return fail(h, DMFT_EINVAL, "poles is NULL");
  if (pol->np < 0) return fail(h, DMFT_EINVAL, "np must be >= 0 (got %d)", pol->np);
  if (pol->np > 0 && (!pol->p || !pol->v)) return fail(h, DMFT_EINVAL, "p and v must be set when np > 0");
  if (!pol->e_dc) return fail(h, DMFT_EINVAL, "e_dc must be set");
  if (!(pol->beta > 0) || !std::isfinite(pol->beta)) return fail(h, DMFT_EINVAL, "beta must be positive and finite");
  if (lat->nb_max + pol->np > 80)
    return fail(h, DMFT_EUNSUPPORTED, "nb_max + np = %d exceeds 80", lat->nb_max + pol->np);
  return DMFT_OK;
}

void pole_layout(const dmft_lattice* lat, const dmft_poles* pol, int ne, PoleLayout& P) {
  const int nk = lat->nk;
  P.mp = lat->nb_max + pol->np;
  P.ragged = lat->nb != nullptr;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  P.err = take(16);
  P.res = take(8 * sizeof(double));
  P.meta_nb = take(sizeof(int32_t) * nk);
  P.meta_offb = take(sizeof(int64_t) * (nk + 1));
  P.meta_offn = take(sizeof(int64_t) * (nk + 1));
  P.kscal = take(sizeof(double) * 3 * nk);
  P.sweeps = take(sizeof(int32_t) * nk);
  P.part = take(sizeof(double) * (size_t)pole_dos_kslices(nk, P.mp) * std::max(ne, 1) * (1 + lat->nc));
  P.epart = take(sizeof(double) * (size_t)pole_energy_parts(nk, P.mp) * (3 + lat->nc));
  P.total = o;
}

int pole_prepare(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, int ne, void* ws, size_t ws_bytes,
                 PoleLayout& P, hipStream_t s) {
  int r = check_poles(h, lat, pol);
  if (r) return r;
  pole_layout(lat, pol, ne, P);
  if (!ws) return fail(h, DMFT_EWORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % kAlign) return fail(h, DMFT_EWORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < P.total) return fail(h, DMFT_EWORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, P.total);
  HIPCHK(h, hipSetDevice(h->device));
  if (!P.ragged) return DMFT_OK;  // uniform windows need no per-k metadata
  const size_t nk = lat->nk;
  const size_t need = sizeof(int32_t) * nk + sizeof(int64_t) * (nk + 1) * 2;
  if (h->staged) HIPCHK(h, hipEventSynchronize(h->staged));
  if (need > h->pinned_bytes) {
    if (h->pinned) HIPCHK(h, hipHostFree(h->pinned));
    h->pinned = nullptr;
    HIPCHK(h, hipHostMalloc(&h->pinned, need, hipHostMallocDefault));
    h->pinned_bytes = need;
  }
  int32_t* nbv = (int32_t*)h->pinned;
  int64_t* offb = (int64_t*)(nbv + nk);
  int64_t* offn = offb + nk + 1;
  offb[0] = offn[0] = 0;
  for (size_t k = 0; k < nk; ++k) {
    nbv[k] = lat->nb[k];
    offb[k + 1] = offb[k] + lat->nb[k];
    offn[k + 1] = offn[k] + (int64_t)lat->nb[k] * lat->nb[k];
  }
  char* w = (char*)ws;
  HIPCHK(h, hipMemcpyAsync(w + P.meta_nb, nbv, sizeof(int32_t) * nk, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(w + P.meta_offb, offb, sizeof(int64_t) * (nk + 1), hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(w + P.meta_offn, offn, sizeof(int64_t) * (nk + 1), hipMemcpyHostToDevice, s));
  if (!h->staged) HIPCHK(h, hipEventCreateWithFlags(&h->staged, hipEventDisableTiming));
  HIPCHK(h, hipEventRecord(h->staged, s));
  return DMFT_OK;
}

PoleArgs pole_args(const dmft_lattice* lat, const dmft_poles* pol, const PoleLayout& P, char* w) {
  PoleArgs a{};
  a.nk = lat->nk;
  a.nc = lat->nc;
  a.np = pol->np;
  a.mp = P.mp;
  a.nb_max = lat->nb_max;
  a.nb_uniform = P.ragged ? 0 : lat->nb_max;
  a.nb = (const int32_t*)(w + P.meta_nb);
  a.off_b = (const int64_t*)(w + P.meta_offb);
  a.off_n = (const int64_t*)(w + P.meta_offn);
  a.eps = lat->eps;
  a.wk = lat->wk;
  a.proj = lat->proj;
  a.p = pol->p;
  a.v = pol->v;
  a.sigma_inf = pol->sigma_inf;
  a.e_dc = pol->e_dc;
  a.beta = pol->beta;
  a.sweeps = (int*)(w + P.sweeps);
  a.err = (int*)(w + P.err);
  a.max_sweeps = 30;
  return a;
}

}  // namespace

extern "C" {

int dmft_pole_workspace_size(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, int ne_max,
                             size_t* bytes) {
  if (!bytes) return fail(h, DMFT_EINVAL, "bytes is NULL");
  int r = check_poles(h, lat, pol);
  if (r) return r;
  if (ne_max < 0) return fail(h, DMFT_EINVAL, "ne_max must be >= 0");
  PoleLayout P;
  pole_layout(lat, pol, ne_max, P);
  *bytes = P.total;
  return DMFT_OK;
}

int dmft_pole_eig(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, double* evals, double* evecs,
                  double* wphys, double* worb, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!evals || !evecs || !wphys) return fail(h, DMFT_EINVAL, "evals, evecs and wphys are required");
  PoleLayout P;
  int r = pole_prepare(h, lat, pol, 0, ws, ws_bytes, P, stream);
  if (r) return r;
  const size_t lds = pole_eig_lds_bytes(lat->nb_max, pol->np);
  int lim = 0, optin = 0;
  HIPCHK(h, hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, h->device) != hipSuccess) optin = 0;
  lim = std::max(lim, optin);
  // dynamic LDS plus the kernel's static arrays (at most 10 KB with 1024 threads)
  if (lds + 12288 > (size_t)lim)
    return fail(h, DMFT_EUNSUPPORTED, "eigensolver needs %zu B of LDS, the device allows %d", lds + 12288, lim);
  PoleArgs a = pole_args(lat, pol, P, (char*)ws);
  a.evals = evals;
  a.evecs = evecs;
  a.wphys = wphys;
  a.worb = worb;
  HIPCHK(h, launch_pole_eig(a, lds, stream));
  return DMFT_OK;
}

int dmft_pole_sweeps(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, const void* ws, int32_t* out,
                     hipStream_t stream) {
  if (!out || !ws) return fail(h, DMFT_EINVAL, "out and ws are required");
  int r = check_poles(h, lat, pol);
  if (r) return r;
  PoleLayout P;
  pole_layout(lat, pol, 0, P);
  HIPCHK(h, hipMemcpyAsync(out, (const char*)ws + P.sweeps, sizeof(int32_t) * lat->nk, hipMemcpyDeviceToHost,
                           stream));
  HIPCHK(h, hipStreamSynchronize(stream));
  return DMFT_OK;
}

int dmft_pole_density(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, double mu, int nw_trunc,
                      const double* evals, const double* evecs, double* nk, double* scalars, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
  if (!evals || !evecs) return fail(h, DMFT_EINVAL, "evals and evecs are required");
  if (!nk && !scalars) return fail(h, DMFT_EINVAL, "no output requested");
  if (nw_trunc < 0) return fail(h, DMFT_EINVAL, "nw_trunc must be >= 0");
  if (!std::isfinite(mu)) return fail(h, DMFT_EINVAL, "mu is not finite");
  PoleLayout P;
  int r = pole_prepare(h, lat, pol, 0, ws, ws_bytes, P, stream);
  if (r) return r;
  char* w = (char*)ws;
  PoleArgs a = pole_args(lat, pol, P, w);
  a.evals = const_cast<double*>(evals);
  a.evecs = const_cast<double*>(evecs);
  double* kscal = (double*)(w + P.kscal);
  HIPCHK(h, launch_pole_density(a, mu, nw_trunc, nk, kscal, stream));
  if (scalars) HIPCHK(h, launch_scalar_reduce_mask(lat->nk, lat->wk, kscal, 3, 0, scalars, stream));
  return DMFT_OK;
}

int dmft_pole_find_mu(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, const double* evals,
                      const double* wphys, double n_target, double tol_n, int method, double mu_lo, double mu_hi,
                      int max_iter, double* mu_out, int* passes_out, double* n_out, void* ws, size_t ws_bytes,
                      hipStream_t stream) {
  if (!evals || !wphys) return fail(h, DMFT_EINVAL, "evals and wphys are required");
  if (method != DMFT_NEWTON && method != DMFT_BISECT) return fail(h, DMFT_EINVAL, "unknown method");
  if (!(mu_lo < mu_hi) || !std::isfinite(mu_lo) || !std::isfinite(mu_hi))
    return fail(h, DMFT_EINVAL, "need finite mu_lo < mu_hi");
  if (!(tol_n > 0) || max_iter < 1) return fail(h, DMFT_EINVAL, "need tol_n > 0 and max_iter >= 1");
  if (!std::isfinite(n_target)) return fail(h, DMFT_EINVAL, "n_target is not finite");
  PoleLayout P;
  int r = pole_prepare(h, lat, pol, 0, ws, ws_bytes, P, stream);
  if (r) return r;
  char* w = (char*)ws;
  PoleArgs a = pole_args(lat, pol, P, w);
  a.evals = const_cast<double*>(evals);
  a.wphys = const_cast<double*>(wphys);
  double* res = (double*)(w + P.res);
  HIPCHK(h, launch_pole_find_mu(a, n_target, tol_n, method, mu_lo, mu_hi, 0.5 * (mu_lo + mu_hi), max_iter, res,
                                stream));
  double host[4];
  HIPCHK(h, hipMemcpyAsync(host, res, sizeof host, hipMemcpyDeviceToHost, stream));
  HIPCHK(h, hipStreamSynchronize(stream));
  if (mu_out) *mu_out = host[0];
  if (n_out) *n_out = host[1];
  if (passes_out) *passes_out = (int)host[2];
  if (host[3] != 0.0)
    return fail(h, DMFT_ENOCONV, "no convergence after %d passes (N=%g)", (int)host[2], host[1]);
  return DMFT_OK;
}

int dmft_pole_dos(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, const double* evals,
                  const double* wphys, const double* worb, double mu, double eta, double e_min, double e_max, int ne,
                  double* dos, double* pdos, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!evals || !wphys || !dos) return fail(h, DMFT_EINVAL, "evals, wphys and dos are required");
  if (pdos && !worb) return fail(h, DMFT_EINVAL, "pdos needs worb");
  if (ne < 1) return fail(h, DMFT_EINVAL, "ne must be >= 1");
  if (!(eta > 0) || !std::isfinite(eta)) return fail(h, DMFT_EINVAL, "eta must be positive and finite");
  if (!std::isfinite(e_min) || !std::isfinite(e_max) || e_max < e_min || !std::isfinite(mu))
    return fail(h, DMFT_EINVAL, "need finite mu and e_min <= e_max");
  PoleLayout P;
  int r = pole_prepare(h, lat, pol, ne, ws, ws_bytes, P, stream);
  if (r) return r;
  char* w = (char*)ws;
  PoleArgs a = pole_args(lat, pol, P, w);
  a.evals = const_cast<double*>(evals);
  a.wphys = const_cast<double*>(wphys);
  a.worb = pdos ? const_cast<double*>(worb) : nullptr;
  HIPCHK(h, launch_pole_dos(a, mu, eta, e_min, e_max, ne, (double*)(w + P.part), dos, pdos, stream));
  return DMFT_OK;
}

int dmft_pole_energy(dmft_handle h, const dmft_lattice* lat, const dmft_poles* pol, double mu, const double* evals,
                     const double* evecs, const double* wphys, const double* worb, double* out, void* ws,
                     size_t ws_bytes, hipStream_t stream) {
  if (!evals || !evecs || !wphys || !worb || !out)
    return fail(h, DMFT_EINVAL, "evals, evecs, wphys, worb and out are required");
  if (!std::isfinite(mu)) return fail(h, DMFT_EINVAL, "mu is not finite");
  PoleLayout P;
  int r = pole_prepare(h, lat, pol, 0, ws, ws_bytes, P, stream);
  if (r) return r;
  char* w = (char*)ws;
  PoleArgs a = pole_args(lat, pol, P, w);
  a.evals = const_cast<double*>(evals);
  a.evecs = const_cast<double*>(evecs);
  a.wphys = const_cast<double*>(wphys);
  a.worb = const_cast<double*>(worb);
  HIPCHK(h, launch_pole_energy(a, mu, (double*)(w + P.epart), out, stream));
  return DMFT_OK;
}

int dmft_hubbard1(dmft_handle h, int natoms, int nc, const double* eps, const double* U, const double* mu,
                  double beta, double wtol, double* sigma_inf, int32_t* npoles, double* pos, double* wgt, double* occ,
                  double* e_u, hipStream_t stream) {
  if (!h) return DMFT_EINVAL;
  if (natoms < 1) return fail(h, DMFT_EINVAL, "natoms must be >= 1");
  if (nc < 1 || nc > 16) return fail(h, DMFT_EINVAL, "nc must be in 1..16 (got %d)", nc);
  if (!(beta > 0) || !std::isfinite(beta)) return fail(h, DMFT_EINVAL, "beta must be positive and finite");
  if (!(wtol >= 0) || !std::isfinite(wtol) || wtol >= 1.0) return fail(h, DMFT_EINVAL, "wtol must be in [0, 1)");
  if (!eps || !U || !mu || !sigma_inf || !npoles || !pos || !wgt)
    return fail(h, DMFT_EINVAL, "eps, U, mu, sigma_inf, npoles, pos and wgt are required");
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, launch_hubbard1(natoms, nc, eps, U, mu, beta, wtol, sigma_inf, npoles, pos, wgt, occ, e_u, stream));
  return DMFT_OK;
}

int dmft_sigma_from_poles(dmft_handle h, int nc, const dmft_poles* pol, int nw, double mu, double* sigma,
                          hipStream_t stream) {
  if (!h) return DMFT_EINVAL;
  if (!pol || !sigma) return fail(h, DMFT_EINVAL, "poles and sigma are required");
  if (nc < 1 || nc > 16) return fail(h, DMFT_EINVAL, "nc must be in 1..16 (got %d)", nc);
  if (nw < 1) return fail(h, DMFT_EINVAL, "nw must be >= 1");
  if (pol->np < 0 || (pol->np > 0 && (!pol->p || !pol->v))) return fail(h, DMFT_EINVAL, "bad pole arrays");
  if (!(pol->beta > 0) || !std::isfinite(pol->beta)) return fail(h, DMFT_EINVAL, "beta must be positive and finite");
  if (!std::isfinite(mu)) return fail(h, DMFT_EINVAL, "mu is not finite");
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, launch_sigma_from_poles(nw, nc, pol->np, pol->beta, mu, pol->p, pol->v, pol->sigma_inf, sigma, stream));
  return DMFT_OK;
}

int dmft_hubbard1_poles(dmft_handle h, int nc, int nc_lat, int a0, const int32_t* npoles, const double* pos,
                        const double* wgt, double* p, double* v, int32_t* np_out, hipStream_t stream) {
  if (!h) return DMFT_EINVAL;
  if (nc < 1 || nc > 16 || nc_lat < 1 || nc_lat > 16 || a0 < 0 || a0 + nc > nc_lat)
    return fail(h, DMFT_EINVAL, "need 1 <= nc, nc_lat <= 16 and 0 <= a0, a0 + nc <= nc_lat");
  if (!npoles || !pos || !wgt || !p || !v || !np_out) return fail(h, DMFT_EINVAL, "all arrays are required");
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, launch_hubbard1_poles(nc, nc_lat, a0, npoles, pos, wgt, p, v, np_out, stream));
  return DMFT_OK;
}

}  // extern "C"
