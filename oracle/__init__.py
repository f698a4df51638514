"""FP64 CPU oracle for the lattice Dyson step (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library does not import, link or call
anything here, and nothing here imports the product.

The arithmetic lives in ``dmft_oracle.c`` (plain loops, Gaussian elimination
with partial pivoting, no BLAS/LAPACK); this module only compiles it with gcc
when needed and marshals numpy arrays through ctypes.  See the C file's header
for the formulas and the paper passages they follow.

Inputs are duck-typed: a *lattice* is any object with attributes ``nk, nc, nb``
(int array [nk]), ``eps`` (float64, bands of all k concatenated), ``wk``
(float64 [nk]) and ``proj`` (complex128, each k's nc x nb_k projector
row-major, concatenated); a *self-energy* has ``nw, beta, sigma``
(complex128 [nw, nc, nc]), ``sigma_inf`` (complex128 [nc, nc] or None) and
``e_dc`` (float64 [nc]).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dmft_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no fast-math) and OpenMP."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-D_GNU_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Lattice(C.Structure):
    _fields_ = [("nk", C.c_int), ("nc", C.c_int), ("nb", C.c_void_p), ("off_b", C.c_void_p),
                ("off_p", C.c_void_p), ("eps", C.c_void_p), ("wk", C.c_void_p),
                ("proj", C.c_void_p)]


class _Sigma(C.Structure):
    _fields_ = [("nw", C.c_int), ("beta", C.c_double), ("sigma", C.c_void_p),
                ("sigma_inf", C.c_void_p), ("e_dc", C.c_void_p)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = C.CDLL(_LIB)
            P, I, D = C.c_void_p, C.c_int, C.c_double
            lib.orc_density.argtypes = [P, P, D, I, P, I, P, P, I]
            lib.orc_gloc.argtypes = [P, P, D, P, I, P, I]
            lib.orc_trace.argtypes = [P, P, D, I, P, P, I]
            lib.orc_vjp.argtypes = [P, P, D, I, P, P, P, P, I]
            lib.orc_find_mu_bisect.argtypes = [P, P, I, D, D, D, D, I, P, P, P, I]
            lib.orc_invert.argtypes = [I, P, P]
            lib.orc_green.argtypes = [P, P, D, I, I, P]
            for f in (lib.orc_density, lib.orc_gloc, lib.orc_trace, lib.orc_vjp,
                      lib.orc_find_mu_bisect, lib.orc_invert, lib.orc_green):
                f.restype = C.c_int
            _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class _Pack:
    """Keeps the contiguous arrays alive while the C structs point at them."""

    def __init__(self, lat, sig):
        self.nb = np.ascontiguousarray(lat.nb, dtype=np.int32)
        nk, nc = int(lat.nk), int(lat.nc)
        assert self.nb.shape == (nk,)
        self.off_b = np.zeros(nk + 1, np.int64)
        self.off_b[1:] = np.cumsum(self.nb)
        self.off_p = self.off_b * nc
        self.eps = np.ascontiguousarray(lat.eps, dtype=np.float64)
        self.wk = np.ascontiguousarray(lat.wk, dtype=np.float64)
        self.proj = np.ascontiguousarray(lat.proj, dtype=np.complex128)
        assert self.eps.size == self.off_b[-1] and self.proj.size == self.off_p[-1]
        self.sigma = np.ascontiguousarray(sig.sigma, dtype=np.complex128)
        assert self.sigma.shape == (int(sig.nw), nc, nc)
        self.sigma_inf = (None if sig.sigma_inf is None
                          else np.ascontiguousarray(sig.sigma_inf, dtype=np.complex128))
        self.e_dc = np.ascontiguousarray(sig.e_dc, dtype=np.float64)
        self.lat = _Lattice(nk, nc, _ptr(self.nb), _ptr(self.off_b), _ptr(self.off_p),
                            _ptr(self.eps), _ptr(self.wk), _ptr(self.proj))
        self.sig = _Sigma(int(sig.nw), float(sig.beta), _ptr(self.sigma), _ptr(self.sigma_inf),
                          _ptr(self.e_dc))
        self.nk, self.nc, self.nw = nk, nc, int(sig.nw)

    @property
    def refs(self):
        return C.byref(self.lat), C.byref(self.sig)


def _threads(nthreads):
    """OpenMP threads: the argument, else ORACLE_THREADS, else the host's cores up to 16."""
    if nthreads:
        return int(nthreads)
    return int(os.environ.get("ORACLE_THREADS", min(16, os.cpu_count() or 1)))


def density(lat, sig, mu, tail_order=2, klist=None, nthreads=None):
    """N(k) for the k in ``klist`` (default: all).  Returns (list of nb_k x nb_k
    complex arrays, array of tr N(k))."""
    pk = _Pack(lat, sig)
    ks = np.arange(pk.nk, dtype=np.int32) if klist is None else np.ascontiguousarray(klist, np.int32)
    sizes = pk.nb[ks].astype(np.int64) ** 2
    out = np.zeros(int(sizes.sum()), np.complex128)
    ntr = np.zeros(len(ks), np.float64)
    r = _load().orc_density(*pk.refs, float(mu), int(tail_order), _ptr(ks), len(ks), _ptr(out),
                            _ptr(ntr), _threads(nthreads))
    if r:
        raise RuntimeError("oracle density failed (%d)" % r)
    mats, o = [], 0
    for k in ks:
        n = int(pk.nb[k])
        mats.append(out[o:o + n * n].reshape(n, n))
        o += n * n
    return mats, ntr


def gloc(lat, sig, mu, nlist=None, nthreads=None):
    """G_loc(i w_n) for the n in ``nlist`` (default: all): [len, nc, nc]."""
    pk = _Pack(lat, sig)
    ns = np.arange(pk.nw, dtype=np.int32) if nlist is None else np.ascontiguousarray(nlist, np.int32)
    out = np.zeros((len(ns), pk.nc, pk.nc), np.complex128)
    r = _load().orc_gloc(*pk.refs, float(mu), _ptr(ns), len(ns), _ptr(out), _threads(nthreads))
    if r:
        raise RuntimeError("oracle gloc failed (%d)" % r)
    return out


def trace(lat, sig, mu, tail_order=2, nthreads=None):
    """(N_tot(mu), dN_tot/dmu)."""
    pk = _Pack(lat, sig)
    n, d = np.zeros(1), np.zeros(1)
    r = _load().orc_trace(*pk.refs, float(mu), int(tail_order), _ptr(n), _ptr(d), _threads(nthreads))
    if r:
        raise RuntimeError("oracle trace failed (%d)" % r)
    return float(n[0]), float(d[0])


def vjp(lat, sig, mu, nbar=None, gbar=None, tail_order=2, nthreads=None):
    """(sigma_bar [nw, nc, nc], mu_bar) for upstream ``nbar`` (list of nb_k x nb_k
    complex arrays, one per k, or None) and ``gbar`` ([nw, nc, nc] or None)."""
    pk = _Pack(lat, sig)
    nb_flat = None
    if nbar is not None:
        nb_flat = np.ascontiguousarray(np.concatenate([np.asarray(m, np.complex128).ravel() for m in nbar]))
        assert nb_flat.size == int((pk.nb.astype(np.int64) ** 2).sum())
    gb = None if gbar is None else np.ascontiguousarray(gbar, np.complex128)
    out = np.zeros((pk.nw, pk.nc, pk.nc), np.complex128)
    mub = np.zeros(1)
    r = _load().orc_vjp(*pk.refs, float(mu), int(tail_order), _ptr(nb_flat), _ptr(gb), _ptr(out),
                        _ptr(mub), _threads(nthreads))
    if r:
        raise RuntimeError("oracle vjp failed (%d)" % r)
    return out, float(mub[0])


def find_mu_bisect(lat, sig, n_target, tol, lo, hi, max_iter=200, tail_order=2, nthreads=None):
    """Plain bisection; returns (mu, passes, N(mu))."""
    pk = _Pack(lat, sig)
    mu, p, n = np.zeros(1), np.zeros(1, np.int32), np.zeros(1)
    r = _load().orc_find_mu_bisect(*pk.refs, int(tail_order), float(n_target), float(tol), float(lo),
                                   float(hi), int(max_iter), _ptr(mu), _ptr(p), _ptr(n),
                                   _threads(nthreads))
    if r:
        raise RuntimeError("oracle bisection failed (%d)" % r)
    return float(mu[0]), int(p[0]), float(n[0])


def invert(a):
    """Inverse of one dense complex matrix by the oracle's own elimination."""
    a = np.ascontiguousarray(a, np.complex128)
    g = np.zeros_like(a)
    if _load().orc_invert(a.shape[0], _ptr(a), _ptr(g)):
        raise ZeroDivisionError("singular")
    return g


def green(lat, sig, mu, k, n):
    """G_kn = A_kn^{-1} for one k-point and one Matsubara index."""
    pk = _Pack(lat, sig)
    nb = int(pk.nb[k])
    g = np.zeros((nb, nb), np.complex128)
    if _load().orc_green(*pk.refs, float(mu), int(k), int(n), _ptr(g)):
        raise ZeroDivisionError("singular")
    return g


def impurity_level(lat, sig):
    """E_imp = sum_k w_k S_k diag(E_k) S_k^dag - diag(V_DC) (nc x nc): the level
    of the correlated orbitals in the impurity model of Sec. 3.2.2 (eq. H_imp),
    with V_DC entering as it does in the lattice resolvent (eq. dmftloop1)."""
    nc = int(lat.nc)
    e = np.zeros((nc, nc), np.complex128)
    for k in range(int(lat.nk)):
        p = lat.proj_k(k)
        eps = lat.eps_k(k)
        for a in range(nc):
            for b in range(nc):
                e[a, b] += lat.wk[k] * np.sum(p[a] * eps * np.conj(p[b]))
    return e - np.diag(np.asarray(sig.e_dc, np.float64))


def hybridization(lat, sig, mu, nlist=None, nthreads=None):
    """Hybridization function of the DMFT self-consistency (Sec. 3.2.2 eq.
    dmftloop2), Delta(i w_n) = i w_n + mu - E_imp - Sigma(i w_n) - G_loc(i w_n)^-1,
    for the n in ``nlist`` (default: all).  Returns (delta [len, nc, nc], E_imp).
    G_loc is the oracle's own; its inverse is the oracle's pivoting elimination."""
    ns = list(range(int(sig.nw))) if nlist is None else list(nlist)
    g = gloc(lat, sig, mu, ns, nthreads=nthreads)
    eimp = impurity_level(lat, sig)
    nc = int(lat.nc)
    out = np.zeros((len(ns), nc, nc), np.complex128)
    for i, n in enumerate(ns):
        w = (2.0 * n + 1.0) * np.pi / float(sig.beta)
        out[i] = (1j * w + mu) * np.eye(nc) - eimp - np.asarray(sig.sigma[n]) - invert(g[i])
    return out, eimp
