"""PyTorch-facing binding of libdmft (device memory and streams come from torch).

The functions keep the C ABI's names and only marshal arguments: they pass
``tensor.data_ptr()`` and torch's current HIP stream to the library, whose
kernels do all of the computation.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import _lib
from ._lib import BISECT, FORM_AUTO, FORM_DENSE, FORM_LOWRANK, NEWTON, DmftLattice, DmftPoles, DmftSigma, check

__all__ = ["Lattice", "SelfEnergy", "PoleSelfEnergy", "PoleEigensystem", "Context", "NEWTON", "BISECT",
           "FORM_AUTO", "FORM_DENSE", "FORM_LOWRANK"]


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


@dataclass
class Lattice:
    """Band windows, energies and projectors of every k (device-resident)."""

    nk: int
    nc: int
    nb_max: int
    nb: Optional[np.ndarray]      # host int32 [nk], or None when every k has nb_max bands
    eps: torch.Tensor             # float64, all k concatenated
    wk: torch.Tensor              # float64 [nk]
    proj: torch.Tensor            # complex128, all k concatenated (nc x nb_k row-major)

    @classmethod
    def from_host(cls, lat, device="cuda"):
        nb = np.ascontiguousarray(lat.nb, np.int32)
        uniform = bool((nb == nb[0]).all())
        return cls(int(lat.nk), int(lat.nc), int(nb.max()), None if uniform else nb,
                   torch.as_tensor(np.ascontiguousarray(lat.eps, np.float64), device=device),
                   torch.as_tensor(np.ascontiguousarray(lat.wk, np.float64), device=device),
                   torch.as_tensor(np.ascontiguousarray(lat.proj, np.complex128), device=device))

    def nb_array(self):
        return np.full(self.nk, self.nb_max, np.int32) if self.nb is None else self.nb

    def n_size(self):
        return int((self.nb_array().astype(np.int64) ** 2).sum())

    def struct(self):
        self._nb_keep = None if self.nb is None else np.ascontiguousarray(self.nb, np.int32)
        return DmftLattice(self.nk, self.nc, self.nb_max,
                           None if self._nb_keep is None else self._nb_keep.ctypes.data_as(C.c_void_p),
                           _ptr(self.eps), _ptr(self.wk), _ptr(self.proj))


@dataclass
class SelfEnergy:
    nw: int
    beta: float
    sigma: torch.Tensor                 # complex128 [nw, nc, nc]
    sigma_inf: Optional[torch.Tensor]   # complex128 [nc, nc] or None
    e_dc: torch.Tensor                  # float64 [nc]

    @classmethod
    def from_host(cls, sig, device="cuda"):
        si = None if sig.sigma_inf is None else torch.as_tensor(
            np.ascontiguousarray(sig.sigma_inf, np.complex128), device=device)
        return cls(int(sig.nw), float(sig.beta),
                   torch.as_tensor(np.ascontiguousarray(sig.sigma, np.complex128), device=device), si,
                   torch.as_tensor(np.ascontiguousarray(sig.e_dc, np.float64), device=device))

    def struct(self):
        return DmftSigma(self.nw, self.beta, _ptr(self.sigma), _ptr(self.sigma_inf), _ptr(self.e_dc))


@dataclass
class PoleSelfEnergy:
    """Pole form Sigma(i w) = Sigma_inf + sum_i V_i^dag V_i / (i w - p_i) (device-resident)."""

    np: int
    beta: float
    p: Optional[torch.Tensor]           # float64 [np]
    v: Optional[torch.Tensor]           # complex128 [np, nc]
    sigma_inf: Optional[torch.Tensor]   # complex128 [nc, nc] or None
    e_dc: torch.Tensor                  # float64 [nc]

    @classmethod
    def from_host(cls, sig, device="cuda"):
        """From an object with ``beta``, ``poles`` (list of (p_i, V_i[nc])),
        ``sigma_inf`` and ``e_dc``."""
        poles = list(sig.poles)
        p = v = None
        if poles:
            p = torch.as_tensor(np.array([float(q) for q, _ in poles], np.float64), device=device)
            v = torch.as_tensor(np.ascontiguousarray(np.stack([np.asarray(x, np.complex128) for _, x in poles])),
                                device=device)
        si = None if sig.sigma_inf is None else torch.as_tensor(
            np.ascontiguousarray(sig.sigma_inf, np.complex128), device=device)
        return cls(len(poles), float(sig.beta), p, v, si,
                   torch.as_tensor(np.ascontiguousarray(sig.e_dc, np.float64), device=device))

    def struct(self):
        return DmftPoles(self.np, self.beta, _ptr(self.p), _ptr(self.v), _ptr(self.sigma_inf), _ptr(self.e_dc))


@dataclass
class PoleEigensystem:
    """Output of Context.pole_eig: per k, mp = nb_max + np entries (zero past nb_k + np)."""

    mp: int
    evals: torch.Tensor                 # float64 [nk, mp], ascending per k
    evecs: torch.Tensor                 # complex128 [nk, nb_max, mp]: <phi_n | psi_l>
    wphys: torch.Tensor                 # float64 [nk, mp]
    worb: Optional[torch.Tensor]        # float64 [nk, mp, nc] or None


class Context:
    """One library handle on one GPU plus a cached workspace."""

    def __init__(self, device: int = 0):
        self.lib = _lib.load()
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        code = self.lib.dmft_create(C.byref(h), device)
        if code:
            raise _lib.DmftError(code, "dmft_create")
        self.h = h
        self._ws = None

    def close(self):
        if self.h:
            self.lib.dmft_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ workspace
    def workspace(self, nbytes: int) -> torch.Tensor:
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            ws[:256].zero_()
            assert ws.data_ptr() % 256 == 0
            self._ws = ws
        return self._ws

    def workspace_size(self, lat: Lattice, sig: SelfEnergy) -> int:
        n = C.c_size_t()
        ls, ss = lat.struct(), sig.struct()
        check(self.h, self.lib.dmft_workspace_size(self.h, C.byref(ls), C.byref(ss), C.byref(n)))
        return int(n.value)

    def _call_ws(self, lat, sig):
        ws = self.workspace(self.workspace_size(lat, sig))
        return ws, C.c_size_t(ws.numel())

    # ------------------------------------------------------------------ entry points
    def gloc_compute(self, lat: Lattice, sig: SelfEnergy, mu: float) -> torch.Tensor:
        gloc = torch.empty((sig.nw, lat.nc, lat.nc), dtype=torch.complex128, device=self.device)
        ws, nws = self._call_ws(lat, sig)
        ls, ss = lat.struct(), sig.struct()
        check(self.h, self.lib.gloc_compute(self.h, C.byref(ls), C.byref(ss), float(mu), _ptr(gloc),
                                            _ptr(ws), nws, _stream(self.device)))
        return gloc

    def hybridization(self, lat: Lattice, sig: SelfEnergy, mu: float, gloc: torch.Tensor):
        """DMFT self-consistency step: (Delta [nw, nc, nc], E_imp [nc, nc]) from
        G_loc (as returned by gloc_compute / density_matrix at the same mu)."""
        delta = torch.empty((sig.nw, lat.nc, lat.nc), dtype=torch.complex128, device=self.device)
        eimp = torch.empty((lat.nc, lat.nc), dtype=torch.complex128, device=self.device)
        gloc = gloc.contiguous()
        ws, nws = self._call_ws(lat, sig)
        ls, ss = lat.struct(), sig.struct()
        check(self.h, self.lib.dmft_hybridization(self.h, C.byref(ls), C.byref(ss), float(mu), _ptr(gloc), _ptr(delta),
                                                  _ptr(eimp), _ptr(ws), nws, _stream(self.device)))
        return delta, eimp

    def density_matrix(self, lat: Lattice, sig: SelfEnergy, mu: float, tail_order: int = 2, nk=True,
                       gloc=True, scalars=True):
        """Returns (nk_flat or None, gloc or None, scalars or None); nk_flat holds
        N(k) for all k concatenated (nb_k x nb_k each); scalars = [N_tot, n_corr, <H_KS>]."""
        nk_t = torch.empty(lat.n_size(), dtype=torch.complex128, device=self.device) if nk else None
        gl_t = torch.empty((sig.nw, lat.nc, lat.nc), dtype=torch.complex128, device=self.device) if gloc else None
        sc_t = torch.empty(3, dtype=torch.float64, device=self.device) if scalars else None
        ws, nws = self._call_ws(lat, sig)
        ls, ss = lat.struct(), sig.struct()
        check(self.h, self.lib.density_matrix(self.h, C.byref(ls), C.byref(ss), float(mu), int(tail_order),
                                              _ptr(nk_t), _ptr(gl_t), _ptr(sc_t), _ptr(ws), nws,
                                              _stream(self.device)))
        return nk_t, gl_t, sc_t

    def dmft_ntot(self, lat: Lattice, sig: SelfEnergy, mu: float, tail_order: int = 2) -> torch.Tensor:
        """[N_tot(mu), dN_tot/dmu] on the device."""
        out = torch.empty(2, dtype=torch.float64, device=self.device)
        ws, nws = self._call_ws(lat, sig)
        ls, ss = lat.struct(), sig.struct()
        check(self.h, self.lib.dmft_ntot(self.h, C.byref(ls), C.byref(ss), float(mu), int(tail_order),
                                         _ptr(out), _ptr(ws), nws, _stream(self.device)))
        return out

    def density_matrix_vjp(self, lat: Lattice, sig: SelfEnergy, mu: float, nk_bar=None, gloc_bar=None,
                           tail_order: int = 2):
        """(sigma_bar [nw, nc, nc] complex128, mu_bar [1] float64) on the device."""
        sb = torch.empty((sig.nw, lat.nc, lat.nc), dtype=torch.complex128, device=self.device)
        mb = torch.empty(1, dtype=torch.float64, device=self.device)
        nkb = None if nk_bar is None else nk_bar.contiguous()
        gb = None if gloc_bar is None else gloc_bar.contiguous()
        ws, nws = self._call_ws(lat, sig)
        ls, ss = lat.struct(), sig.struct()
        check(self.h, self.lib.density_matrix_vjp(self.h, C.byref(ls), C.byref(ss), float(mu), int(tail_order),
                                                  _ptr(nkb), _ptr(gb), _ptr(sb), _ptr(mb), _ptr(ws), nws,
                                                  _stream(self.device)))
        return sb, mb

    def dmft_ntot_vjp(self, lat: Lattice, sig: SelfEnergy, mu: float, tail_order: int = 2):
        """(out [N_tot, dN/dmu] float64, dN/dSigma [nw, nc, nc] complex128) on the device."""
        out = torch.empty(2, dtype=torch.float64, device=self.device)
        sb = torch.empty((sig.nw, lat.nc, lat.nc), dtype=torch.complex128, device=self.device)
        ws, nws = self._call_ws(lat, sig)
        ls, ss = lat.struct(), sig.struct()
        check(self.h, self.lib.dmft_ntot_vjp(self.h, C.byref(ls), C.byref(ss), float(mu), int(tail_order),
                                             _ptr(sb), _ptr(out), _ptr(ws), nws, _stream(self.device)))
        return out, sb

    def find_mu(self, lat: Lattice, sig: SelfEnergy, n_target: float, tol_n: float = 1e-8, method=NEWTON,
                mu_lo: float = -40.0, mu_hi: float = 40.0, mu0: Optional[float] = None, max_iter: int = 200,
                tail_order: int = 2):
        """(mu, passes, N(mu))."""
        ws, nws = self._call_ws(lat, sig)
        ls, ss = lat.struct(), sig.struct()
        mu, passes, n = C.c_double(), C.c_int(), C.c_double()
        m0 = 0.5 * (mu_lo + mu_hi) if mu0 is None else mu0
        check(self.h, self.lib.find_mu(self.h, C.byref(ls), C.byref(ss), int(tail_order), float(n_target),
                                       float(tol_n), int(method), float(mu_lo), float(mu_hi), float(m0),
                                       int(max_iter), C.byref(mu), C.byref(passes), C.byref(n), _ptr(ws), nws,
                                       _stream(self.device)))
        return mu.value, passes.value, n.value

    def autotune(self, lat: Lattice, sig: SelfEnergy, mu: float) -> str:
        """Times the kernel variants and tile sizes of this shape and keeps the
        fastest in the handle; returns the library's report."""
        ws = self.workspace(2 * self.workspace_size(lat, sig))
        nws = C.c_size_t(ws.numel())
        ls, ss = lat.struct(), sig.struct()
        buf = C.create_string_buffer(8192)
        check(self.h, self.lib.dmft_autotune(self.h, C.byref(ls), C.byref(ss), float(mu), _ptr(ws), nws,
                                             _stream(self.device), buf, 8192))
        return buf.value.decode()

    # ------------------------------------------------------------------ batched pass
    def batched_plan(self, lats: List[Lattice], sigs: List[SelfEnergy], tail_order: int = 2):
        """Plan one persistent pass over several (lattice, self-energy) iterates.
        Returns the plan's workspace (kept alive by the context)."""
        n = len(lats)
        self._b_ls = [l.struct() for l in lats]
        self._b_ss = [s.struct() for s in sigs]
        lp = (C.c_void_p * n)(*[C.addressof(x) for x in self._b_ls])
        sp = (C.c_void_p * n)(*[C.addressof(x) for x in self._b_ss])
        self._b_lp, self._b_sp = lp, sp
        nb = C.c_size_t()
        check(self.h, self.lib.dmft_batched_workspace_size(self.h, n, lp, sp, C.byref(nb)))
        self._b_ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        self._b_ws[:256].zero_()
        self._b_keep = (lats, sigs)
        check(self.h, self.lib.dmft_batched_plan(self.h, n, lp, sp, int(tail_order), _ptr(self._b_ws),
                                                 C.c_size_t(self._b_ws.numel()), _stream(self.device)))
        return self._b_ws

    def batched_set_form(self, form: int):
        """Form of the step for later batched plans: FORM_AUTO (timed), FORM_DENSE, FORM_LOWRANK."""
        check(self.h, self.lib.dmft_batched_set_form(self.h, int(form)))

    def batched_form(self) -> int:
        """Form of the current batched plan (FORM_DENSE or FORM_LOWRANK), -1 without a plan."""
        return int(self.lib.dmft_batched_form(self.h))

    def batched_set_concurrent(self, mode: int) -> None:
        """Class kernels of later low-rank batched plans: 1 concurrent, 0 one after
        another, -1 (default) whichever the plan times faster."""
        check(self.h, self.lib.dmft_batched_set_concurrent(self.h, int(mode)))

    def batched_set_tile_candidate(self, index: int) -> None:
        """Tiles of later batched plans: candidate `index` of the plan's list
        without timing the others, or -1 (default) the fastest of all."""
        check(self.h, self.lib.dmft_batched_set_tile_candidate(self.h, int(index)))

    def batched_tile_candidate(self) -> int:
        """Tile candidate of the current batched plan (-1 without a plan)."""
        return int(self.lib.dmft_batched_tile_candidate(self.h))

    def batched_concurrent(self) -> int:
        """1 if the class kernels of the low-rank batched plan run concurrently,
        0 if one after another, -1 without such a plan."""
        return int(self.lib.dmft_batched_concurrent(self.h))

    def batched_classes(self):
        """Item classes of the low-rank batched plan: list of dicts with the
        padded size, inversion columns, item count and summed kernel ms since
        timing was enabled."""
        n = self.lib.dmft_batched_classes(self.h, 0, None, None, None, None)
        if n < 0:
            check(self.h, n)
        nbp, ncls, items = (np.zeros(max(n, 1), np.int32) for _ in range(3))
        ms = np.zeros(max(n, 1), np.float64)
        n = self.lib.dmft_batched_classes(self.h, n, nbp.ctypes.data_as(C.c_void_p), ncls.ctypes.data_as(C.c_void_p),
                                          items.ctypes.data_as(C.c_void_p), ms.ctypes.data_as(C.c_void_p))
        if n < 0:
            check(self.h, n)
        return [{"nbp": int(nbp[i]), "ncls": int(ncls[i]), "items": int(items[i]), "kernel_ms": float(ms[i])}
                for i in range(n)]

    def _batched_ptrs(self, outs):
        n = len(self._b_ls)
        return (C.c_void_p * n)(*[(o.data_ptr() if o is not None else 0) for o in outs])

    def batched_outputs(self):
        lats, sigs = self._b_keep
        nks = [torch.empty(l.n_size(), dtype=torch.complex128, device=self.device) for l in lats]
        gls = [torch.empty((s.nw, l.nc, l.nc), dtype=torch.complex128, device=self.device) for l, s in zip(lats, sigs)]
        return nks, gls

    def batched_pass(self, mu_dev: torch.Tensor, nks, gls):
        check(self.h, self.lib.dmft_batched_pass(self.h, _ptr(mu_dev), self._batched_ptrs(nks), self._batched_ptrs(gls),
                                                 _ptr(self._b_ws), C.c_size_t(self._b_ws.numel()),
                                                 _stream(self.device)))

    def batched_graph_capture(self, mu_dev: torch.Tensor, nks, gls):
        check(self.h, self.lib.dmft_batched_graph_capture(self.h, _ptr(mu_dev), self._batched_ptrs(nks),
                                                          self._batched_ptrs(gls), _ptr(self._b_ws),
                                                          C.c_size_t(self._b_ws.numel()), _stream(self.device)))

    def batched_graph_launch(self):
        check(self.h, self.lib.dmft_batched_graph_launch(self.h, _stream(self.device)))

    def batched_sync_status(self):
        check(self.h, self.lib.dmft_sync_status(self.h, _ptr(self._b_ws), _stream(self.device)))

    def variants(self, kind: int, nbp: int):
        buf = (C.c_int * 16)()
        n = self.lib.dmft_variants(int(kind), int(nbp), buf, 16)
        return list(buf[:n])

    def set_variant(self, kind: int, nbp: int, var: int):
        check(self.h, self.lib.dmft_set_variant(self.h, int(kind), int(nbp), int(var)))

    def get_variant(self, kind: int, nbp: int) -> int:
        """The variant code later calls of this kind and padded size use."""
        return int(self.lib.dmft_get_variant(self.h, int(kind), int(nbp)))

    # ------------------------------------------------------------------ pole-expansion route
    def _pole_ws(self, lat: Lattice, pol: PoleSelfEnergy, ne_max: int = 0):
        n = C.c_size_t()
        ls, ps = lat.struct(), pol.struct()
        check(self.h, self.lib.dmft_pole_workspace_size(self.h, C.byref(ls), C.byref(ps), int(ne_max), C.byref(n)))
        ws = self.workspace(int(n.value))
        return ws, C.c_size_t(ws.numel())

    def pole_eig(self, lat: Lattice, pol: PoleSelfEnergy, orb: bool = True) -> PoleEigensystem:
        mp = lat.nb_max + pol.np
        dev = self.device
        es = PoleEigensystem(mp, torch.empty((lat.nk, mp), dtype=torch.float64, device=dev),
                             torch.empty((lat.nk, lat.nb_max, mp), dtype=torch.complex128, device=dev),
                             torch.empty((lat.nk, mp), dtype=torch.float64, device=dev),
                             torch.empty((lat.nk, mp, lat.nc), dtype=torch.float64, device=dev) if orb else None)
        ws, nws = self._pole_ws(lat, pol)
        ls, ps = lat.struct(), pol.struct()
        check(self.h, self.lib.dmft_pole_eig(self.h, C.byref(ls), C.byref(ps), _ptr(es.evals), _ptr(es.evecs),
                                             _ptr(es.wphys), _ptr(es.worb), _ptr(ws), nws, _stream(self.device)))
        return es

    def pole_sweeps(self, lat: Lattice, pol: PoleSelfEnergy) -> np.ndarray:
        out = np.zeros(lat.nk, np.int32)
        ls, ps = lat.struct(), pol.struct()
        check(self.h, self.lib.dmft_pole_sweeps(self.h, C.byref(ls), C.byref(ps), _ptr(self._ws),
                                                out.ctypes.data_as(C.c_void_p), _stream(self.device)))
        return out

    def pole_density(self, lat: Lattice, pol: PoleSelfEnergy, es: PoleEigensystem, mu: float, nw_trunc: int = 0,
                     nk=True, scalars=True):
        """(N(k) of all k concatenated or None, [N_tot, n_corr, <H_KS>] or None)."""
        nk_t = torch.empty(lat.n_size(), dtype=torch.complex128, device=self.device) if nk else None
        sc_t = torch.empty(3, dtype=torch.float64, device=self.device) if scalars else None
        ws, nws = self._pole_ws(lat, pol)
        ls, ps = lat.struct(), pol.struct()
        check(self.h, self.lib.dmft_pole_density(self.h, C.byref(ls), C.byref(ps), float(mu), int(nw_trunc),
                                                 _ptr(es.evals), _ptr(es.evecs), _ptr(nk_t), _ptr(sc_t), _ptr(ws),
                                                 nws, _stream(self.device)))
        return nk_t, sc_t

    def pole_find_mu(self, lat: Lattice, pol: PoleSelfEnergy, es: PoleEigensystem, n_target: float,
                     tol_n: float = 1e-8, method=NEWTON, mu_lo: float = -40.0, mu_hi: float = 40.0,
                     max_iter: int = 200):
        """(mu, evaluations of N, N(mu))."""
        ws, nws = self._pole_ws(lat, pol)
        ls, ps = lat.struct(), pol.struct()
        mu, passes, n = C.c_double(), C.c_int(), C.c_double()
        check(self.h, self.lib.dmft_pole_find_mu(self.h, C.byref(ls), C.byref(ps), _ptr(es.evals), _ptr(es.wphys),
                                                 float(n_target), float(tol_n), int(method), float(mu_lo),
                                                 float(mu_hi), int(max_iter), C.byref(mu), C.byref(passes),
                                                 C.byref(n), _ptr(ws), nws, _stream(self.device)))
        return mu.value, passes.value, n.value

    def pole_dos(self, lat: Lattice, pol: PoleSelfEnergy, es: PoleEigensystem, mu: float, eta: float,
                 e_min: float, e_max: float, ne: int, pdos: bool = True):
        """(D [ne], D_alpha [ne, nc] or None) on e_min .. e_max."""
        d = torch.empty(ne, dtype=torch.float64, device=self.device)
        pd = torch.empty((ne, lat.nc), dtype=torch.float64, device=self.device) if pdos else None
        ws, nws = self._pole_ws(lat, pol, ne)
        ls, ps = lat.struct(), pol.struct()
        check(self.h, self.lib.dmft_pole_dos(self.h, C.byref(ls), C.byref(ps), _ptr(es.evals), _ptr(es.wphys),
                                             _ptr(es.worb), float(mu), float(eta), float(e_min), float(e_max),
                                             int(ne), _ptr(d), _ptr(pd), _ptr(ws), nws, _stream(self.device)))
        return d, pd

    def pole_energy(self, lat: Lattice, pol: PoleSelfEnergy, es: PoleEigensystem, mu: float) -> torch.Tensor:
        """Device [5 + nc] = [B, N_tot, <H_KS>, <V_DC>, <H_U>, n_alpha ...] (see dmft_pole_energy)."""
        out = torch.empty(5 + lat.nc, dtype=torch.float64, device=self.device)
        ws, nws = self._pole_ws(lat, pol)
        ls, ps = lat.struct(), pol.struct()
        check(self.h, self.lib.dmft_pole_energy(self.h, C.byref(ls), C.byref(ps), float(mu), _ptr(es.evals),
                                                _ptr(es.evecs), _ptr(es.wphys), _ptr(es.worb), _ptr(out), _ptr(ws),
                                                nws, _stream(self.device)))
        return out

    def hubbard1(self, eps: torch.Tensor, U: torch.Tensor, mu: torch.Tensor, beta: float, wtol: float = 1e-13):
        """Hubbard-I atoms: eps [natoms, nc], U and mu [natoms] (float64, device).
        Returns a dict of device tensors sigma_inf [natoms, nc], npoles [natoms, nc],
        pos and wgt [natoms, nc, nc], occ [natoms, nc], e_u [natoms]."""
        natoms, nc = eps.shape
        dev = self.device
        out = {"sigma_inf": torch.empty((natoms, nc), dtype=torch.float64, device=dev),
               "npoles": torch.empty((natoms, nc), dtype=torch.int32, device=dev),
               "pos": torch.empty((natoms, nc, nc), dtype=torch.float64, device=dev),
               "wgt": torch.empty((natoms, nc, nc), dtype=torch.float64, device=dev),
               "occ": torch.empty((natoms, nc), dtype=torch.float64, device=dev),
               "e_u": torch.empty(natoms, dtype=torch.float64, device=dev)}
        eps, U, mu = eps.contiguous(), U.contiguous(), mu.contiguous()
        check(self.h, self.lib.dmft_hubbard1(self.h, int(natoms), int(nc), _ptr(eps), _ptr(U), _ptr(mu),
                                             float(beta), float(wtol), _ptr(out["sigma_inf"]), _ptr(out["npoles"]),
                                             _ptr(out["pos"]), _ptr(out["wgt"]), _ptr(out["occ"]), _ptr(out["e_u"]),
                                             _stream(self.device)))
        return out

    def hubbard1_poles(self, h1, atom: int, nc_lat: int, a0: int = 0):
        """(p [np], v [np, nc_lat]) of one atom's self-energy poles in the layout of
        PoleSelfEnergy (orbital a of the atom is correlated orbital a0 + a)."""
        nc = h1["npoles"].shape[1]
        p = torch.zeros(max(nc * (nc - 1), 1), dtype=torch.float64, device=self.device)
        v = torch.zeros((max(nc * (nc - 1), 1), nc_lat), dtype=torch.complex128, device=self.device)
        npo = torch.zeros(1, dtype=torch.int32, device=self.device)
        check(self.h, self.lib.dmft_hubbard1_poles(self.h, int(nc), int(nc_lat), int(a0),
                                                   _ptr(h1["npoles"][atom]), _ptr(h1["pos"][atom]),
                                                   _ptr(h1["wgt"][atom]), _ptr(p), _ptr(v), _ptr(npo),
                                                   _stream(self.device)))
        n = int(npo.item())
        return p[:n], v[:n]

    def sigma_from_poles(self, pol: PoleSelfEnergy, nc: int, nw: int, mu: float) -> torch.Tensor:
        """Sigma(i w_n) [nw, nc, nc] of a pole form at chemical potential mu."""
        sig = torch.empty((nw, nc, nc), dtype=torch.complex128, device=self.device)
        ps = pol.struct()
        check(self.h, self.lib.dmft_sigma_from_poles(self.h, int(nc), C.byref(ps), int(nw), float(mu), _ptr(sig),
                                                     _stream(self.device)))
        return sig

    def timing(self, enable: bool):
        """Returns (summed Dyson-kernel ms, timed launches) recorded so far."""
        ms, n = C.c_double(), C.c_int64()
        check(self.h, self.lib.dmft_timing(self.h, 1 if enable else 0, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def sync_status(self):
        ws = self._ws
        check(self.h, self.lib.dmft_sync_status(self.h, _ptr(ws) if ws is not None else None,
                                                _stream(self.device)))


def split_nk(nk_flat: torch.Tensor, lat: Lattice) -> List[torch.Tensor]:
    out, o = [], 0
    for n in lat.nb_array():
        n = int(n)
        out.append(nk_flat[o:o + n * n].reshape(n, n))
        o += n * n
    return out
