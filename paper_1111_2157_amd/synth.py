"""Seeded synthetic inputs for the lattice Dyson step.

This module only *draws inputs*: band energies, projectors, a pole-form local
self-energy tabulated on the Matsubara grid, double-counting shifts and k
weights.  It holds none of the Dyson-step arithmetic (no inversion,
projection, frequency sum or chemical-potential search); both the GPU path and
the CPU oracle are fed from here.

The paper's own workloads (gamma-Ce, Am, NiO, Sec. 4) need a plane-wave DFT
code, pseudopotentials and projected Wannier orbitals that are not available,
so these seeded inputs stand in for them with the same shapes:

* ``E_vk`` band energies in a band window (Sec. 3.1 eq. H_LDA; the window of
  Sec. 2 eq. 3 gives the per-k window size ``nb_k``);
* ``S_k`` projectors with orthonormal rows, made by the Loewdin step
  ``O^{-1/2}`` of Sec. 2 eqs. 6-7 applied to complex Gaussian trial overlaps,
  so that sum_n |S_{alpha n}|^2 = 1 (Sec. 3.1 eq. S_norm);
* ``Sigma(i w_n)`` in the pole form of Sec. 3.2.4 eq. se_pole: the
  single-orbital Hubbard-I self-energy U^2 n(1-n) / (i w - e0 - U(1-n)) on the
  diagonal (the appendix's pole fit of the two-pole atomic Green's function)
  plus, for the multi-orbital cases, a static Hermitian off-diagonal part that
  is also the self-energy's infinite-frequency limit;
* ``V_DC = Ubar (n0 - 1/2)`` with an integer shell occupancy n0
  (Sec. 3.2.3 eqs. V_DC, V_DC_component and the integer choice for
  Hubbard-I) and Ubar = U at J = 0.

Draw order with ``numpy.random.default_rng(seed)``: band energies first (for
mixtures the narrow block, then the broad block), then the real and then the
imaginary parts of the trial overlaps, then the off-diagonal phases.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np


@dataclass
class Lattice:
    """Band window and projectors of every k-point (ragged over k)."""

    nk: int
    nc: int
    nb: np.ndarray      # int32 [nk]
    eps: np.ndarray     # float64, sum(nb): E_vk of all k, k-major
    wk: np.ndarray      # float64 [nk], sums to 1
    proj: np.ndarray    # complex128, sum(nc*nb): S_k (nc x nb_k, row-major), k-major

    @property
    def nb_max(self) -> int:
        return int(self.nb.max())

    @property
    def uniform(self) -> bool:
        return bool((self.nb == self.nb[0]).all())

    def off_b(self) -> np.ndarray:
        o = np.zeros(self.nk + 1, np.int64)
        o[1:] = np.cumsum(self.nb)
        return o

    def eps_k(self, k: int) -> np.ndarray:
        o = self.off_b()
        return self.eps[o[k]:o[k + 1]]

    def proj_k(self, k: int) -> np.ndarray:
        o = self.off_b() * self.nc
        return self.proj[o[k]:o[k + 1]].reshape(self.nc, int(self.nb[k]))

    def subset(self, ks) -> "Lattice":
        """The same band structure restricted to the k-points ``ks`` (weights kept)."""
        ks = np.asarray(ks)
        return Lattice(len(ks), self.nc, self.nb[ks].astype(np.int32).copy(),
                       np.concatenate([self.eps_k(k) for k in ks]), self.wk[ks].copy(),
                       np.concatenate([self.proj_k(k).ravel() for k in ks]))


@dataclass
class SelfEnergy:
    """Local self-energy on the positive Matsubara grid and its pole form."""

    nw: int
    beta: float
    sigma: np.ndarray                 # complex128 [nw, nc, nc]
    sigma_inf: Optional[np.ndarray]   # complex128 [nc, nc] or None
    e_dc: np.ndarray                  # float64 [nc]
    # pole form Sigma = Sigma_inf + sum_i V_i^dag V_i / (i w - p_i): list of (p_i, V_i[nc])
    poles: List[Tuple[float, np.ndarray]] = field(default_factory=list)

    @property
    def nc(self) -> int:
        return int(self.e_dc.shape[0])


@dataclass
class Workload:
    name: str
    lattice: Lattice
    sigmas: List[SelfEnergy]          # one per iterate (a single one except the batched case)
    mu: float = 0.0
    n_target: Optional[float] = None
    lattices: Optional[List[Lattice]] = None   # per-iterate lattices (batched case)
    meta: dict = field(default_factory=dict)

    @property
    def sigma(self) -> SelfEnergy:
        return self.sigmas[0]


# --------------------------------------------------------------------------- draws

def loewdin_rows(z: np.ndarray) -> np.ndarray:
    """O^{-1/2} Z with O = Z Z^dag: rows become orthonormal (Sec. 2 eqs. 6-7)."""
    o = z @ z.conj().T
    w, v = np.linalg.eigh(o)
    return (v * (1.0 / np.sqrt(w))) @ v.conj().T @ z


def _projectors(rng, nk, nc, nb_full, nb_k=None):
    x = rng.standard_normal((nk, nc, nb_full))
    y = rng.standard_normal((nk, nc, nb_full))
    if (nb_full if nb_k is None else int(np.min(nb_k))) < nc:
        raise ValueError("every band window must hold at least nc bands")
    out = []
    for k in range(nk):
        nb = nb_full if nb_k is None else int(nb_k[k])
        z = (x[k, :, :nb] + 1j * y[k, :, :nb]) / np.sqrt(2.0)
        out.append(loewdin_rows(z))
    return out


def hubbard1_pole(U: float, n: float, e0: float = 0.0) -> Tuple[float, float]:
    """(weight a, pole p) of the single-orbital Hubbard-I self-energy
    a / (i w - p) with a = U^2 n (1-n), p = e0 + U (1-n)."""
    return U * U * n * (1.0 - n), e0 + U * (1.0 - n)


def matsubara(nw: int, beta: float) -> np.ndarray:
    """Fermionic grid w_n = (2n+1) pi / beta, n = 0 .. nw-1 (input tabulation only)."""
    return (2.0 * np.arange(nw) + 1.0) * np.pi / beta


def hermitian_offdiag(rng, nc: int, amp: float, blocks=None) -> np.ndarray:
    """Static Hermitian matrix with zero diagonal and |H_ab| = amp, random phases,
    restricted to the diagonal site blocks given as (start, size) pairs."""
    h = np.zeros((nc, nc), np.complex128)
    blocks = blocks or [(0, nc)]
    for s0, sz in blocks:
        for a in range(s0, s0 + sz):
            for b in range(a + 1, s0 + sz):
                phi = rng.uniform(0.0, 1.0)
                h[a, b] = amp * np.exp(2j * np.pi * phi)
                h[b, a] = np.conj(h[a, b])
    return h


def pole_sigma(nw, beta, nc, a, p, e_dc, h_static=None) -> SelfEnergy:
    """Sigma(i w_n) = a/(i w_n - p) I + H_static, Sigma_inf = H_static."""
    w = matsubara(nw, beta)
    sig = np.zeros((nw, nc, nc), np.complex128)
    diag = a / (1j * w - p)
    idx = np.arange(nc)
    sig[:, idx, idx] = diag[:, None]
    sinf = None
    if h_static is not None:
        sig += h_static[None, :, :]
        sinf = h_static.copy()
    poles = [(p, np.sqrt(a) * np.eye(nc)[al]) for al in range(nc)]
    return SelfEnergy(nw, float(beta), sig, sinf, np.full(nc, float(e_dc)), poles)


def _lattice(nk, nc, nb_k, eps_rows, projs):
    nb = np.asarray(nb_k, np.int32)
    return Lattice(nk, nc, nb, np.concatenate(eps_rows).astype(np.float64),
                   np.full(nk, 1.0 / nk), np.concatenate([p.ravel() for p in projs]))


def _dc(U: float, n: float, nc_site: int) -> float:
    """V_DC = U (n0 - 1/2) with n0 the integer occupancy of one site's shell."""
    n0 = int(round(nc_site * n))
    return U * (n0 - 0.5)


# --------------------------------------------------------------------------- configs

def plain(seed=0, nk=64, nb=12, nc=5, nw=256, beta=20.0, U=6.0, n=0.4, e0=0.0, n_target=6.0):
    """Plain method at oracle size: eps ~ U[-6,6], diagonal Hubbard-I Sigma."""
    rng = np.random.default_rng(seed)
    eps = rng.uniform(-6.0, 6.0, (nk, nb))
    projs = _projectors(rng, nk, nc, nb)
    lat = _lattice(nk, nc, [nb] * nk, list(eps), projs)
    a, p = hubbard1_pole(U, n, e0)
    sig = pole_sigma(nw, beta, nc, a, p, _dc(U, n, nc))
    return Workload("plain-Nk%d-Nb%d-Nc%d-Nw%d" % (nk, nb, nc, nw), lat, [sig], mu=0.0,
                    n_target=n_target, meta=dict(U=U, n=n, e0=e0))


def _mixture(rng, nk, n_narrow, n_broad, width=1.0, lo=-10.0, hi=10.0):
    narrow = rng.normal(0.0, width, (nk, n_narrow))
    broad = rng.uniform(lo, hi, (nk, n_broad))
    return narrow, broad


def d_shell(seed=0, nk=512, nb=32, nc=10, nw=1024, beta=40.0, U=6.0, n=0.4, e0=0.0, n_narrow=10):
    """Two 5-orbital d sites, block-diagonal Sigma, narrow+broad band mixture."""
    rng = np.random.default_rng(seed)
    narrow, broad = _mixture(rng, nk, n_narrow, nb - n_narrow)
    eps = np.hstack([narrow, broad])
    projs = _projectors(rng, nk, nc, nb)
    lat = _lattice(nk, nc, [nb] * nk, list(eps), projs)
    site = 5
    h = hermitian_offdiag(rng, nc, 0.1, [(s, site) for s in range(0, nc, site)])
    a, p = hubbard1_pole(U, n, e0)
    sig = pole_sigma(nw, beta, nc, a, p, _dc(U, n, site), h)
    return Workload("d-shell-Nk%d-Nb%d-Nc%d-Nw%d" % (nk, nb, nc, nw), lat, [sig], mu=0.0,
                    meta=dict(U=U, n=n, e0=e0))


def f_shell(seed=0, nk=2048, nb=48, nc=14, nw=4096, beta=100.0, U=5.0, n=1.0 / 14, e0=0.0,
            n_narrow=14, n_target=None, name="f-shell"):
    """One 14-orbital f site with spin-orbit-like static off-diagonals (0.1 eV)."""
    rng = np.random.default_rng(seed)
    narrow, broad = _mixture(rng, nk, n_narrow, nb - n_narrow)
    eps = np.hstack([narrow, broad])
    projs = _projectors(rng, nk, nc, nb)
    lat = _lattice(nk, nc, [nb] * nk, list(eps), projs)
    h = hermitian_offdiag(rng, nc, 0.1)
    a, p = hubbard1_pole(U, n, e0)
    sig = pole_sigma(nw, beta, nc, a, p, _dc(U, n, nc), h)
    return Workload("%s-Nk%d-Nb%d-Nc%d-Nw%d" % (name, nk, nb, nc, nw), lat, [sig], mu=0.0,
                    n_target=n_target, meta=dict(U=U, n=n, e0=e0))


def differentiation(seed=0, nk=1024, nb=40, nc=14, nw=2048, beta=50.0, n_target=20.0):
    """The f-shell parameters at Nb=40 with an electron-count target for the mu search."""
    return f_shell(seed=seed, nk=nk, nb=nb, nc=nc, nw=nw, beta=beta, n_target=n_target,
                   name="diff")


def batched(seed=0, nk=4096, nb_lo=20, nb_hi=64, nw=2048, beta=40.0, n_iter=8, n_narrow=14):
    """Uneven band windows nb_k ~ U{nb_lo..nb_hi}; n_iter self-energy iterates that
    alternate between a 5-orbital (d) and a 14-orbital (f) correlated shell on one
    shared band structure."""
    rng = np.random.default_rng(seed)
    nb_k = rng.integers(nb_lo, nb_hi + 1, nk)
    narrow = rng.normal(0.0, 1.0, (nk, n_narrow))
    broad = rng.uniform(-10.0, 10.0, (nk, nb_hi - n_narrow))
    eps_rows = [np.concatenate([narrow[k], broad[k, :nb_k[k] - n_narrow]]) for k in range(nk)]
    proj5 = _projectors(rng, nk, 5, nb_hi, nb_k)
    proj14 = _projectors(rng, nk, 14, nb_hi, nb_k)
    lat5 = _lattice(nk, 5, nb_k, eps_rows, proj5)
    lat14 = _lattice(nk, 14, nb_k, eps_rows, proj14)
    d_ns = [0.3, 0.35, 0.4, 0.45]
    f_ns = [1.0 / 14, 2.0 / 14, 3.0 / 14, 4.0 / 14]
    sigmas, lats = [], []
    for s in range(n_iter):
        if s % 2 == 0:
            U, n = 6.0, d_ns[(s // 2) % 4]
            a, p = hubbard1_pole(U, n)
            sigmas.append(pole_sigma(nw, beta, 5, a, p, _dc(U, n, 5)))
            lats.append(lat5)
        else:
            U, n = 5.0, f_ns[(s // 2) % 4]
            h = hermitian_offdiag(rng, 14, 0.1)
            a, p = hubbard1_pole(U, n)
            sigmas.append(pole_sigma(nw, beta, 14, a, p, _dc(U, n, 14), h))
            lats.append(lat14)
    return Workload("batched-Nk%d-Nb%d..%d-x%d-Nw%d" % (nk, nb_lo, nb_hi, n_iter, nw), lat5, sigmas,
                    mu=0.0, lattices=lats)


CONFIGS = {
    "plain": plain,
    "d-shell": d_shell,
    "f-shell": f_shell,
    "batched": batched,
    "diff": differentiation,
}
