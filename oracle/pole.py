"""Pole-expansion route to G and N (test infrastructure only).

Sec. 3.3 of the paper (eqs. pseudo_H_k and rho_LDA+DMFT_componet_final): when
the local self-energy has the pole form of Sec. 3.2.4 eq. se_pole,

    Sigma(i w) = Sigma_inf + sum_i V_i^dag (i w - p_i)^{-1} V_i ,

the band-window resolvent is the physical block of the resolvent of an
enlarged Hermitian "pseudo-Hamiltonian".  Written relative to the chemical
potential (mu enters the physical block only, because Sigma(i w) does not move
with mu):

    Htil_k = [[ M1_k,        -W_k^dag       ],
              [ -W_k,  diag(p_i) (poles)    ]],
    M1_k   = diag(E_k) - mu + S_k^dag (Sigma_inf - diag(V_DC)) S_k,
    W_k    = rows V_i S_k  (one row per pole),

    G_k(i w) = [ (i w - Htil_k)^{-1} ]_phys = sum_l u_l u_l^dag / (i w - lam_l)
    N_k      = sum_l u_l u_l^dag n_F(lam_l)                    (exact, no frequency sum)

with Htil_k = U diag(lam) U^dag and u_l the physical (band-window) part of
column l of U.  Htil_k is the paper's H_ps(k) shifted by -mu in the physical
block, with the paper's sign of the coupling (the sign does not change the
physical block of any function of it).  The eigen-decomposition is numpy's ``eigh`` (a library
routine).  This route shares nothing with the Matsubara-sum oracle in
``dmft_oracle.c``; the tests use it to pin that oracle.

``truncated_fermi`` is the scalar that the positive-frequency sum with the
analytic 1/(iw) and 1/(iw)^2 tails gives for one level at energy lam:

    f_Nw(lam) = 1/2 - beta lam / 4 + (2/beta) sum_{n<Nw} lam^3 / (w_n^2 (w_n^2 + lam^2)),

obtained by pairing 1/(i w_n - lam) with its n -> -n-1 partner
(1/(iw - lam) + 1/(-iw - lam) = -2 lam / (w^2 + lam^2)) and adding
2 lam / w_n^2; f_Nw -> n_F(lam) as Nw -> infinity (the classic identity
n_F(lam) = 1/2 - (2/beta) sum_{n>=0} lam / (w_n^2 + lam^2) with
sum_{n>=0} 1/w_n^2 = beta^2/8).  Because the first moment of the physical
block is exactly M1_k, the truncated Matsubara density of the oracle equals
sum_l u_l u_l^dag f_Nw(lam_l) identically, at any Nw.
"""
from __future__ import annotations

import numpy as np


def fermi(x, beta):
    """n_F(x) = 1 / (exp(beta x) + 1), evaluated without overflow."""
    x = np.asarray(x, dtype=np.float64) * beta
    out = np.empty_like(x)
    pos = x > 0
    e = np.exp(-x[pos])
    out[pos] = e / (1.0 + e)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def truncated_fermi(lam, beta, nw):
    lam = np.asarray(lam, dtype=np.float64)
    w = (2.0 * np.arange(nw) + 1.0) * np.pi / beta
    l3 = lam[..., None] ** 3
    s = (l3 / (w ** 2 * (w ** 2 + lam[..., None] ** 2))).sum(axis=-1)
    return 0.5 - beta * lam / 4.0 + 2.0 * s / beta


def pseudo_hamiltonian(eps_k, proj_k, sigma_inf, e_dc, poles, mu):
    """Htil_k (see module docstring).  ``poles`` is a list of (p_i, V_i[nc])."""
    nb = eps_k.shape[0]
    nc = proj_k.shape[0]
    sinf = np.zeros((nc, nc), np.complex128) if sigma_inf is None else np.asarray(sigma_inf)
    m1 = np.diag(eps_k - mu).astype(np.complex128) + proj_k.conj().T @ (sinf - np.diag(e_dc)) @ proj_k
    npl = len(poles)
    h = np.zeros((nb + npl, nb + npl), np.complex128)
    h[:nb, :nb] = m1
    for i, (p, v) in enumerate(poles):
        row = np.asarray(v, np.complex128) @ proj_k        # V_i S_k : 1 x nb
        h[nb + i, :nb] = -row
        h[:nb, nb + i] = -row.conj()
        h[nb + i, nb + i] = p
    return h


def _phys_eig(eps_k, proj_k, sigma_inf, e_dc, poles, mu):
    h = pseudo_hamiltonian(eps_k, proj_k, sigma_inf, e_dc, poles, mu)
    lam, u = np.linalg.eigh(h)
    return lam, u[:eps_k.shape[0], :]


def exact_density(eps_k, proj_k, sigma_inf, e_dc, poles, mu, beta):
    """N_k = sum_l u_l u_l^dag n_F(lam_l): the paper's exact pole-route density."""
    lam, up = _phys_eig(eps_k, proj_k, sigma_inf, e_dc, poles, mu)
    return (up * fermi(lam, beta)) @ up.conj().T


def truncated_density(eps_k, proj_k, sigma_inf, e_dc, poles, mu, beta, nw):
    """sum_l u_l u_l^dag f_Nw(lam_l): what the positive-frequency Matsubara sum
    with the analytic tail must return at finite Nw."""
    lam, up = _phys_eig(eps_k, proj_k, sigma_inf, e_dc, poles, mu)
    return (up * truncated_fermi(lam, beta, nw)) @ up.conj().T


def exact_green(eps_k, proj_k, sigma_inf, e_dc, poles, mu, iw):
    """G_k(i w) = sum_l u_l u_l^dag / (i w - lam_l)."""
    lam, up = _phys_eig(eps_k, proj_k, sigma_inf, e_dc, poles, mu)
    return (up / (iw - lam)) @ up.conj().T


def exact_ntot(lat, sig, mu):
    """sum_k w_k tr N_k from the pole route (Sec. 3.3 eq. fix_mu)."""
    tot = 0.0
    for k in range(lat.nk):
        n = exact_density(lat.eps_k(k), lat.proj_k(k), sig.sigma_inf, sig.e_dc, sig.poles, mu, sig.beta)
        tot += lat.wk[k] * np.trace(n).real
    return tot


# --------------------------------------------------------------------------
# Eigensystems, chemical potential and DOS / PDOS of the pole route
# (Sec. 3.3 eqs. pseudo_H_k and fix_mu; Sec. 3.5.2 eqs. DOS and PDOS).

def pseudo_h(eps_k, proj_k, sigma_inf, e_dc, poles):
    """The paper's H_ps(k) (no chemical potential): its eigenvalues are E^ps_l(k).
    Here the pole positions are absolute energies, as eq. rho_LDA+DMFT_componet_final
    has them (occupations n_F(E^ps - mu)); the Matsubara-axis self-energy at a
    chemical potential mu then has its poles at p_i - mu, which is what the
    functions above take."""
    return pseudo_hamiltonian(eps_k, proj_k, sigma_inf, e_dc, poles, 0.0)


def eigensystem(lat, sig, k):
    """(E^ps ascending [m], u = <phi_n|psi_l> [nb, m], |u_l|^2 [m], |S_alpha u_l|^2 [m, nc]) for one k."""
    p = lat.proj_k(k)
    lam, vec = np.linalg.eigh(pseudo_h(lat.eps_k(k), p, sig.sigma_inf, sig.e_dc, sig.poles))
    u = vec[:p.shape[1], :]
    return lam, u, (np.abs(u) ** 2).sum(axis=0), (np.abs(p @ u) ** 2).T


def pole_ntot_and_slope(eigs, wk, mu, beta):
    """N_tot(mu) = sum_k w_k sum_l |u_l|^2 n_F(E^ps_l - mu) (eq. fix_mu) and its mu-derivative,
    from a list of per-k (E^ps, |u|^2)."""
    n = d = 0.0
    for (lam, w), wkk in zip(eigs, wk):
        f = fermi(lam - mu, beta)
        n += wkk * np.sum(w * f)
        d += wkk * np.sum(w * beta * f * (1.0 - f))
    return n, d


def pole_find_mu_bisect(lat, sig, n_target, tol, lo, hi, max_iter=200):
    """Plain bisection on N_tot(mu) of the pole route; returns (mu, evaluations, N)."""
    eigs = []
    for k in range(lat.nk):
        lam, _, w, _ = eigensystem(lat, sig, k)
        eigs.append((lam, w))
    mu = n = 0.0
    for it in range(max_iter):
        mu = 0.5 * (lo + hi)
        n, _ = pole_ntot_and_slope(eigs, lat.wk, mu, sig.beta)
        if abs(n - n_target) <= tol:
            return mu, it + 1, n
        if n < n_target:
            lo = mu
        else:
            hi = mu
    raise RuntimeError("no convergence")


def dos(lat, sig, mu, eta, energies):
    """D(e) and D_alpha(e) (eqs. DOS, PDOS) with the eta -> 0+ limit taken at a finite
    Lorentzian half-width eta: -(1/pi) Im 1/(x + i eta) = (eta/pi) / (x^2 + eta^2),
    x = e + mu - E^ps_l, k-sum with the weights w_k.  Returns ([ne], [ne, nc])."""
    e = np.asarray(energies, np.float64)
    d = np.zeros(e.shape)
    pd = np.zeros(e.shape + (int(lat.nc),))
    for k in range(lat.nk):
        lam, _, w, wo = eigensystem(lat, sig, k)
        x = e[:, None] + mu - lam[None, :]
        lor = (eta / np.pi) / (x * x + eta * eta)
        d += lat.wk[k] * lor @ w
        pd += lat.wk[k] * lor @ wo
    return d, pd


def energy_terms(lat, sig, mu):
    """Pole-route sums of the energy functional (Sec. 3.5.1 eqs. H_KS, H_U_energy
    and <V_DC>), with E^ps absolute (reading of eq. pseudo_H_k above):
        B      = sum_k w_k sum_m E^ps_m |u_m|^2 n_F(E^ps_m - mu)
        N_tot  = sum_k w_k sum_m |u_m|^2 n_F(E^ps_m - mu)
        H_KS   = sum_k w_k sum_n E_n N_nn                      (eq. H_KS)
        n_a    = sum_k w_k sum_m |S_a u_m|^2 n_F(E^ps_m - mu)  (correlated occupations)
        V_DC   = sum_a V_DC,a n_a                              (eq. <V_DC> for this V_DC)
        H_U    = (B - H_KS + V_DC) / 2.
    H_U is the Galitskii-Migdal value (1/2) tr[Sigma G]: the derivation through
    G^-1 = i w + mu - H_KS + V_DC - Sigma gives sum_m (E^ps_m - mu) ... + mu N_tot,
    i.e. B with the absolute E^ps (the printed eq. H_U_energy omits mu N_tot).
    Returns a dict."""
    B = N = hks = 0.0
    na = np.zeros(int(lat.nc))
    for k in range(lat.nk):
        lam, u, w, wo = eigensystem(lat, sig, k)
        f = fermi(lam - mu, sig.beta)
        wk = lat.wk[k]
        B += wk * np.sum(lam * w * f)
        N += wk * np.sum(w * f)
        hks += wk * np.sum(lat.eps_k(k) * ((np.abs(u) ** 2) @ f))
        na += wk * (wo.T @ f)
    vdc = float(np.dot(np.asarray(sig.e_dc, np.float64), na))
    return {"band": B, "n_tot": N, "h_ks": hks, "n_orb": na, "v_dc": vdc, "h_u": 0.5 * (B - hks + vdc)}
