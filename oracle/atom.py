"""Hubbard-I atom and the pole form of its self-energy (test infrastructure only).

Sec. 3.2.4 eqs. Dyson and G_imp_atom, and the appendix (eq. dyson_pole): the
atomic Green's function from exact diagonalisation of one atom, and its
self-energy Sigma(i w) = i w + mu - e_imp - G(i w)^-1 in pole form.

Interaction: H_U = (U/2) sum_{a != b} n_a n_b over the atom's nc spin-orbitals
(the eq. H_U of Sec. 3.2.3 with J = 0, so U_bar = U), one-body levels e_a (the
diagonal of E_imp), energies measured from the chemical potential mu:
    E(Gamma) = sum_{a in Gamma} (e_a - mu) + U N (N - 1) / 2,  X = exp(-beta E) / Z.
Every Fock state is an eigenstate, and <Gamma|f_a|Gamma'> is nonzero only for
Gamma' = Gamma + a, so eq. G_imp_atom gives a diagonal G with poles at
    P_N = e_a - mu + U N   (N = electrons on the other orbitals of Gamma),
    V_N = sum over Gamma without a and with N electrons of X(Gamma) + X(Gamma + a).
Appendix: Sigma(inf) = mu - e_a + sum_N V_N P_N; the self-energy poles Q are
the zeros of sum_N V_N / (Q - P_N), one between each two adjacent poles
(found by bisection), with weights W = [sum_N V_N / (Q - P_N)^2]^-1.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this module; it shares nothing with the product library.
"""
from __future__ import annotations

import numpy as np


def fock_states(nc):
    """All 2^nc occupation patterns as a [2^nc, nc] 0/1 array (bit a of the index)."""
    idx = np.arange(1 << nc)
    return ((idx[:, None] >> np.arange(nc)[None, :]) & 1).astype(np.int64)


def atom_energies(eps, U, mu):
    """E(Gamma) for every Fock state (index = occupation bit pattern)."""
    eps = np.asarray(eps, np.float64)
    occ = fock_states(eps.size)
    n = occ.sum(axis=1)
    return occ @ (eps - mu) + U * n * (n - 1) / 2.0, occ


def boltzmann(E, beta):
    x = np.exp(-beta * (E - E.min()))
    return x / x.sum()


def green_poles(eps, U, mu, beta):
    """(P [nc, nc], V [nc, nc]): G_aa(i w) = sum_N V[a, N] / (i w - P[a, N])."""
    eps = np.asarray(eps, np.float64)
    nc = eps.size
    E, occ = atom_energies(eps, U, mu)
    X = boltzmann(E, beta)
    n = occ.sum(axis=1)
    idx = np.arange(1 << nc)
    P = np.zeros((nc, nc))
    V = np.zeros((nc, nc))
    for a in range(nc):
        P[a] = eps[a] - mu + U * np.arange(nc)
        empty = occ[:, a] == 0                      # Gamma without a; Gamma + a = index | bit a
        V[a] = np.bincount(n[empty], weights=X[empty] + X[idx[empty] | (1 << a)], minlength=nc)[:nc]
    return P, V


def pole_fit(P, V, e_imp, mu, wtol=0.0):
    """Appendix: (Q, W, Sigma_inf) of Sigma = Sigma_inf + sum W / (i w - Q) for one
    orbital from G = sum V / (i w - P).  Poles with V <= wtol are dropped and the
    rest renormalised to unit total weight: a pole of weight V has its
    self-energy neighbour within about V of it, which double precision cannot
    resolve below V ~ 1e-16, and it changes G by about V."""
    keep = V > wtol
    p = np.asarray(P, np.float64)[keep]
    v = np.asarray(V, np.float64)[keep]
    order = np.argsort(p)
    p, v = p[order], v[order]
    v = v / v.sum()
    sinf = mu - e_imp + np.sum(v * p)
    Q, W = [], []
    for i in range(p.size - 1):
        lo, hi = p[i], p[i + 1]
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid <= lo or mid >= hi:
                break
            if np.sum(v / (mid - p)) > 0.0:   # decreasing from +inf to -inf between the poles
                lo = mid
            else:
                hi = mid
        q = 0.5 * (lo + hi)
        Q.append(q)
        W.append(1.0 / np.sum(v / (q - p) ** 2))
    return np.array(Q), np.array(W), sinf


def hubbard1_sigma(eps, U, mu, beta, wtol=1e-13):
    """Per orbital a: (Q_a, W_a, Sigma_inf_a) of the Hubbard-I self-energy."""
    P, V = green_poles(eps, U, mu, beta)
    return [pole_fit(P[a], V[a], float(eps[a]), mu, wtol) for a in range(len(eps))]


def interaction_energy(eps, U, mu, beta):
    """(<H_U>, <n_a>) of the atom in its grand-canonical ensemble."""
    E, occ = atom_energies(eps, U, mu)
    X = boltzmann(E, beta)
    n = occ.sum(axis=1)
    return float(np.sum(X * U * n * (n - 1) / 2.0)), X @ occ
