"""GPU parity of the pole-expansion route (pseudo-Hamiltonian eigensystems,
N(k) with exact and truncated occupations, the mu search from the
eigenvalues, DOS and PDOS) against the oracle.

Eigenvalues are compared directly; eigenvectors are not unique (degenerate
pole levels, phases), so they are checked through what is unique: N(k)
(a function of H_ps), the DOS and PDOS, and the completeness and
reconstruction identities sum_l u_l u_l^dag = I, sum_l u_l E_l u_l^dag = the
physical block of H_ps.

The pole positions handed to the GPU are absolute energies (as in the
pseudo-Hamiltonian of the paper); the synthetic self-energies carry them
measured from the chemical potential mu0 of each case, so the GPU gets p + mu0
and the oracle's Matsubara-route functions take the self-energy as it is at
mu0."""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle import pole
from paper_1111_2157_amd import synth
from gpu_util import RTOL, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1111_2157_amd.dyson import Context

    c = Context(0)
    yield c
    c.close()


def _no_poles():
    """Sigma = Sigma_inf (static, Hermitian) and no poles: H_ps is the band window alone."""
    wl = synth.d_shell(nk=5, nb=20, nw=24, n_narrow=6)
    s = wl.sigma
    static = np.broadcast_to(s.sigma_inf, s.sigma.shape).copy()
    return wl.lattice, dataclasses.replace(s, sigma=static, poles=[])


def _tiny():
    lat = synth.Lattice(3, 1, np.full(3, 1, np.int32), np.array([0.4, -0.2, 1.1]), np.full(3, 1.0 / 3),
                        np.exp(1j * np.array([0.1, 0.7, -0.4])))
    w = synth.matsubara(16, 10.0)
    a, p = 0.8, 0.3
    sig = synth.SelfEnergy(16, 10.0, (a / (1j * w - p))[:, None, None], None, np.array([0.25]),
                           [(p, np.array([np.sqrt(a) * np.exp(0.2j)]))])
    return lat, sig


def _ragged():
    wl = synth.batched(nk=8, nb_lo=14, nb_hi=50, nw=16, n_iter=2)
    return wl.lattices[1], wl.sigmas[1]


def _batched78():
    """Windows of 60..64 bands with 14 poles: pseudo-Hamiltonians of up to 78 rows."""
    wl = synth.batched(nk=6, nb_lo=60, nb_hi=64, nw=16, n_iter=2)
    return wl.lattices[1], wl.sigmas[1]


def _w(maker):
    def f():
        wl = maker()
        return wl.lattice, wl.sigma
    return f


CASES = {
    "plain-m17": (_w(lambda: synth.plain(nk=8, nw=32)), -2.0),
    "d-shell-m42": (_w(lambda: synth.d_shell(nk=6, nw=32)), 0.3),
    "f-shell-m62": (_w(lambda: synth.f_shell(nk=4, nw=32)), -0.4),
    "diff-m54": (_w(lambda: synth.differentiation(nk=4, nw=32)), 0.1),
    "ragged": (_ragged, 0.2),
    "batched-m78": (_batched78, 0.1),
    "no-poles": (_no_poles, 0.0),
    "tiny-m2": (_tiny, 0.1),
}


def _absolute(sig, mu0):
    return dataclasses.replace(sig, poles=[(p + mu0, v) for p, v in sig.poles])


def _gpu_eig(ctx, lat, sig_abs):
    import torch

    from paper_1111_2157_amd.dyson import Lattice, PoleSelfEnergy

    dl, dp = Lattice.from_host(lat), PoleSelfEnergy.from_host(sig_abs)
    es = ctx.pole_eig(dl, dp)
    torch.cuda.synchronize()
    ctx.sync_status()
    return dl, dp, es


@pytest.mark.parametrize("name", list(CASES))
def test_pole_eigensystem(ctx, name):
    maker, mu0 = CASES[name]
    lat, sig = maker()
    sa = _absolute(sig, mu0)
    print("pole eig", name, flush=True)
    dl, dp, es = _gpu_eig(ctx, lat, sa)
    lam = es.evals.cpu().numpy()
    u = es.evecs.cpu().numpy()
    w = es.wphys.cpu().numpy()
    wo = es.worb.cpu().numpy()
    sweeps = ctx.pole_sweeps(dl, dp)
    assert sweeps.min() >= 1 and sweeps.max() <= 30
    npl = len(sig.poles)
    for k in range(lat.nk):
        nb = int(lat.nb[k])
        m = nb + npl
        ref, _, _, _ = pole.eigensystem(lat, sa, k)
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(lam[k, :m] - ref).max() <= 1e-12 * scale, k
        assert np.all(lam[k, m:] == 0) and np.all(w[k, m:] == 0) and np.all(wo[k, m:] == 0)
        uk = u[k, :nb, :m]
        assert np.abs(u[k, nb:, :]).max(initial=0.0) == 0 and np.abs(u[k, :, m:]).max(initial=0.0) == 0
        assert np.abs(uk @ uk.conj().T - np.eye(nb)).max() <= 1e-12
        h = pole.pseudo_h(lat.eps_k(k), lat.proj_k(k), sa.sigma_inf, sa.e_dc, sa.poles)[:nb, :nb]
        assert np.abs((uk * lam[k, :m]) @ uk.conj().T - h).max() <= 1e-12 * scale
        assert np.abs(w[k, :m] - (np.abs(uk) ** 2).sum(axis=0)).max() <= 1e-13
        assert np.abs(wo[k, :m] - (np.abs(lat.proj_k(k) @ uk) ** 2).T).max() <= 1e-13
        assert abs(w[k].sum() - nb) <= 1e-11
        assert np.all(np.diff(lam[k, :m]) >= 0)


@pytest.mark.parametrize("name", list(CASES))
def test_pole_density(ctx, name):
    import torch

    from paper_1111_2157_amd.dyson import split_nk

    maker, mu0 = CASES[name]
    lat, sig = maker()
    sa = _absolute(sig, mu0)
    print("pole density", name, flush=True)
    dl, dp, es = _gpu_eig(ctx, lat, sa)
    for nw_trunc in (0, sig.nw):
        nk, sc = ctx.pole_density(dl, dp, es, mu0, nw_trunc)
        torch.cuda.synchronize()
        ctx.sync_status()
        mats = [m.cpu().numpy() for m in split_nk(nk, dl)]
        if nw_trunc == 0:
            ref = [pole.exact_density(lat.eps_k(k), lat.proj_k(k), sig.sigma_inf, sig.e_dc, sig.poles, mu0,
                                      sig.beta) for k in range(lat.nk)]
        else:
            # the Matsubara-sum oracle at the same Nw (the truncated weights make the routes agree)
            ref, _ = oracle.density(lat, sig, mu0, 2)
        for k in range(lat.nk):
            assert relerr(mats[k], ref[k]) <= RTOL, (nw_trunc, k)
        sc = sc.cpu().numpy()
        ntot = sum(lat.wk[k] * np.trace(ref[k]).real for k in range(lat.nk))
        ncor = sum(lat.wk[k] * np.trace(lat.proj_k(k) @ ref[k] @ lat.proj_k(k).conj().T).real
                   for k in range(lat.nk))
        hks = sum(lat.wk[k] * np.sum(lat.eps_k(k) * np.diag(ref[k]).real) for k in range(lat.nk))
        assert abs(sc[0] - ntot) <= RTOL * max(abs(ntot), 1.0)
        assert abs(sc[1] - ncor) <= RTOL * max(abs(ncor), 1.0)
        assert abs(sc[2] - hks) <= RTOL * max(abs(hks), 1.0)


def test_pole_truncated_equals_matsubara_route_on_gpu(ctx):
    """The two GPU routes at the same Nw: density_matrix (frequency sum) and the
    pole route with truncated weights."""
    import torch

    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy, split_nk

    wl = synth.d_shell(nk=16, nw=64)
    mu0 = 0.3
    sa = _absolute(wl.sigma, mu0)
    dl, dp, es = _gpu_eig(ctx, wl.lattice, sa)
    nk_p, sc_p = ctx.pole_density(dl, dp, es, mu0, wl.sigma.nw)
    nk_m, _, sc_m = ctx.density_matrix(dl, SelfEnergy.from_host(wl.sigma), mu0)
    torch.cuda.synchronize()
    ctx.sync_status()
    for a, b in zip(split_nk(nk_p, dl), split_nk(nk_m, dl)):
        assert relerr(a.cpu().numpy(), b.cpu().numpy()) <= RTOL
    assert relerr(sc_p.cpu().numpy(), sc_m.cpu().numpy()) <= RTOL


@pytest.mark.parametrize("name,n0", [("plain-m17", 6.0), ("d-shell-m42", 20.0), ("ragged", 18.0)])
def test_pole_find_mu(ctx, name, n0):
    from paper_1111_2157_amd.dyson import BISECT, NEWTON

    maker, mu0 = CASES[name]
    lat, sig = maker()
    sa = _absolute(sig, mu0)
    dl, dp, es = _gpu_eig(ctx, lat, sa)
    tol = 1e-10
    mu_n, pn, nn = ctx.pole_find_mu(dl, dp, es, n0, tol, NEWTON)
    mu_b, pb, nb_ = ctx.pole_find_mu(dl, dp, es, n0, tol, BISECT)
    print(name, "newton", mu_n, pn, "bisect", mu_b, pb, flush=True)
    mu_r, _, _ = pole.pole_find_mu_bisect(lat, sa, n0, 1e-12, -40.0, 40.0)
    eigs = [pole.eigensystem(lat, sa, k)[::2] for k in range(lat.nk)]
    n_at, d_at = pole.pole_ntot_and_slope(eigs, lat.wk, mu_n, sig.beta)
    assert abs(nn - n0) <= tol and abs(nb_ - n0) <= tol
    assert abs(n_at - n0) <= 2 * tol
    assert abs(mu_n - mu_r) <= 3 * tol / d_at and abs(mu_b - mu_r) <= 3 * tol / d_at
    assert pn < pb


@pytest.mark.parametrize("name", ["plain-m17", "f-shell-m62", "ragged", "no-poles"])
def test_pole_dos(ctx, name):
    import torch

    maker, mu0 = CASES[name]
    lat, sig = maker()
    sa = _absolute(sig, mu0)
    dl, dp, es = _gpu_eig(ctx, lat, sa)
    e = np.linspace(-15.0, 15.0, 301)
    for eta in (0.05, 0.5):
        d, pd = ctx.pole_dos(dl, dp, es, mu0, eta, e[0], e[-1], e.size)
        torch.cuda.synchronize()
        ctx.sync_status()
        dref, pref = pole.dos(lat, sa, mu0, eta, e)
        assert relerr(d.cpu().numpy(), dref) <= RTOL
        assert relerr(pd.cpu().numpy(), pref) <= RTOL
    d1, _ = ctx.pole_dos(dl, dp, es, mu0, 0.1, 0.5, 0.5, 1, pdos=False)
    torch.cuda.synchronize()
    assert relerr(d1.cpu().numpy(), pole.dos(lat, sa, mu0, 0.1, [0.5])[0]) <= RTOL


@pytest.mark.parametrize("which", ["d-shell", "f-shell", "batched-iterate"])
def test_pole_fullsize(ctx, which):
    """The benchmark's workloads at full size: sampled k-points against the
    oracle, completeness at every k, the mu search and the DOS against the
    oracle over all k."""
    import torch

    from paper_1111_2157_amd.dyson import NEWTON, split_nk

    if which == "batched-iterate":
        # one 14-orbital iterate of the batched workload: 4096 k, 20..64 bands, m up to 78
        wl = synth.batched()
        lat, sig, mu0 = wl.lattices[1], wl.sigmas[1], 0.0
    else:
        wl = synth.d_shell() if which == "d-shell" else synth.f_shell()
        lat, sig, mu0 = wl.lattice, wl.sigma, wl.mu
    sa = _absolute(sig, mu0)
    print("pole full", which, flush=True)
    dl, dp, es = _gpu_eig(ctx, lat, sa)
    lam = es.evals.cpu().numpy()
    w = es.wphys.cpu().numpy()
    assert np.abs(w.sum(axis=1) - lat.nb).max() <= 1e-10
    nk, sc = ctx.pole_density(dl, dp, es, mu0, 0)
    torch.cuda.synchronize()
    ctx.sync_status()
    mats = split_nk(nk, dl)
    rng = np.random.default_rng(3)
    ks = sorted({0, lat.nk - 1} | {int(x) for x in rng.integers(lat.nk, size=3)})
    for k in ks:
        ref, _, _, _ = pole.eigensystem(lat, sa, k)
        assert np.abs(lam[k, :ref.size] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
        nref = pole.exact_density(lat.eps_k(k), lat.proj_k(k), sig.sigma_inf, sig.e_dc, sig.poles, mu0, sig.beta)
        assert relerr(mats[k].cpu().numpy(), nref) <= RTOL, k
    n_tot = float(sc[0])
    mu, passes, n = ctx.pole_find_mu(dl, dp, es, n_tot + 0.5, 1e-10, NEWTON)
    eigs = [pole.eigensystem(lat, sa, k)[::2] for k in range(lat.nk)]
    n_ref, _ = pole.pole_ntot_and_slope(eigs, lat.wk, mu0, sig.beta)
    assert abs(n_tot - n_ref) <= RTOL * n_ref
    n_at, _ = pole.pole_ntot_and_slope(eigs, lat.wk, mu, sig.beta)
    assert abs(n_at - (n_tot + 0.5)) <= 1e-9
    e = np.linspace(-12.0, 12.0, 97)
    d, pd = ctx.pole_dos(dl, dp, es, mu0, 0.1, e[0], e[-1], e.size)
    torch.cuda.synchronize()
    dref, pref = pole.dos(lat, sa, mu0, 0.1, e)
    assert relerr(d.cpu().numpy(), dref) <= RTOL and relerr(pd.cpu().numpy(), pref) <= RTOL


def test_pole_errors(ctx):
    from paper_1111_2157_amd._lib import DmftError
    from paper_1111_2157_amd.dyson import Lattice, PoleSelfEnergy

    wl = synth.plain(nk=2, nb=64, nw=8)     # 64 bands + 5 + 12 poles > 80
    extra = [(0.1 * i, np.eye(wl.lattice.nc)[i % wl.lattice.nc]) for i in range(12)]
    sig = dataclasses.replace(wl.sigma, poles=list(wl.sigma.poles) + extra)
    with pytest.raises(DmftError) as e:
        ctx.pole_eig(Lattice.from_host(wl.lattice), PoleSelfEnergy.from_host(sig))
    assert e.value.name == "DMFT_EUNSUPPORTED"
    wl = synth.plain(nk=4, nw=8)
    lat = dataclasses.replace(wl.lattice, eps=wl.lattice.eps.copy())
    lat.eps[3] = np.nan
    with pytest.raises(DmftError) as e:
        _gpu_eig(ctx, lat, wl.sigma)
    assert e.value.name == "DMFT_ENONFINITE"
    ctx.sync_status()
