"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Sizes here finish in seconds on the oracle and still span several 16x16 tiles,
padded band windows and ragged k; full-size workloads are checked on sampled
k-points and frequencies in test_gpu_fullsize.py.
"""
import numpy as np
import pytest

import oracle
from paper_1111_2157_amd import synth
from gpu_util import RTOL, assert_gloc_parity, assert_nk_parity, gpu_density, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1111_2157_amd.dyson import Context

    c = Context(0)
    yield c
    c.close()


CASES = {
    # name: (maker, mu)
    "plain-full": (lambda: synth.plain(), -2.0),
    "d-shell-small": (lambda: synth.d_shell(nk=24, nw=96), 0.3),
    "f-shell-small": (lambda: synth.f_shell(nk=10, nw=48), -0.4),
    "diff-nb40-small": (lambda: synth.differentiation(nk=10, nw=40), 0.1),
    "nb19-pad": (lambda: synth.f_shell(nk=6, nb=19, nc=14, nw=40, n_narrow=5), 0.2),
    "nb16-nc16": (lambda: synth.f_shell(nk=6, nb=16, nc=16, nw=36, n_narrow=5), 0.0),
    "nb33-nc1": (lambda: synth.plain(nk=5, nb=33, nc=1, nw=30), 0.5),
    "nb64-f": (lambda: synth.f_shell(nk=5, nb=64, nw=24), -0.2),
    "nb57-d": (lambda: synth.d_shell(nk=4, nb=57, nw=20), 0.3),
}


@pytest.mark.parametrize("name", list(CASES))
def test_density_and_gloc_parity(ctx, name):
    maker, mu = CASES[name]
    wl = maker()
    print("case", name, flush=True)
    mats, gl, sc = gpu_density(ctx, wl, mu)
    assert_nk_parity(mats, wl.lattice, wl.sigma, mu)
    assert_gloc_parity(gl, wl.lattice, wl.sigma, mu)
    lat = wl.lattice
    ntot = sum(lat.wk[k] * np.trace(m).real for k, m in enumerate(mats))
    ref_n, _ = oracle.trace(lat, wl.sigma, mu)
    assert abs(sc[0] - ref_n) <= RTOL * abs(ref_n)
    assert abs(sc[0] - ntot) <= 1e-12 * abs(ntot)
    ncor = sum(lat.wk[k] * np.trace(lat.proj_k(k) @ m @ lat.proj_k(k).conj().T).real for k, m in enumerate(mats))
    hks = sum(lat.wk[k] * np.dot(lat.eps_k(k), np.diag(m).real) for k, m in enumerate(mats))
    assert abs(sc[1] - ncor) <= 1e-11 * max(1.0, abs(ncor))
    assert abs(sc[2] - hks) <= 1e-11 * max(1.0, abs(hks))


def test_tail_order_zero(ctx):
    wl = synth.d_shell(nk=8, nw=64)
    mats, gl, sc = gpu_density(ctx, wl, 0.1, tail=0)
    assert_nk_parity(mats, wl.lattice, wl.sigma, 0.1, tail=0)


def test_ragged_windows(ctx):
    wl = synth.batched(nk=24, nb_lo=14, nb_hi=64, nw=40, n_iter=2)
    for s in range(2):
        lat = wl.lattices[s]
        assert len(set(lat.nb.tolist())) > 5
        mats, gl, sc = gpu_density(ctx, wl, 0.2, sig_index=s)
        assert_nk_parity(mats, lat, wl.sigmas[s], 0.2)
        assert_gloc_parity(gl, lat, wl.sigmas[s], 0.2)


def test_ntot_trace_pass(ctx):
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    for wl, mu in ((synth.plain(), -2.1), (synth.f_shell(nk=8, nw=48), 0.3),
                   (synth.batched(nk=12, nb_lo=14, nb_hi=64, nw=32, n_iter=1), 0.0),
                   (synth.f_shell(nk=3, nb=64, nw=20), 0.1)):
        out = ctx.dmft_ntot(Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma), mu).cpu().numpy()
        ctx.sync_status()
        n, d = oracle.trace(wl.lattice, wl.sigma, mu)
        assert abs(out[0] - n) <= RTOL * abs(n)
        assert abs(out[1] - d) <= RTOL * abs(d)


def test_gloc_compute_entry(ctx):
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = synth.d_shell(nk=8, nw=40)
    gl = ctx.gloc_compute(Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma), 0.0).cpu().numpy()
    ctx.sync_status()
    assert_gloc_parity(gl, wl.lattice, wl.sigma, 0.0)


def test_bitwise_deterministic(ctx):
    wl = synth.d_shell(nk=16, nw=64)
    a = gpu_density(ctx, wl, 0.0)
    b = gpu_density(ctx, wl, 0.0)
    for x, y in zip(a[0], b[0]):
        assert np.array_equal(x, y)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("method", ["newton", "bisect"])
def test_find_mu_parity(ctx, method):
    from paper_1111_2157_amd.dyson import BISECT, NEWTON, Lattice, SelfEnergy

    wl = synth.plain()
    lat, sig = wl.lattice, wl.sigma
    tol = 1e-12
    mu_ref, _, _ = oracle.find_mu_bisect(lat, sig, 6.0, tol, -40.0, 40.0, max_iter=300)
    mu, passes, n = ctx.find_mu(Lattice.from_host(lat), SelfEnergy.from_host(sig), 6.0, tol,
                                NEWTON if method == "newton" else BISECT, -40.0, 40.0, max_iter=300)
    assert abs(n - 6.0) <= tol
    _, d = oracle.trace(lat, sig, mu)
    assert d > 1e-2
    assert abs(mu - mu_ref) <= 1e-10 * max(1.0, abs(mu_ref))


def test_newton_fewer_passes_than_bisection(ctx):
    from paper_1111_2157_amd.dyson import BISECT, NEWTON, Lattice, SelfEnergy

    wl = synth.plain()
    dl, ds = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
    _, pn, nn = ctx.find_mu(dl, ds, 6.0, 1e-8, NEWTON, -40.0, 40.0)
    _, pb, nb = ctx.find_mu(dl, ds, 6.0, 1e-8, BISECT, -40.0, 40.0)
    assert abs(nn - 6.0) <= 1e-8 and abs(nb - 6.0) <= 1e-8
    assert pn * 3 <= pb, (pn, pb)


def test_nonfinite_sigma_is_reported(ctx):
    from paper_1111_2157_amd._lib import DmftError
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = synth.plain(nk=4, nw=16)
    sig = wl.sigma
    bad = sig.sigma.copy()
    bad[3, 1, 1] = np.nan
    s2 = synth.SelfEnergy(sig.nw, sig.beta, bad, sig.sigma_inf, sig.e_dc)
    ctx.density_matrix(Lattice.from_host(wl.lattice), SelfEnergy.from_host(s2), 0.0)
    with pytest.raises(DmftError) as e:
        ctx.sync_status()
    assert e.value.name == "DMFT_ENONFINITE"
    ctx.sync_status()  # the error word was cleared


def test_invalid_arguments_rejected_before_launch(ctx):
    from paper_1111_2157_amd._lib import DmftError
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = synth.plain(nk=4, nw=16)
    dl, ds = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
    with pytest.raises(DmftError) as e:
        ctx.density_matrix(dl, ds, 0.0, tail_order=1)
    assert e.value.name == "DMFT_EINVAL"
    ds.beta = -1.0
    with pytest.raises(DmftError) as e:
        ctx.density_matrix(dl, ds, 0.0)
    assert e.value.name == "DMFT_EINVAL"


def test_autotune_then_parity(ctx):
    from paper_1111_2157_amd.dyson import Context, Lattice, SelfEnergy

    c = Context(0)
    wl = synth.d_shell(nk=32, nw=128)
    dl, ds = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
    rep = c.autotune(dl, ds, 0.1)
    assert "best density" in rep and "best trace" in rep
    assert "rejected" not in rep, rep
    mats, gl, sc = gpu_density(c, wl, 0.1)
    assert_nk_parity(mats, wl.lattice, wl.sigma, 0.1)
    assert_gloc_parity(gl, wl.lattice, wl.sigma, 0.1)
    out = c.dmft_ntot(dl, ds, 0.1).cpu().numpy()
    n, d = oracle.trace(wl.lattice, wl.sigma, 0.1)
    assert abs(out[0] - n) <= RTOL * abs(n) and abs(out[1] - d) <= RTOL * abs(d)
    c.close()


VARIANT_CASES = [(16, lambda: synth.plain(nk=6, nw=40), -1.0), (32, lambda: synth.d_shell(nk=8, nw=40), 0.0),
                 (48, lambda: synth.f_shell(nk=6, nw=32), 0.1), (64, lambda: synth.f_shell(nk=3, nb=64, nw=20), 0.0)]


@pytest.mark.parametrize("nbp,maker,mu", VARIANT_CASES)
def test_every_kernel_variant_matches_oracle(nbp, maker, mu):
    from paper_1111_2157_amd.dyson import Context, Lattice, SelfEnergy

    wl = maker()
    c = Context(0)
    dl, ds = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
    n_ref, d_ref = oracle.trace(wl.lattice, wl.sigma, mu)
    for var in c.variants(0, nbp):
        print("density variant", nbp, var, flush=True)
        c.set_variant(0, nbp, var)
        mats, gl, sc = gpu_density(c, wl, mu)
        assert_nk_parity(mats, wl.lattice, wl.sigma, mu)
        assert_gloc_parity(gl, wl.lattice, wl.sigma, mu)
    for var in c.variants(1, nbp):
        print("trace variant", nbp, var, flush=True)
        c.set_variant(1, nbp, var)
        out = c.dmft_ntot(dl, ds, mu).cpu().numpy()
        c.sync_status()
        assert abs(out[0] - n_ref) <= RTOL * abs(n_ref) and abs(out[1] - d_ref) <= RTOL * abs(d_ref)
    c.close()


def test_tail_order_zero_trace_vjp_and_mu(ctx):
    """dmft_ntot, density_matrix_vjp and find_mu without the analytic tail
    against the oracle's tail-free sums (pinned on the CPU against the
    spectral closed forms)."""
    import torch

    from paper_1111_2157_amd.dyson import BISECT, NEWTON, Lattice, SelfEnergy

    wl = synth.f_shell(nk=8, nb=20, nc=14, nw=48, beta=15.0, n_narrow=6)
    lat, sig = wl.lattice, wl.sigma
    dl, ds = Lattice.from_host(lat), SelfEnergy.from_host(sig)
    mu = 0.2
    out = ctx.dmft_ntot(dl, ds, mu, tail_order=0).cpu().numpy()
    ctx.sync_status()
    n, d = oracle.trace(lat, sig, mu, tail_order=0)
    assert abs(out[0] - n) <= RTOL * abs(n) and abs(out[1] - d) <= RTOL * abs(d)
    rng = np.random.default_rng(12)
    nbar = [rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)) for m in lat.nb]
    gbar = rng.standard_normal(sig.sigma.shape) + 1j * rng.standard_normal(sig.sigma.shape)
    sb, mb = ctx.density_matrix_vjp(dl, ds, mu, torch.as_tensor(np.concatenate([x.ravel() for x in nbar]),
                                                                device="cuda"),
                                    torch.as_tensor(gbar, device="cuda"), tail_order=0)
    ctx.sync_status()
    ref, mub = oracle.vjp(lat, sig, mu, nbar=nbar, gbar=gbar, tail_order=0)
    assert abs(float(mb[0]) - mub) <= RTOL * max(1.0, abs(mub))
    sbn = sb.cpu().numpy()
    for nn in range(sig.nw):
        assert relerr(sbn[nn], ref[nn]) <= RTOL, nn
    n0 = 9.0
    mu_ref, _, _ = oracle.find_mu_bisect(lat, sig, n0, 1e-12, -40.0, 40.0, max_iter=300, tail_order=0)
    for m in (NEWTON, BISECT):
        mu_g, _, ng = ctx.find_mu(dl, ds, n0, 1e-12, m, -40.0, 40.0, max_iter=300, tail_order=0)
        assert abs(ng - n0) <= 1e-12
        assert abs(mu_g - mu_ref) <= 1e-10 * max(1.0, abs(mu_ref))


def test_mu_parity_on_differentiation_subset(ctx):
    """Parity mode of the mu search on the differentiation workload (beta = 50,
    Nb = 40, Nc = 14) at full Nw = 2048 on its first 32 k-points (weights
    1/32): the oracle's bisection and both GPU searches solve to
    |N - N0| <= 1e-13 N0, and the roots agree to 1e-10 max(1, |mu|)."""
    from paper_1111_2157_amd.dyson import BISECT, NEWTON, Lattice, SelfEnergy

    wl = synth.differentiation()
    sub = wl.lattice.subset(np.arange(32))
    sub.wk[:] = 1.0 / 32
    sig = wl.sigma
    n0 = wl.n_target
    tol = 1e-13 * n0
    print("oracle bisection on the 32-k subset", flush=True)
    mu_ref, p_ref, n_ref = oracle.find_mu_bisect(sub, sig, n0, tol, -40.0, 40.0, max_iter=200)
    _, d_ref = oracle.trace(sub, sig, mu_ref)
    assert d_ref > 1e-2
    dl, ds = Lattice.from_host(sub), SelfEnergy.from_host(sig)
    for m in (NEWTON, BISECT):
        mu_g, passes, ng = ctx.find_mu(dl, ds, n0, tol, m, -40.0, 40.0, max_iter=200)
        print("gpu", m, mu_g, passes, "oracle", mu_ref, p_ref, flush=True)
        assert abs(ng - n0) <= tol
        assert abs(mu_g - mu_ref) <= 1e-10 * max(1.0, abs(mu_ref))
