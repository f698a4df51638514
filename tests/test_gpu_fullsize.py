"""Full-size workloads in the launch configuration the benchmark times (the
autotuned kernel variant and tiles of each shape), checked against the oracle
on sampled outputs it can compute one by one -- N(k) at a few k-points, G_loc
at a few Matsubara frequencies, the trace pass on a few k-points -- and
through properties that hold at any size: N(k) Hermitian, the reduced scalars
equal to the same sums taken on the host from the returned N(k), the trace
pass equal to the density pass, and dN/dmu equal to central differences."""
import numpy as np
import pytest

import oracle
from paper_1111_2157_amd import synth
from gpu_util import RTOL, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1111_2157_amd.dyson import Context

    c = Context(0)
    yield c
    c.close()


WORKLOADS = {
    "d-shell": lambda: synth.d_shell(),
    "f-shell": lambda: synth.f_shell(),
    "diff": lambda: synth.differentiation(),
}


def _sample(n, count, rng):
    picks = {0, n - 1}
    while len(picks) < min(count, n):
        picks.add(int(rng.integers(n)))
    return sorted(picks)


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_fullsize_density_pass(ctx, name):
    import torch

    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy, split_nk

    wl = WORKLOADS[name]()
    lat, sig, mu = wl.lattice, wl.sigma, wl.mu + 0.05
    dl, ds = Lattice.from_host(lat), SelfEnergy.from_host(sig)
    print("autotune", name, flush=True)
    ctx.autotune(dl, ds, mu)
    nbp = (lat.nb_max + 15) // 16 * 16
    print("density pass", name, "variant", ctx.get_variant(0, nbp), flush=True)
    nk, gl, sc = ctx.density_matrix(dl, ds, mu)
    torch.cuda.synchronize()
    ctx.sync_status()
    mats = [m.cpu().numpy() for m in split_nk(nk, dl)]
    gl = gl.cpu().numpy()
    sc = sc.cpu().numpy()
    rng = np.random.default_rng(11)

    ks = _sample(lat.nk, 4, rng)
    print("oracle N(k) at", ks, flush=True)
    ref, _ = oracle.density(lat, sig, mu, 2, klist=ks)
    for i, k in enumerate(ks):
        assert relerr(mats[k], ref[i]) <= RTOL, k

    ns = _sample(sig.nw, 3, rng)
    print("oracle G_loc at", ns, flush=True)
    gref = oracle.gloc(lat, sig, mu, ns)
    for i, n in enumerate(ns):
        assert relerr(gl[n], gref[i]) <= RTOL, n

    # properties over every k: Hermitian N(k); the scalars are the w_k sums
    ntot = ncor = hks = 0.0
    herm = 0.0
    for k, m in enumerate(mats):
        herm = max(herm, np.abs(m - m.conj().T).max() / max(np.abs(m).max(), 1e-300))
        p = lat.proj_k(k)
        ntot += lat.wk[k] * np.trace(m).real
        ncor += lat.wk[k] * np.trace(p @ m @ p.conj().T).real
        hks += lat.wk[k] * np.sum(lat.eps_k(k) * np.diag(m).real)
    assert herm <= 1e-12
    assert abs(sc[0] - ntot) <= RTOL * abs(ntot)
    assert abs(sc[1] - ncor) <= RTOL * max(abs(ncor), 1.0)
    assert abs(sc[2] - hks) <= RTOL * max(abs(hks), 1.0)

    # the trace pass (mu search) at full size: same N_tot, and dN/dmu against
    # central differences of the GPU N_tot
    print("trace pass", name, "variant", ctx.get_variant(1, nbp), flush=True)
    out = ctx.dmft_ntot(dl, ds, mu).cpu().numpy()
    ctx.sync_status()
    assert abs(out[0] - ntot) <= RTOL * abs(ntot)
    h = 1e-5
    fd = (float(ctx.dmft_ntot(dl, ds, mu + h)[0]) - float(ctx.dmft_ntot(dl, ds, mu - h)[0])) / (2 * h)
    assert abs(fd - out[1]) <= 1e-6 * abs(out[1])

    # the same trace kernel on a few k-points, against the oracle
    sub = lat.subset(ks)
    out_s = ctx.dmft_ntot(Lattice.from_host(sub), ds, mu).cpu().numpy()
    ctx.sync_status()
    n_ref, d_ref = oracle.trace(sub, sig, mu)
    assert abs(out_s[0] - n_ref) <= RTOL * abs(n_ref)
    assert abs(out_s[1] - d_ref) <= RTOL * abs(d_ref)


def test_fullsize_batched_pass(ctx):
    import torch

    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = synth.batched()
    lats = [Lattice.from_host(l) for l in wl.lattices]
    sigs = [SelfEnergy.from_host(s) for s in wl.sigmas]
    print("batched plan", flush=True)
    ctx.batched_plan(lats, sigs, 2)
    print("batched form", ctx.batched_form(), flush=True)
    mus = np.linspace(-0.2, 0.2, len(lats))
    mu_dev = torch.as_tensor(mus, device="cuda")
    nks, gls = ctx.batched_outputs()
    ctx.batched_graph_capture(mu_dev, nks, gls)
    torch.cuda.synchronize()
    ctx.batched_sync_status()
    rng = np.random.default_rng(5)
    for s, (lat, sig) in enumerate(zip(wl.lattices, wl.sigmas)):
        offs = np.concatenate([[0], np.cumsum(lat.nb.astype(np.int64) ** 2)])
        ks = _sample(lat.nk, 2, rng)
        print("iterate", s, "oracle N(k) at", ks, flush=True)
        ref, _ = oracle.density(lat, sig, mus[s], 2, klist=ks)
        for i, k in enumerate(ks):
            nb = int(lat.nb[k])
            got = nks[s][int(offs[k]):int(offs[k + 1])].cpu().numpy().reshape(nb, nb)
            assert relerr(got, ref[i]) <= RTOL, (s, k)
        n = int(rng.integers(sig.nw))
        gref = oracle.gloc(lat, sig, mus[s], [n])
        assert relerr(gls[s][n].cpu().numpy(), gref[0]) <= RTOL, (s, n)
    del nks, gls
    ctx._b_ws = None
    torch.cuda.empty_cache()


def test_fullsize_newton_mu_search(ctx):
    from paper_1111_2157_amd.dyson import BISECT, NEWTON, Lattice, SelfEnergy

    wl = synth.differentiation()
    dl, ds = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
    ctx.autotune(dl, ds, 0.0)
    mu_n, pn, nn = ctx.find_mu(dl, ds, wl.n_target, 1e-8, NEWTON, -40.0, 40.0)
    mu_b, pb, nb = ctx.find_mu(dl, ds, wl.n_target, 1e-8, BISECT, -40.0, 40.0)
    print("newton", mu_n, pn, "bisect", mu_b, pb, flush=True)
    assert abs(nn - wl.n_target) <= 1e-8 and abs(nb - wl.n_target) <= 1e-8
    assert pn * 3 <= pb
    # N(mu) of the density pass at Newton's root
    _, _, sc = ctx.density_matrix(dl, ds, mu_n)
    assert abs(float(sc[0]) - wl.n_target) <= 1e-8 + RTOL * wl.n_target
    d = float(ctx.dmft_ntot(dl, ds, mu_n)[1])
    assert abs(mu_n - mu_b) <= 2e-8 / d
