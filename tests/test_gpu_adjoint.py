"""GPU adjoint: dN/dmu and dN/dSigma from the fused scalar adjoint, the general
vector-Jacobian product, and the autograd.Function, against the oracle's
gradient and against central finite differences of the GPU forward."""
import numpy as np
import pytest

import oracle
from paper_1111_2157_amd import synth
from gpu_util import relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1111_2157_amd.dyson import Context

    c = Context(0)
    yield c
    c.close()


CASES = [
    ("plain", lambda: synth.plain(nk=6, nw=40), -1.5),
    ("d-shell", lambda: synth.d_shell(nk=6, nw=32), 0.2),
    ("diff-nb40", lambda: synth.differentiation(nk=4, nw=24), -0.5),
    ("ragged", lambda: synth.batched(nk=6, nb_lo=14, nb_hi=44, nw=24, n_iter=1), 0.0),
]


@pytest.mark.parametrize("name,maker,mu", CASES)
def test_scalar_adjoint_matches_oracle(ctx, name, maker, mu):
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = maker()
    lat, sig = wl.lattice, wl.sigma
    out, sb = ctx.dmft_ntot_vjp(Lattice.from_host(lat), SelfEnergy.from_host(sig), mu)
    out, sb = out.cpu().numpy(), sb.cpu().numpy()
    ctx.sync_status()
    n, d = oracle.trace(lat, sig, mu)
    assert abs(out[0] - n) <= 1e-10 * abs(n)
    assert abs(out[1] - d) <= 1e-10 * abs(d)
    nbar = [lat.wk[k] * np.eye(lat.nb[k]) for k in range(lat.nk)]
    ref, mub = oracle.vjp(lat, sig, mu, nbar=nbar)
    assert abs(mub - d) <= 1e-10 * abs(d)
    for nn in range(sig.nw):
        assert relerr(sb[nn], ref[nn]) <= 1e-10, nn


GEN_CASES = CASES + [
    ("ragged-to-64", lambda: synth.batched(nk=6, nb_lo=40, nb_hi=64, nw=20, n_iter=1), 0.1),
    ("f-shell-nb60", lambda: synth.f_shell(nk=3, nb=60, nc=14, nw=16, beta=20.0), 0.0),
]


def _padded_sizes(lat):
    return sorted({(int(n) + 15) // 16 * 16 for n in lat.nb})


@pytest.mark.parametrize("form", ["lowrank", "dense", "mixed"])
@pytest.mark.parametrize("name,maker,mu", GEN_CASES)
def test_general_vjp_matches_oracle(ctx, name, maker, mu, form):
    """density_matrix_vjp against the oracle in the low-rank form (the default),
    the dense adjoint kernel (code 0), and both at once on a ragged lattice
    (dense on the smallest padded size), whose partial sums then mix forms."""
    import torch

    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = maker()
    lat, sig = wl.lattice, wl.sigma
    sizes = _padded_sizes(lat)
    if form == "dense" and sizes[-1] > 48:
        pytest.skip("the dense adjoint kernel covers band windows up to 48")
    if form == "mixed" and len(sizes) < 2:
        pytest.skip("needs band windows of several padded sizes")
    rng = np.random.default_rng(5)
    nbar = [rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for n in lat.nb]
    gbar = rng.standard_normal(sig.sigma.shape) + 1j * rng.standard_normal(sig.sigma.shape)
    dl, ds = Lattice.from_host(lat), SelfEnergy.from_host(sig)
    nbt = torch.as_tensor(np.concatenate([m.ravel() for m in nbar]), device="cuda")
    gbt = torch.as_tensor(gbar, device="cuda")
    try:
        for p in sizes:
            if form == "dense" or (form == "mixed" and p == sizes[0]):
                ctx.set_variant(3, p, 0)
            else:
                assert ctx.get_variant(3, p) & 8
        for use_n, use_g in ((True, True), (True, False), (False, True)):
            sb, mb = ctx.density_matrix_vjp(dl, ds, mu, nbt if use_n else None, gbt if use_g else None)
            sb, mb = sb.cpu().numpy(), float(mb.cpu().numpy()[0])
            ctx.sync_status()
            ref, mref = oracle.vjp(lat, sig, mu, nbar=nbar if use_n else None, gbar=gbar if use_g else None)
            assert abs(mb - mref) <= 1e-10 * max(1.0, abs(mref)), (use_n, use_g, mb, mref)
            assert relerr(sb, ref) <= 1e-10, (use_n, use_g)
    finally:
        for p in sizes:
            ctx.set_variant(3, p, -1)


@pytest.mark.parametrize("var", [8, 9, 24])
def test_general_vjp_lowrank_variants(ctx, var):
    """Every compiled low-rank variant of the general product on a 40-band
    case against the oracle."""
    import torch

    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    if var not in ctx.variants(3, 48):
        pytest.skip("variant not compiled for 48 bands")
    wl = synth.differentiation(nk=4, nw=20)
    lat, sig = wl.lattice, wl.sigma
    rng = np.random.default_rng(11)
    nbar = [rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for n in lat.nb]
    gbar = rng.standard_normal(sig.sigma.shape) + 1j * rng.standard_normal(sig.sigma.shape)
    nbt = torch.as_tensor(np.concatenate([m.ravel() for m in nbar]), device="cuda")
    gbt = torch.as_tensor(gbar, device="cuda")
    try:
        ctx.set_variant(3, 48, var)
        sb, mb = ctx.density_matrix_vjp(Lattice.from_host(lat), SelfEnergy.from_host(sig), -0.4, nbt, gbt)
        sb, mb = sb.cpu().numpy(), float(mb.cpu().numpy()[0])
        ctx.sync_status()
    finally:
        ctx.set_variant(3, 48, -1)
    ref, mref = oracle.vjp(lat, sig, -0.4, nbar=nbar, gbar=gbar)
    assert abs(mb - mref) <= 1e-10 * max(1.0, abs(mref))
    assert relerr(sb, ref) <= 1e-10


def test_general_vjp_fullsize_forms_agree(ctx):
    """At the differentiation workload's full size (Nk=1024, Nb=40, Nc=14,
    Nw=2048) the low-rank and the dense general product agree to 1e-10, the
    first eight frequencies of Sigma-bar match the oracle, and with
    Nbar_k = w_k I and no G_loc cotangent the general product equals the fused
    scalar adjoint (dN_tot/dSigma, dN_tot/dmu)."""
    import torch

    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = synth.differentiation()
    lat, sig = wl.lattice, wl.sigma
    dl, ds = Lattice.from_host(lat), SelfEnergy.from_host(sig)
    mu = -0.8
    rng = np.random.default_rng(3)
    nbar = np.concatenate([(rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)) for n in lat.nb])
    gbar = rng.standard_normal(sig.sigma.shape) + 1j * rng.standard_normal(sig.sigma.shape)
    nbt, gbt = torch.as_tensor(nbar, device="cuda"), torch.as_tensor(gbar, device="cuda")
    assert ctx.get_variant(3, 48) & 8
    sl, ml = ctx.density_matrix_vjp(dl, ds, mu, nbt, gbt)
    sl, ml = sl.cpu().numpy(), float(ml.cpu().numpy()[0])
    ctx.sync_status()
    try:
        ctx.set_variant(3, 48, 0)
        sd, md = ctx.density_matrix_vjp(dl, ds, mu, nbt, gbt)
        sd, md = sd.cpu().numpy(), float(md.cpu().numpy()[0])
        ctx.sync_status()
    finally:
        ctx.set_variant(3, 48, -1)
    assert relerr(sl, sd) <= 1e-10
    assert abs(ml - md) <= 1e-10 * max(1.0, abs(md))
    # oracle on the first frequencies over every k: sigma_bar_n depends only on
    # Sigma(i w_n) and the cotangents at that n, so a self-energy cut to the
    # first m frequencies gives the same slices
    m = 8
    cut = synth.SelfEnergy(m, sig.beta, sig.sigma[:m].copy(), sig.sigma_inf, sig.e_dc)
    nbar_k, off = [], 0
    for n in lat.nb:
        nbar_k.append(nbar[off:off + n * n].reshape(n, n))
        off += n * n
    ref, _ = oracle.vjp(lat, cut, mu, nbar=nbar_k, gbar=gbar[:m])
    assert relerr(sl[:m], ref) <= 1e-10
    eye = np.concatenate([(lat.wk[k] * np.eye(n)).ravel() for k, n in enumerate(lat.nb)]).astype(np.complex128)
    sg, mg = ctx.density_matrix_vjp(dl, ds, mu, torch.as_tensor(eye, device="cuda"), None)
    out, sf = ctx.dmft_ntot_vjp(dl, ds, mu)
    sg, mg, out, sf = sg.cpu().numpy(), float(mg.cpu().numpy()[0]), out.cpu().numpy(), sf.cpu().numpy()
    ctx.sync_status()
    assert relerr(sg, sf) <= 1e-10
    assert abs(mg - out[1]) <= 1e-10 * abs(out[1])


def test_dn_dsigma_central_differences_on_gpu(ctx):
    """dN/dSigma of the adjoint against central differences (h = 1e-6) of the GPU
    forward N_tot, to 1e-6 of the gradient's largest entry."""
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = synth.differentiation(nk=6, nw=32)
    lat, sig = wl.lattice, wl.sigma
    dl = Lattice.from_host(lat)
    mu, h = -0.6, 1e-6
    out, sb = ctx.dmft_ntot_vjp(dl, SelfEnergy.from_host(sig), mu)
    sb = sb.cpu().numpy()
    d = float(out[1])
    gmax = np.abs(sb).max()

    def ntot(s, m):
        return float(ctx.dmft_ntot(dl, SelfEnergy.from_host(s), m)[0])

    fdmu = (ntot(sig, mu + h) - ntot(sig, mu - h)) / (2 * h)
    assert abs(fdmu - d) <= 1e-6 * abs(d)
    for (n, a, b) in [(0, 0, 0), (0, 3, 7), (5, 13, 2), (sig.nw - 1, 9, 9)]:
        fd = 0j
        for unit in (1.0, 1j):
            vals = []
            for sgn in (+1, -1):
                s2 = sig.sigma.copy()
                s2[n, a, b] += sgn * h * unit
                vals.append(ntot(synth.SelfEnergy(sig.nw, sig.beta, s2, sig.sigma_inf, sig.e_dc), mu))
            fd += unit * (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - sb[n, a, b]) <= 1e-6 * gmax, (n, a, b, fd, sb[n, a, b])


def test_autograd_function_gradcheck(ctx):
    import torch

    from paper_1111_2157_amd.autograd import dyson_density
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = synth.f_shell(nk=2, nb=6, nc=3, nw=6, beta=5.0, n_narrow=2)
    dl, base = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
    sigma = base.sigma.clone().requires_grad_(True)
    mu = torch.tensor(0.25, dtype=torch.float64, device="cuda", requires_grad=True)

    def f(s, m):
        nk, gl = dyson_density(s, m, ctx, dl, base)
        return nk, gl

    assert torch.autograd.gradcheck(f, (sigma, mu), eps=1e-6, atol=1e-7, rtol=1e-6)


def test_autograd_matches_oracle_gradient(ctx):
    import torch

    from paper_1111_2157_amd.autograd import dyson_density
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = synth.d_shell(nk=4, nw=24)
    lat, sig = wl.lattice, wl.sigma
    dl, base = Lattice.from_host(lat), SelfEnergy.from_host(sig)
    sigma = base.sigma.clone().requires_grad_(True)
    mu = torch.tensor(0.1, dtype=torch.float64, device="cuda", requires_grad=True)
    nk, gl = dyson_density(sigma, mu, ctx, dl, base)
    # loss = N_tot (real part of the weighted trace) + Re sum G_loc
    nbs = lat.nb.astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(nbs * nbs)])
    loss = gl.real.sum()
    for k in range(lat.nk):
        m = nk[offs[k]:offs[k + 1]].reshape(int(nbs[k]), int(nbs[k]))
        loss = loss + lat.wk[k] * torch.diagonal(m).real.sum()
    loss.backward()
    nbar = [lat.wk[k] * np.eye(lat.nb[k]) for k in range(lat.nk)]
    gbar = np.ones_like(sig.sigma)
    ref, mref = oracle.vjp(lat, sig, 0.1, nbar=nbar, gbar=gbar)
    assert relerr(sigma.grad.cpu().numpy(), ref) <= 1e-10
    assert abs(float(mu.grad) - mref) <= 1e-10 * max(1.0, abs(mref))


ADJ_VARIANT_CASES = [(16, lambda: synth.plain(nk=6, nw=40), -1.5), (32, lambda: synth.d_shell(nk=6, nw=32), 0.2),
                     (48, lambda: synth.differentiation(nk=4, nw=24), -0.5),
                     (64, lambda: synth.f_shell(nk=3, nb=64, nw=20), 0.0)]


@pytest.mark.parametrize("nbp,maker,mu", ADJ_VARIANT_CASES)
def test_every_adjoint_variant_matches_oracle(nbp, maker, mu):
    """Kind 2 (fused scalar adjoint): the low-rank variants and, up to 48
    bands, the dense adjoint kernel (code 0), each against the oracle."""
    from paper_1111_2157_amd.dyson import Context, Lattice, SelfEnergy

    wl = maker()
    lat, sig = wl.lattice, wl.sigma
    n, d = oracle.trace(lat, sig, mu)
    nbar = [lat.wk[k] * np.eye(lat.nb[k]) for k in range(lat.nk)]
    ref, _ = oracle.vjp(lat, sig, mu, nbar=nbar)
    c = Context(0)
    dl, ds = Lattice.from_host(lat), SelfEnergy.from_host(sig)
    vars_ = c.variants(2, nbp)
    assert any(v & 8 for v in vars_) and ((0 in vars_) == (nbp <= 48))
    for var in vars_:
        print("adjoint variant", nbp, var, flush=True)
        c.set_variant(2, nbp, var)
        out, sb = c.dmft_ntot_vjp(dl, ds, mu)
        out, sb = out.cpu().numpy(), sb.cpu().numpy()
        c.sync_status()
        assert abs(out[0] - n) <= 1e-10 * abs(n), var
        assert abs(out[1] - d) <= 1e-10 * abs(d), var
        for nn in range(sig.nw):
            assert relerr(sb[nn], ref[nn]) <= 1e-10, (var, nn)
    c.close()


def test_lowrank_adjoint_ragged_up_to_64(ctx):
    """Ragged windows 14..64 (the dense adjoint stops at 48)."""
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = synth.batched(nk=8, nb_lo=14, nb_hi=64, nw=24, n_iter=2)
    for s in range(2):
        lat, sig = wl.lattices[s], wl.sigmas[s]
        assert lat.nb.max() > 48
        out, sb = ctx.dmft_ntot_vjp(Lattice.from_host(lat), SelfEnergy.from_host(sig), 0.1)
        out, sb = out.cpu().numpy(), sb.cpu().numpy()
        ctx.sync_status()
        n, d = oracle.trace(lat, sig, 0.1)
        assert abs(out[0] - n) <= 1e-10 * abs(n)
        assert abs(out[1] - d) <= 1e-10 * abs(d)
        nbar = [lat.wk[k] * np.eye(lat.nb[k]) for k in range(lat.nk)]
        ref, _ = oracle.vjp(lat, sig, 0.1, nbar=nbar)
        for nn in range(sig.nw):
            assert relerr(sb[nn], ref[nn]) <= 1e-10, (s, nn)
