"""Edge cases of the Dyson pass, the trace pass and the general vector-Jacobian
product in both forms (dense and low-rank) against the FP64 oracle: square
projectors (nb = nc, including 1 and 16), the maximum sizes (nb = 64, nc = 16),
a single frequency, a single k-point and a vanishing self-energy (G = D, where
the low-rank form has R = 0); and the shapes the library rejects before any
launch (no k-points, no frequencies, windows or orbital counts out of range)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1111_2157_amd import synth
from gpu_util import RTOL, assert_gloc_parity, assert_nk_parity, gpu_density, relerr

pytestmark = pytest.mark.gpu


def _noninteracting():
    wl = synth.plain(nk=6, nb=12, nc=5, nw=32)
    s = wl.sigma
    zero = synth.SelfEnergy(s.nw, s.beta, np.zeros_like(s.sigma),
                            None if s.sigma_inf is None else np.zeros_like(s.sigma_inf), np.zeros_like(s.e_dc))
    return synth.Workload("plain-sigma0", wl.lattice, [zero], mu=0.0)


EDGE = {
    "nb=nc=5": (lambda: synth.plain(nk=5, nb=5, nc=5, nw=24), 0.3),
    "nb=nc=1": (lambda: synth.plain(nk=5, nb=1, nc=1, nw=24), -0.2),
    "nb=nc=16": (lambda: synth.plain(nk=3, nb=16, nc=16, nw=12), 0.1),
    "nb=64,nc=16": (lambda: synth.plain(nk=2, nb=64, nc=16, nw=8), 0.0),
    "nw=1": (lambda: synth.plain(nk=7, nw=1), -1.0),
    "nk=1": (lambda: synth.plain(nk=1, nw=20), 0.5),
    "sigma=0": (_noninteracting, 0.0),
}


def _context(form):
    """Context pinned to the first dense (form 'dense') or low-rank variant of
    every kind and padded size; the adjoint kinds' dense code is 0."""
    from paper_1111_2157_amd.dyson import Context

    c = Context(0)
    for kind in (0, 1, 2, 3):
        for nbp in (16, 32, 48, 64):
            vs = c.variants(kind, nbp)
            pick = [v for v in vs if (v & 8) == (8 if form == "lowrank" else 0)]
            if pick:
                c.set_variant(kind, nbp, pick[0])
    return c


@pytest.fixture(scope="module", params=["dense", "lowrank"])
def fctx(request):
    c = _context(request.param)
    yield request.param, c
    c.close()


@pytest.mark.parametrize("name", list(EDGE))
def test_edge_density_trace_and_vjp(fctx, name):
    import torch

    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    form, ctx = fctx
    maker, mu = EDGE[name]
    wl = maker()
    lat, sig = wl.lattice, wl.sigma
    mats, gl, _ = gpu_density(ctx, wl, mu)
    assert_nk_parity(mats, lat, sig, mu)
    assert_gloc_parity(gl, lat, sig, mu)
    dl, ds = Lattice.from_host(lat), SelfEnergy.from_host(sig)
    out = ctx.dmft_ntot(dl, ds, mu).cpu().numpy()
    ctx.sync_status()
    n, d = oracle.trace(lat, sig, mu)
    assert abs(out[0] - n) <= RTOL * max(1.0, abs(n))
    assert abs(out[1] - d) <= RTOL * max(1.0, abs(d))
    if form == "dense" and lat.nb_max > 48:
        return  # the dense adjoint kernel covers windows up to 48
    rng = np.random.default_rng(9)
    nbar = [rng.standard_normal((b, b)) + 1j * rng.standard_normal((b, b)) for b in lat.nb]
    gbar = rng.standard_normal(sig.sigma.shape) + 1j * rng.standard_normal(sig.sigma.shape)
    nbt = torch.as_tensor(np.concatenate([m.ravel() for m in nbar]), device="cuda")
    sb, mb = ctx.density_matrix_vjp(dl, ds, mu, nbt, torch.as_tensor(gbar, device="cuda"))
    sb, mb = sb.cpu().numpy(), float(mb.cpu().numpy()[0])
    ctx.sync_status()
    ref, mref = oracle.vjp(lat, sig, mu, nbar=nbar, gbar=gbar)
    assert relerr(sb, ref) <= RTOL
    assert abs(mb - mref) <= RTOL * max(1.0, abs(mref))


def test_noninteracting_green_function_is_diagonal(fctx):
    """With Sigma = 0 and V_DC = 0, G_kn = D_kn, so G_loc(n) = sum_k w_k S D S^dag:
    the GPU G_loc equals that sum formed directly on the host."""
    form, ctx = fctx
    wl = _noninteracting()
    lat, sig = wl.lattice, wl.sigma
    _, gl, _ = gpu_density(ctx, wl, 0.0)
    wn = (2 * np.arange(sig.nw) + 1) * np.pi / sig.beta
    ref = np.zeros_like(gl)
    for k in range(lat.nk):
        s = lat.proj_k(k)
        d = 1.0 / (1j * wn[:, None] - lat.eps_k(k)[None, :])
        ref += lat.wk[k] * np.einsum("ab,nb,cb->nac", s, d, s.conj())
    assert relerr(gl, ref) <= RTOL


def test_rejected_shapes(fctx):
    from paper_1111_2157_amd._lib import DmftError
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    _, ctx = fctx
    wl = synth.plain(nk=4, nw=8)
    dl, ds = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
    bad = [
        (dataclasses.replace(dl, nk=0), ds),
        (dl, dataclasses.replace(ds, nw=0)),
        (dataclasses.replace(dl, nb_max=65), ds),
        (dataclasses.replace(dl, nc=17), ds),
        (dataclasses.replace(dl, nb_max=4), ds),  # fewer bands than correlated orbitals
    ]
    for lat, sig in bad:
        with pytest.raises(DmftError) as e:
            ctx.dmft_ntot(lat, sig, 0.0)
        assert e.value.name == "DMFT_EINVAL"
