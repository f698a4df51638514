"""GPU parity of the low-rank density kernel that packs three frequencies into
each matrix-core tile (variant code 42, nc <= 5; 64-band windows on four
wavefronts) against the FP64 oracle: every padded size, nc from 1 to 5, full
self-energies with off-diagonal elements, frequency counts that leave a partial
group (of twelve, or of 48 on 64-band windows) and counts below one group,
ragged windows, skewed projectors, and the fallback to the size's default
variant for nc > 5."""
import numpy as np
import pytest

from paper_1111_2157_amd import synth
from gpu_util import assert_gloc_parity, assert_nk_parity, gpu_density, relerr

pytestmark = pytest.mark.gpu

P3 = 42


def p3_context():
    """Context with the packed variant for the density kind of every size it serves."""
    from paper_1111_2157_amd.dyson import Context

    c = Context(0)
    for nbp in (16, 32, 48, 64):
        assert P3 in c.variants(0, nbp), nbp
        c.set_variant(0, nbp, P3)
    return c


@pytest.fixture(scope="module")
def ctx():
    c = p3_context()
    yield c
    c.close()


CASES = {
    # nb 12 -> 16-band windows; Nw = 256 leaves a group of four frequencies
    "plain-full": (lambda: synth.plain(), -2.0),
    "nb32-nc5-full-sigma": (lambda: synth.f_shell(nk=8, nb=32, nc=5, nw=50, n_narrow=6), 0.2),
    "nb40-nc5": (lambda: synth.f_shell(nk=6, nb=40, nc=5, nw=37, n_narrow=8), -0.3),
    "nb48-nc4": (lambda: synth.f_shell(nk=5, nb=48, nc=4, nw=25, n_narrow=6), 0.1),
    "nb20-nc3": (lambda: synth.f_shell(nk=7, nb=20, nc=3, nw=13, n_narrow=4), 0.4),
    "nb9-nc2-nw7": (lambda: synth.plain(nk=5, nb=9, nc=2, nw=7), 0.0),
    "nb17-nc1": (lambda: synth.plain(nk=4, nb=17, nc=1, nw=30), 0.5),
    "nb33-nc5-nw12": (lambda: synth.plain(nk=4, nb=33, nc=5, nw=12), -1.0),
    # 64-band windows: groups of 48 frequencies on four wavefronts
    "nb64-nc5-full-sigma": (lambda: synth.f_shell(nk=5, nb=64, nc=5, nw=53, n_narrow=10), 0.25),
    "nb57-nc3-nw30": (lambda: synth.plain(nk=4, nb=57, nc=3, nw=30), -0.5),
    "nb49-nc1-nw100": (lambda: synth.plain(nk=3, nb=49, nc=1, nw=100), 0.7),
}


@pytest.mark.parametrize("name", list(CASES))
def test_p3_density_and_gloc(ctx, name):
    maker, mu = CASES[name]
    wl = maker()
    assert wl.lattice.nc <= 5
    print("packed-by-3 density", name, flush=True)
    mats, gl, sc = gpu_density(ctx, wl, mu)
    assert_nk_parity(mats, wl.lattice, wl.sigma, mu)
    assert_gloc_parity(gl, wl.lattice, wl.sigma, mu)


@pytest.mark.parametrize("tail", [0, 2])
def test_p3_ragged_windows(ctx, tail):
    """Band windows 14..64 of a 5-orbital iterate: every bucket runs the packed
    kernel (the 64-band one on four wavefronts)."""
    wl = synth.batched(nk=24, nb_lo=14, nb_hi=64, nw=40, n_iter=1)
    lat = wl.lattices[0]
    assert lat.nc == 5
    print("packed-by-3 ragged, tail", tail, flush=True)
    mats, gl, sc = gpu_density(ctx, wl, 0.15, tail=tail)
    assert_nk_parity(mats, lat, wl.sigmas[0], 0.15, tail=tail)
    assert_gloc_parity(gl, lat, wl.sigmas[0], 0.15)


def test_p3_non_orthonormal_projectors(ctx):
    from test_gpu_lowrank import skewed_projectors

    wl = synth.f_shell(nk=6, nb=30, nc=5, nw=29, n_narrow=6)
    lat = skewed_projectors(wl)
    print("packed-by-3 skewed projectors", flush=True)
    mats, gl, sc = gpu_density(ctx, wl, 0.2, lat=lat)
    assert_nk_parity(mats, lat, wl.sigma, 0.2)
    assert_gloc_parity(gl, lat, wl.sigma, 0.2)


def test_p3_agrees_with_default_variant():
    """The packed kernel and the size's default low-rank variant give the same
    N(k), G_loc and scalars to rounding."""
    from paper_1111_2157_amd.dyson import Context

    wl = synth.f_shell(nk=12, nb=44, nc=5, nw=100, n_narrow=8)
    c0 = Context(0)
    c1 = p3_context()
    print("packed-by-3 vs default", flush=True)
    m0, g0, s0 = gpu_density(c0, wl, 0.05)
    m1, g1, s1 = gpu_density(c1, wl, 0.05)
    for a, b in zip(m1, m0):
        assert relerr(a, b) <= 1e-12
    assert relerr(g1, g0) <= 1e-12
    assert relerr(s1, s0) <= 1e-12
    c0.close()
    c1.close()


def test_p3_falls_back_for_larger_nc(ctx):
    """With the packed variant selected, an nc = 10 lattice runs the size's
    default variant and still matches the oracle."""
    wl = synth.d_shell(nk=6, nw=30)
    assert wl.lattice.nc > 5
    print("packed-by-3 fallback nc", wl.lattice.nc, flush=True)
    mats, gl, sc = gpu_density(ctx, wl, 0.3)
    assert_nk_parity(mats, wl.lattice, wl.sigma, 0.3)
    assert_gloc_parity(gl, wl.lattice, wl.sigma, 0.3)


def test_p3_autotune_candidates_agree():
    """The autotuner times the packed variant for an nc = 5 shape next to the
    others and accepts it (each candidate must reproduce the first to 1e-11)."""
    from paper_1111_2157_amd.dyson import Context, Lattice, SelfEnergy

    wl = synth.f_shell(nk=16, nb=30, nc=5, nw=64, n_narrow=6)
    c = Context(0)
    print("packed-by-3 autotune", flush=True)
    rep = c.autotune(Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma), 0.0)
    lines = [l for l in rep.splitlines() if l.startswith("density") and "var=%d " % P3 in l]
    assert lines, rep
    assert not any("rejected" in l for l in lines), rep
    c.close()
