"""GPU parity of the partial-fraction running sum of the low-rank kernels
(nc > 8: the two-wavefront kernel of 64-band windows, variant 40, and the
single-wavefront kernel's variants 74 and 90 on 32- and 48-band windows;
nc <= 5: the four-wavefront kernel of 64-band windows that packs three
frequencies per tile, variant 42) against the FP64 oracle, on band structures built to reach
each of its branches: distinct bands (the divided form), exactly degenerate and
nearly degenerate pairs (the directly summed close pair), a triple degeneracy
(more than one close partner: the k-point takes the direct running sum), and
pairs just outside the closeness threshold (the smallest divisors the divided
form meets)."""
import numpy as np
import pytest

from paper_1111_2157_amd import synth
from gpu_util import assert_gloc_parity, assert_nk_parity, gpu_density

pytestmark = pytest.mark.gpu


def crafted(nc=14, nb=60, nk=8, nw=40, beta=40.0, seed=5):
    """f-shell-like lattice whose k-points carry the degeneracy patterns above;
    delta = pi / (16 beta) is the kernel's closeness threshold."""
    wl = synth.f_shell(nk=nk, nb=nb, nc=nc, nw=nw, beta=beta, n_narrow=12, seed=seed)
    lat = wl.lattice
    eps = lat.eps.copy().reshape(nk, nb)
    delta = np.pi / (16.0 * beta)
    eps[0, 3] = eps[0, 7] = eps[0, nb - 20] = eps[0, 20]      # triple degeneracy: direct sum
    eps[1, 5] = eps[1, nb - 7]                                # exact pair
    eps[2, 9] = eps[2, nb - 10] + 1e-4                         # near pair
    eps[3, 2] = eps[3, 17] + 0.5 * delta                  # close pair, half the threshold
    eps[4, 11] = eps[4, nb - 3] + 2.0 * delta                 # just outside: divided form
    eps[5, 0] = eps[5, nb - 1] + 1.001 * delta                # at the threshold
    eps[6, 8] = eps[6, 9]                                 # exact pair in one column tile
    eps[6, 24] = eps[6, 25] + 1e-9
    assert nb >= 26
    lat2 = synth.Lattice(lat.nk, lat.nc, lat.nb, eps.ravel(), lat.wk, lat.proj)
    return wl, lat2


@pytest.mark.parametrize("nb,var", [(60, 40), (44, 90), (30, 74)])
@pytest.mark.parametrize("nc", [9, 14, 16])
def test_pf_degeneracy_patterns(nc, nb, var):
    from paper_1111_2157_amd.dyson import Context

    wl, lat = crafted(nc=nc, nb=nb)
    c = Context(0)
    nbp = 16 * ((nb + 15) // 16)
    assert var in c.variants(0, nbp)
    c.set_variant(0, nbp, var)
    print("partial fractions, nc", nc, "nb", nb, "variant", var, flush=True)
    mats, gl, sc = gpu_density(c, wl, 0.05, lat=lat)
    assert_nk_parity(mats, lat, wl.sigma, 0.05)
    assert_gloc_parity(gl, lat, wl.sigma, 0.05)
    c.close()


@pytest.mark.parametrize("beta,nw", [(10.0, 30), (100.0, 200)])
def test_pf_temperatures(beta, nw):
    """The threshold scales with the first Matsubara frequency."""
    from paper_1111_2157_amd.dyson import Context

    wl, lat = crafted(nc=14, nb=56, nk=7, nw=nw, beta=beta, seed=9)
    c = Context(0)
    c.set_variant(0, 64, 40)
    print("partial fractions, beta", beta, flush=True)
    mats, gl, sc = gpu_density(c, wl, -0.1, lat=lat)
    assert_nk_parity(mats, lat, wl.sigma, -0.1)
    assert_gloc_parity(gl, lat, wl.sigma, -0.1)
    c.close()


@pytest.mark.parametrize("nc", [1, 3, 5])
@pytest.mark.parametrize("beta", [40.0, 100.0])
@pytest.mark.parametrize("nbs", [(60, 52), (44, 36), (30, 28)])
def test_pf_packed(nc, beta, nbs):
    """Three frequencies per tile (variant 42) on 64-band windows (four
    wavefronts) and on 48- and 32-band windows (one wavefront), with the same
    degeneracy patterns; 100 frequencies leave a partial group (of 48 and 12)."""
    from paper_1111_2157_amd.dyson import Context

    c = Context(0)
    nbp = 16 * ((nbs[0] + 15) // 16)
    assert 42 in c.variants(0, nbp)
    c.set_variant(0, nbp, 42)
    for nb in nbs:
        wl, lat = crafted(nc=nc, nb=nb, nw=100, beta=beta, seed=11 + nc)
        print("partial fractions, packed, nc", nc, "nb", nb, "beta", beta, flush=True)
        mats, gl, sc = gpu_density(c, wl, 0.15, lat=lat)
        assert_nk_parity(mats, lat, wl.sigma, 0.15)
        assert_gloc_parity(gl, lat, wl.sigma, 0.15)
    c.close()
