"""GPU tests of the device error word and the host checks on a real handle:
a vanishing pivot (DMFT_ESINGULAR), a bracket without the target
(DMFT_ENOCONV, stopping early), and a workspace that is missing, misaligned or
too small (DMFT_EWORKSPACE).  Every kernel here exits normally; only the error
word reports the condition."""
import ctypes as C

import numpy as np
import pytest

from paper_1111_2157_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1111_2157_amd.dyson import Context

    c = Context(0)
    yield c
    c.close()


def singular_case(nw=1):
    """One band, one orbital, S = [1], E = -1, mu = 0, V_DC = 0, beta = pi, so
    w_0 = pi / beta = 1 and i w_0 + mu - E = 1 + i exactly.  Sigma(i w_0) = 1 + i
    makes A = (1 + i) - Sigma exactly zero (dense form); in the low-rank form
    X = 1/(1 + i) = (1 - i)/2 and X^-1 = 1 + i are exact in binary, so
    K = X^-1 - Sigma is exactly zero too.  Later frequencies get Sigma = 0."""
    lat = synth.Lattice(1, 1, np.array([1], np.int32), np.array([-1.0]), np.array([1.0]), np.array([1.0 + 0j]))
    s = np.zeros((nw, 1, 1), np.complex128)
    s[0, 0, 0] = 1.0 + 1.0j
    sig = synth.SelfEnergy(nw, float(np.pi), s, None, np.zeros(1), [])
    return lat, sig


@pytest.mark.parametrize("form", ["dense", "lowrank"])
def test_vanishing_pivot_reports_esingular(ctx, form):
    import torch

    from paper_1111_2157_amd._lib import DmftError
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    lat, sig = singular_case()
    dl, ds = Lattice.from_host(lat), SelfEnergy.from_host(sig)
    for kind in (0, 1):
        codes = [v for v in ctx.variants(kind, 16) if bool(v & 8) == (form == "lowrank")]
        assert codes, (kind, form)
        ctx.set_variant(kind, 16, codes[0])
    print("singular pivot", form, flush=True)
    ctx.density_matrix(dl, ds, 0.0)
    with pytest.raises(DmftError) as e:
        ctx.sync_status()
    assert e.value.name == "DMFT_ESINGULAR"
    ctx.sync_status()  # cleared
    ctx.dmft_ntot(dl, ds, 0.0)
    torch.cuda.synchronize()
    with pytest.raises(DmftError) as e:
        ctx.sync_status()
    assert e.value.name == "DMFT_ESINGULAR"
    # find_mu reports it from the pass that hit it (its bracket is centred on 0)
    with pytest.raises(DmftError) as e:
        ctx.find_mu(dl, ds, 0.5, 1e-8, 1, -1.0, 1.0)
    assert e.value.name == "DMFT_ESINGULAR"
    ctx.sync_status()
    # a regular Sigma on the same lattice is fine afterwards
    sig.sigma[0, 0, 0] = 0.3 - 0.2j
    ctx.density_matrix(dl, SelfEnergy.from_host(sig), 0.0)
    ctx.sync_status()
    for kind in (0, 1):
        ctx.set_variant(kind, 16, -1)


def test_vanishing_pivot_in_the_batched_pass(ctx):
    import torch

    from paper_1111_2157_amd._lib import DmftError
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    lat, sig = singular_case(nw=4)
    ok = synth.plain(nk=3, nb=6, nc=2, nw=4, beta=float(np.pi))
    lats = [Lattice.from_host(ok.lattice), Lattice.from_host(lat)]
    sigs = [SelfEnergy.from_host(ok.sigma), SelfEnergy.from_host(sig)]
    ctx.batched_plan(lats, sigs, 2)
    nks, gls = ctx.batched_outputs()
    mu = torch.zeros(2, dtype=torch.float64, device="cuda")
    ctx.batched_pass(mu, nks, gls)
    with pytest.raises(DmftError) as e:
        ctx.batched_sync_status()
    assert e.value.name == "DMFT_ESINGULAR"
    ctx._b_ws = None


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("target", [30.0, -5.0])
def test_find_mu_without_bracket_stops_early(ctx, method, target):
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = synth.plain(nk=8, nw=64)  # 12 bands: 0 < N < 12 for every mu
    dl, ds = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
    ws, nws = ctx._call_ws(dl, ds)
    ls, ss = dl.struct(), ds.struct()
    mu, passes, n = C.c_double(), C.c_int(), C.c_double()
    r = ctx.lib.find_mu(ctx.h, C.byref(ls), C.byref(ss), 2, C.c_double(target), C.c_double(1e-8), method,
                        C.c_double(-40.0), C.c_double(40.0), C.c_double(0.0), 300, C.byref(mu), C.byref(passes),
                        C.byref(n), C.c_void_p(ws.data_ptr()), nws, C.c_void_p(0))
    print("no bracket", method, target, r, passes.value, mu.value, n.value, flush=True)
    assert r == -5  # DMFT_ENOCONV
    assert "does not bracket" in ctx.lib.dmft_last_error(ctx.h).decode()
    assert passes.value <= 70, passes.value
    assert abs(mu.value - (40.0 if target > 0 else -40.0)) < 1e-12
    assert (n.value < target) if target > 0 else (n.value > target)


def test_workspace_missing_misaligned_or_short(ctx):
    import torch

    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = synth.plain(nk=4, nw=16)
    dl, ds = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
    need = ctx.workspace_size(dl, ds)
    buf = torch.zeros(need + 512, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr()
    assert base % 256 == 0
    nk = torch.empty(dl.n_size(), dtype=torch.complex128, device="cuda")
    ls, ss = dl.struct(), ds.struct()

    def call(ptr, nbytes):
        return ctx.lib.density_matrix(ctx.h, C.byref(ls), C.byref(ss), C.c_double(0.0), 2,
                                      C.c_void_p(nk.data_ptr()), None, None, ptr, C.c_size_t(nbytes),
                                      C.c_void_p(0))

    assert call(None, need) == -6
    assert call(C.c_void_p(base + 8), need) == -6
    assert call(C.c_void_p(base), need - 1) == -6
    assert "too small" in ctx.lib.dmft_last_error(ctx.h).decode()
    assert call(C.c_void_p(base), need) == 0
    torch.cuda.synchronize()
    ctx.sync_status()


@pytest.mark.parametrize("nc", [3, 8])
def test_nonfinite_pass_leaves_no_trace(nc):
    """A pass whose self-energy holds NaN fills the LDS of every CU it ran on
    with non-finite values; the next, regular pass of the same shape (nc <= 8:
    two frequencies per X product, which leaves rows 8 .. 15 of the staged tile
    unwritten) must report no error and match the oracle."""
    from gpu_util import assert_gloc_parity, assert_nk_parity, gpu_density
    from paper_1111_2157_amd._lib import DmftError
    from paper_1111_2157_amd.dyson import Context, Lattice, SelfEnergy

    wl = synth.f_shell(nk=384, nb=30, nc=nc, nw=64, n_narrow=6)
    c = Context(0)
    for nbp in (16, 32):
        lr = [v for v in c.variants(0, nbp) if v & 8 and v != 42]
        c.set_variant(0, nbp, lr[0])
    bad = wl.sigma.sigma.copy()
    bad[:, 0, 0] = np.nan
    s_bad = synth.SelfEnergy(wl.sigma.nw, wl.sigma.beta, bad, wl.sigma.sigma_inf, wl.sigma.e_dc)
    print("non-finite pass then regular pass, nc", nc, flush=True)
    c.density_matrix(Lattice.from_host(wl.lattice), SelfEnergy.from_host(s_bad), 0.1)
    with pytest.raises(DmftError) as e:
        c.sync_status()
    assert e.value.name == "DMFT_ENONFINITE"
    mats, gl, sc = gpu_density(c, wl, 0.1)  # raises on a flagged error word
    ks = list(range(0, wl.lattice.nk, 37))
    assert_nk_parity(mats, wl.lattice, wl.sigma, 0.1, klist=ks)
    assert_gloc_parity(gl, wl.lattice, wl.sigma, 0.1, nlist=[0, 1, 31, 63])
    c.close()
