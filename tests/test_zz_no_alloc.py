"""GPU test of the allocation-free entry point density_matrix_noalloc, called
through the C ABI: two calls in a row on the library's shared scratch (the
second with a smaller input), each checked against density_matrix on a
caller-owned workspace and against the oracle; a shape beyond the scratch is
rejected before any launch."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1111_2157_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-10


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def noalloc(ctx, dl, ds, mu, tail=2):
    import torch

    nk = torch.full((dl.n_size(),), float("nan"), dtype=torch.complex128, device="cuda")
    gl = torch.full((ds.nw, dl.nc, dl.nc), float("nan"), dtype=torch.complex128, device="cuda")
    sc = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
    st = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    ls, ss = dl.struct(), ds.struct()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    r = ctx.lib.density_matrix_noalloc(ctx.h, C.byref(ls), C.byref(ss), C.c_double(mu), tail,
                                       C.c_void_p(nk.data_ptr()), C.c_void_p(gl.data_ptr()),
                                       C.c_void_p(sc.data_ptr()), C.c_void_p(st.data_ptr()), stream)
    torch.cuda.synchronize()
    return r, nk, gl, sc, int(st.item())


def test_noalloc_matches_density_matrix_twice():
    from paper_1111_2157_amd.dyson import Context, Lattice, SelfEnergy, split_nk

    ctx = Context(0)
    cases = [(synth.d_shell(nk=24, nw=96), 0.3), (synth.f_shell(nk=6, nb=20, nc=14, nw=40, n_narrow=6), -0.2)]
    for wl, mu in cases:
        print("noalloc case", wl.name, flush=True)
        dl, ds = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
        r, nk, gl, sc, st = noalloc(ctx, dl, ds, mu)
        assert r == 0, ctx.lib.dmft_last_error(ctx.h).decode()
        assert st == 0
        ref_nk, ref_gl, ref_sc = ctx.density_matrix(dl, ds, mu)
        ctx.sync_status()
        for a, b in zip(split_nk(nk, dl), split_nk(ref_nk, dl)):
            assert relerr(a.cpu().numpy(), b.cpu().numpy()) <= 1e-12
        for n in range(ds.nw):
            assert relerr(gl[n].cpu().numpy(), ref_gl[n].cpu().numpy()) <= 1e-12
        assert np.allclose(sc.cpu().numpy(), ref_sc.cpu().numpy(), rtol=1e-12, atol=0)
        # and the oracle, on a few k-points and frequencies
        ks = [0, wl.lattice.nk - 1]
        ref, _ = oracle.density(wl.lattice, wl.sigma, mu, 2, klist=ks)
        mats = split_nk(nk, dl)
        for i, k in enumerate(ks):
            assert relerr(mats[k].cpu().numpy(), ref[i]) <= RTOL
        g = oracle.gloc(wl.lattice, wl.sigma, mu, [0, ds.nw - 1])
        assert relerr(gl[0].cpu().numpy(), g[0]) <= RTOL
        assert relerr(gl[ds.nw - 1].cpu().numpy(), g[1]) <= RTOL
    ctx.close()


def test_noalloc_reports_device_errors_and_rejects_oversize():
    import torch

    from paper_1111_2157_amd.dyson import Context, Lattice, SelfEnergy

    ctx = Context(0)
    # a vanishing pivot (see test_gpu_errors.singular_case): status says so
    lat = synth.Lattice(1, 1, np.array([1], np.int32), np.array([-1.0]), np.array([1.0]), np.array([1.0 + 0j]))
    sig = synth.SelfEnergy(1, float(np.pi), np.array([[[1.0 + 1.0j]]]), None, np.zeros(1), [])
    r, _, _, _, st = noalloc(ctx, Lattice.from_host(lat), SelfEnergy.from_host(sig), 0.0)
    assert r == 0 and st == -4  # DMFT_ESINGULAR
    # the next call starts from a cleared error word
    wl = synth.plain(nk=4, nw=16)
    r, _, _, _, st = noalloc(ctx, Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma), -1.0)
    assert r == 0 and st == 0
    # ragged windows are refused
    rg = synth.batched(nk=6, nb_lo=14, nb_hi=30, nw=8, n_iter=1)
    r, *_ = noalloc(ctx, Lattice.from_host(rg.lattices[0]), SelfEnergy.from_host(rg.sigmas[0]), 0.0)
    assert r == -1 and "uniform band windows" in ctx.lib.dmft_last_error(ctx.h).decode()
    # a shape whose smallest layout exceeds the scratch is refused before any launch
    big = synth.f_shell(nk=2048, nb=64, nc=14, nw=8)  # sum_n G partials alone: 2048 x 64^2 x 16 B = 128 MiB
    dl, ds = Lattice.from_host(big.lattice), SelfEnergy.from_host(big.sigma)
    r, *_ = noalloc(ctx, dl, ds, 0.0)
    assert r == -6 and "allocation-free scratch" in ctx.lib.dmft_last_error(ctx.h).decode()
    torch.cuda.synchronize()
    ctx.close()
