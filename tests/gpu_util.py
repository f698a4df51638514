"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and compare it with the oracle, normwise per k and per frequency."""
import numpy as np

import oracle

RTOL = 1e-10


def relerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu_density(ctx, wl, mu, tail=2, sig_index=0, lat=None):
    import torch

    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy, split_nk

    host_lat = lat if lat is not None else (wl.lattices[sig_index] if wl.lattices else wl.lattice)
    dlat = Lattice.from_host(host_lat)
    dsig = SelfEnergy.from_host(wl.sigmas[sig_index])
    nk, gl, sc = ctx.density_matrix(dlat, dsig, mu, tail)
    torch.cuda.synchronize()
    ctx.sync_status()
    mats = [m.cpu().numpy() for m in split_nk(nk, dlat)]
    return mats, gl.cpu().numpy(), sc.cpu().numpy()


def assert_nk_parity(mats_gpu, lat, sig, mu, tail=2, klist=None, rtol=RTOL):
    ks = list(range(lat.nk)) if klist is None else list(klist)
    ref, _ = oracle.density(lat, sig, mu, tail, klist=ks)
    worst = 0.0
    for i, k in enumerate(ks):
        e = relerr(mats_gpu[k], ref[i])
        worst = max(worst, e)
        assert e <= rtol, "N(k=%d): rel err %.3e" % (k, e)
    return worst


def assert_gloc_parity(gl_gpu, lat, sig, mu, nlist=None, rtol=RTOL):
    ns = list(range(sig.nw)) if nlist is None else list(nlist)
    ref = oracle.gloc(lat, sig, mu, ns)
    worst = 0.0
    for i, n in enumerate(ns):
        e = relerr(gl_gpu[n], ref[i])
        worst = max(worst, e)
        assert e <= rtol, "G_loc(n=%d): rel err %.3e" % (n, e)
    return worst
