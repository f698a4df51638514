"""The persistent batched pass over several self-energy iterates with uneven
band windows, eager and replayed from its hipGraph, against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1111_2157_amd import synth
from gpu_util import assert_gloc_parity, assert_nk_parity

pytestmark = pytest.mark.gpu


FORMS = ["dense", "lowrank", "auto"]


def _setup(n_iter=4, nk=10, nw=24, form="auto"):
    from paper_1111_2157_amd.dyson import FORM_AUTO, FORM_DENSE, FORM_LOWRANK, Context, Lattice, SelfEnergy

    wl = synth.batched(nk=nk, nb_lo=14, nb_hi=64, nw=nw, n_iter=n_iter)
    ctx = Context(0)
    lats = [Lattice.from_host(l) for l in wl.lattices]
    sigs = [SelfEnergy.from_host(s) for s in wl.sigmas]
    code = {"dense": FORM_DENSE, "lowrank": FORM_LOWRANK, "auto": FORM_AUTO}[form]
    ctx.batched_set_form(code)
    ctx.batched_plan(lats, sigs, 2)
    if form != "auto":
        assert ctx.batched_form() == code
    else:
        assert ctx.batched_form() in (FORM_DENSE, FORM_LOWRANK)
    return wl, ctx, lats, sigs


def _split(nk_flat, lat):
    out, o = [], 0
    for n in lat.nb:
        n = int(n)
        out.append(nk_flat[o:o + n * n].reshape(n, n))
        o += n * n
    return out


@pytest.mark.parametrize("form", FORMS)
def test_batched_pass_matches_oracle(form):
    import torch

    wl, ctx, lats, sigs = _setup(form=form)
    mus = np.array([0.1, -0.3, 0.25, 0.0][:len(lats)])
    mu_dev = torch.as_tensor(mus, device="cuda")
    nks, gls = ctx.batched_outputs()
    ctx.batched_pass(mu_dev, nks, gls)
    torch.cuda.synchronize()
    ctx.batched_sync_status()
    for s in range(len(lats)):
        print("form", form, "iterate", s, flush=True)
        lat, sig = wl.lattices[s], wl.sigmas[s]
        assert_nk_parity(_split(nks[s].cpu().numpy(), lat), lat, sig, mus[s])
        assert_gloc_parity(gls[s].cpu().numpy(), lat, sig, mus[s])
    ctx.close()


@pytest.mark.parametrize("form", ["dense", "lowrank"])
def test_batched_graph_replays(form):
    import torch

    wl, ctx, lats, sigs = _setup(n_iter=2, nk=8, nw=20, form=form)
    mu_dev = torch.zeros(2, dtype=torch.float64, device="cuda")
    nks, gls = ctx.batched_outputs()
    ctx.batched_graph_capture(mu_dev, nks, gls)
    torch.cuda.synchronize()
    first = [x.clone() for x in nks] + [x.clone() for x in gls]
    results = []
    for rep, mus in enumerate(([0.2, -0.1], [0.0, 0.0], [0.2, -0.1])):
        mu_dev.copy_(torch.as_tensor(mus, dtype=torch.float64))
        torch.cuda.synchronize()
        # eager work on the same stream between replays
        _ = torch.ones(1000, device="cuda").sum()
        ctx.batched_graph_launch()
        torch.cuda.synchronize()
        ctx.batched_sync_status()
        results.append([x.clone() for x in nks] + [x.clone() for x in gls])
        for s in range(2):
            lat, sig = wl.lattices[s], wl.sigmas[s]
            assert_nk_parity(_split(nks[s].cpu().numpy(), lat), lat, sig, mus[s])
            assert_gloc_parity(gls[s].cpu().numpy(), lat, sig, mus[s])
    # replays with the same mu are bitwise equal, and equal to the captured run at mu = 0
    for a, b in zip(results[0], results[2]):
        assert torch.equal(a, b)
    for a, b in zip(results[1], first):
        assert torch.equal(a, b)
    # the eager batched pass gives the same bits as the graph
    mu_dev.copy_(torch.as_tensor([0.2, -0.1], dtype=torch.float64))
    ctx.batched_pass(mu_dev, nks, gls)
    torch.cuda.synchronize()
    for a, b in zip(results[0], list(nks) + list(gls)):
        assert torch.equal(a, b)
    ctx.close()


def test_batched_class_launch_orders_agree():
    """The low-rank plan's class kernels run concurrently on side streams or one
    after another on the pass's stream; both orders (eager and replayed from the
    graph) give the same bits, since every class writes its own partials, and
    they match the oracle."""
    import torch
    from paper_1111_2157_amd.dyson import FORM_LOWRANK, Context, Lattice, SelfEnergy

    wl = synth.batched(nk=10, nb_lo=14, nb_hi=64, nw=24, n_iter=2)
    lats = [Lattice.from_host(l) for l in wl.lattices]
    sigs = [SelfEnergy.from_host(s) for s in wl.sigmas]
    mus = [0.15, -0.2]
    outs = {}
    for mode in (1, 0, -1):
        print("concurrency mode", mode, flush=True)
        ctx = Context(0)
        ctx.batched_set_form(FORM_LOWRANK)
        ctx.batched_set_concurrent(mode)
        ctx.batched_plan(lats, sigs, 2)
        assert len(ctx.batched_classes()) > 1
        if mode >= 0:
            assert ctx.batched_concurrent() == mode
        else:
            assert ctx.batched_concurrent() in (0, 1)
        mu_dev = torch.as_tensor(mus, dtype=torch.float64, device="cuda")
        nks, gls = ctx.batched_outputs()
        ctx.batched_pass(mu_dev, nks, gls)
        torch.cuda.synchronize()
        ctx.batched_sync_status()
        eager = [x.clone() for x in list(nks) + list(gls)]
        ctx.batched_graph_capture(mu_dev, nks, gls)
        torch.cuda.synchronize()
        ctx.batched_sync_status()
        for a, b in zip(eager, list(nks) + list(gls)):
            assert torch.equal(a, b)
        outs[mode] = eager
        ctx.close()
    for a, b, c in zip(outs[1], outs[0], outs[-1]):
        assert torch.equal(a, b) and torch.equal(a, c)
    for s in range(2):
        lat, sig = wl.lattices[s], wl.sigmas[s]
        assert_nk_parity(_split(outs[0][s].cpu().numpy(), lat), lat, sig, mus[s])
        assert_gloc_parity(outs[0][2 + s].cpu().numpy(), lat, sig, mus[s])
    ctx = Context(0)
    with pytest.raises(Exception):
        ctx.batched_set_concurrent(2)
    ctx.close()


def test_batched_tile_candidate_choice():
    """dmft_batched_set_tile_candidate: candidate 0 (the default tiles) is taken
    without timing the others and reported back, and the pass matches the
    oracle; an index past the plan's list restores the timing; an index below
    -1 is refused."""
    import torch
    from paper_1111_2157_amd._lib import DmftError
    from paper_1111_2157_amd.dyson import FORM_LOWRANK, Context, Lattice, SelfEnergy

    wl = synth.batched(nk=10, nb_lo=14, nb_hi=64, nw=24, n_iter=2)
    lats = [Lattice.from_host(l) for l in wl.lattices]
    sigs = [SelfEnergy.from_host(s) for s in wl.sigmas]
    ctx = Context(0)
    ctx.batched_set_form(FORM_LOWRANK)
    assert ctx.batched_tile_candidate() == -1
    with pytest.raises(DmftError):
        ctx.batched_set_tile_candidate(-2)
    mus = [0.05, -0.15]
    for pick in (0, 99):
        print("tile candidate", pick, flush=True)
        ctx.batched_set_tile_candidate(pick)
        ctx.batched_plan(lats, sigs, 2)
        got = ctx.batched_tile_candidate()
        assert got == 0 if pick == 0 else got >= 0
        mu_dev = torch.as_tensor(mus, dtype=torch.float64, device="cuda")
        nks, gls = ctx.batched_outputs()
        ctx.batched_pass(mu_dev, nks, gls)
        torch.cuda.synchronize()
        ctx.batched_sync_status()
        for s in range(2):
            lat, sig = wl.lattices[s], wl.sigmas[s]
            assert_nk_parity(_split(nks[s].cpu().numpy(), lat), lat, sig, mus[s])
            assert_gloc_parity(gls[s].cpu().numpy(), lat, sig, mus[s])
    ctx.close()
