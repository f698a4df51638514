#!/usr/bin/env python3
"""Benchmark of the lattice Dyson step on one MI355X.

A step is one full pass of the hot path over the batched workload: 8
self-energy iterates (4 with Nc = 5, 4 with Nc = 14) on Nk = 4096 k-points whose
band windows are drawn from U{20..64}, beta = 40/eV, Nw = 2048 positive
Matsubara frequencies, complex128.  For every iterate, k and frequency the
pass builds A(k, i w_n), inverts it (low-rank form), projects to G_loc and
Matsubara-sums N(k) with the analytic tail -- the batched plan's persistent
launches, replayed from the hipGraph they were captured into.  Inputs are
seeded synthetic arrays resident in HBM before the timed region starts.

The JSON line also carries
  * "roofline": achieved FP64 rate of the batched Dyson section (the class
    kernels of one pass, which run concurrently) from its average duration,
    measured with hipEvents captured into the graph around it and read after
    every replay of the timed region, against the MI355X FP64 peak; the
    algorithmic count is the low-rank form's 8 (Nb^2 Nc + 2 Nb Nc^2 + 5 Nc^3)
    flop per (k, i w_n) evaluation, summed over the ragged windows;
  * "cpu_baseline": the FP64 CPU oracle timed on a bounded k-sample of every
    iterate on this host's cores;
  * "mu_search": Newton (dN/dmu from the adjoint trace pass) against
    bisection, same kernels, bracket [-40, 40] eV, start at its midpoint,
    stop at |N - N0| < 1e-8, on the differentiation workload (Nk=1024, Nb=40,
    Nc=14, beta=50, Nw=2048, N0=20);
  * "workloads": the d-shell and f-shell density passes and the differentiation
    workload's fused forward + adjoint pass, each with its own kernel rate.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
# LDS bandwidth of the chip: 256 CUs x 128 B/clk x 2.4 GHz
LDS_PEAK_TBPS = 256 * 128 * 2.4e9 / 1e12

# HBM traffic of the batched Dyson section per pass: the sum over its class
# kernels of rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch, scaled
# by 2 and 1, the factors a plain 1 GiB copy reads under --copy-calibration),
# recorded in the profile named below.  Valid only for the kernel sources it
# was measured on (their SHA-256) and the same workload, form and item classes
# (padded size, inversion columns, items); otherwise "traffic" is null.
TRAFFIC_SOURCES = ["paper_1111_2157_amd/csrc/lowrank_impl.h", "paper_1111_2157_amd/csrc/lowrank_pair_impl.h",
                   "paper_1111_2157_amd/csrc/lowrank_p3_impl.h",
                   "paper_1111_2157_amd/csrc/batched_lr.h", "paper_1111_2157_amd/csrc/dyson_impl.h",
                   "paper_1111_2157_amd/csrc/batched_lr16.hip", "paper_1111_2157_amd/csrc/batched_lr32.hip",
                   "paper_1111_2157_amd/csrc/batched_lr48.hip", "paper_1111_2157_amd/csrc/batched_lr64.hip"]
TRAFFIC = {
    ("batched-Nk4096-Nb20..64-x8-Nw2048", "low-rank",
     ((32, 5, 5256), (32, 14, 5256), (48, 5, 6552), (48, 14, 6552), (64, 5, 6660), (64, 14, 6660))): {
        "bytes": 244.49e9,  # FETCH 109.96 GB + WRITE 134.52 GB
        "profile": "profiles/batched_cfg4.md",
        "sources_sha256": "de41587efc8a209589a8d114de9e1f41446dd861fb72014a234b37fdaca0f207",
    },
    # the plan's quarter k-tile with the default frequency tile of 256
    ("batched-Nk4096-Nb20..64-x8-Nw2048", "low-rank",
     ((32, 5, 4672), (32, 14, 4672), (48, 5, 5824), (48, 14, 5824), (64, 5, 5920), (64, 14, 5920))): {
        "bytes": 243.15e9,  # FETCH 110.09 GB + WRITE 133.06 GB
        "profile": "profiles/batched_cfg4.md",
        "sources_sha256": "de41587efc8a209589a8d114de9e1f41446dd861fb72014a234b37fdaca0f207",
    },
}


def class_key(classes):
    return tuple(sorted((c["nbp"], c["ncls"], c["items"]) for c in classes))


def sources_sha256():
    import hashlib

    h = hashlib.sha256()
    for p in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, form, classes):
    """Counter-measured HBM bytes per pass of the class kernels, or None."""
    rec = TRAFFIC.get((workload, form, class_key(classes)))
    if rec is None or rec["sources_sha256"] != sources_sha256():
        return None
    return rec


def flops_per_eval(nb, nc):
    """Algorithmic FP64 flops of one (k, i w_n) evaluation in the dense form:
    embed S^dag Sigma' S (Nb^2 Nc + Nb Nc^2 complex MACs), invert (Nb^3), project
    S G S^dag (Nb^2 Nc + Nb Nc^2); 8 real flops per complex multiply-add."""
    return 8.0 * (nb ** 3 + 2.0 * nb * nb * nc + 2.0 * nb * nc * nc)


def flops_per_eval_lowrank(nb, nc):
    """Algorithmic FP64 flops of one density-pass evaluation in the low-rank
    (Woodbury) form, 8 (Nb^2 Nc + 2 Nb Nc^2 + 5 Nc^3): X = S D S^dag and R S
    (Nb Nc^2 complex multiply-adds each), D S^dag (R S D) (Nb^2 Nc), and the
    nc x nc work -- two inversions, R = Sigma' + Sigma' Gl Sigma', the G_loc
    share -- counted as 5 Nc^3; 8 real flops per complex multiply-add."""
    return 8.0 * (nb * nb * nc + 2.0 * nb * nc * nc + 5.0 * nc ** 3)


def density_kernel(ctx, nb, nc):
    """(kernel name, algorithmic flops per evaluation) of the density-pass
    kernel the context will run for this band window."""
    nbp = (nb + 15) // 16 * 16
    var = ctx.get_variant(0, nbp)
    if var >= 0 and var & 8:
        return "lr_kernel<%d, density> (low-rank, variant %d)" % (nbp, var), flops_per_eval_lowrank(nb, nc)
    if nbp == 64:
        return "d64::kernel<density> (variant %d)" % var, flops_per_eval(nb, nc)
    return "dyson_kernel<%d, density> (variant %d)" % (nbp, var), flops_per_eval(nb, nc)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mu", action="store_true", help="skip the mu-search comparison")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the d-shell, f-shell and fused-adjoint passes")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU oracle sample time")
    ap.add_argument("--extra", action="store_true",
                    help="also time the general VJP, the pole route, the self-consistency step and the atom")
    ap.add_argument("--section", choices=["pole", "sc", "atom", "adj", "d-shell", "f-shell"], default=None,
                    help="time only the pole route, the self-consistency step, the atom and energy "
                         "sums, the two adjoint passes or the autotuned density pass of the d-shell "
                         "or f-shell workload, and print that record")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (use the default variants)")
    ap.add_argument("--plan-candidate", type=int, default=-1,
                    help="batched plan: take this tile candidate without timing the others "
                         "(reproducible profiles; -1, the default, times every candidate)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device-to-device three times (reference for the HBM byte counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain device copy of known size: under rocprofv3 --pmc FETCH_SIZE /
    WRITE_SIZE it gives the factors that turn those counters into bytes."""
    import torch

    x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
    y = torch.empty_like(x)
    x.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_per_copy": x.numel() * 8, "copies": 3}}), flush=True)


def time_density(ctx, lat, sig, mu, steps, warmup, tail=2):
    import torch

    for _ in range(warmup):
        ctx.density_matrix(lat, sig, mu, tail)
    torch.cuda.synchronize()
    ctx.sync_status()
    ctx.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.density_matrix(lat, sig, mu, tail)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, launches = ctx.timing(False)
    ctx.sync_status()
    return (t1 - t0) / steps, kms, launches


def host_cpu():
    """Model name of the host CPU (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_nproc():
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count()


def cpu_baseline(wl, mu, target_s):
    """The FP64 oracle (N(k) of every iterate) on this host's cores -- OpenMP
    over k with ORACLE_THREADS threads, else the host's cores up to 16, the CPU
    share of one GPU on the machines this runs on -- over the first m k-points
    of each of the batched workload's iterates, all frequencies; m is sized
    for about target_s seconds.  The rate is evaluations per second of that
    sample, which scales linearly (every (k, i w_n) evaluation is independent),
    plus a single-thread rate on a smaller sample."""
    import oracle

    lats, sigs = wl.lattices, wl.sigmas
    cores = int(os.environ.get("ORACLE_THREADS", min(16, host_nproc() or 1)))

    def run(m, threads):
        t0 = time.perf_counter()
        for lat, sig in zip(lats, sigs):
            oracle.density(lat, sig, mu, 2, klist=list(range(m)), nthreads=threads)
        return time.perf_counter() - t0

    t_cal = run(1, 1)  # one k of each iterate on one thread
    m = int(max(1, min(lats[0].nk, target_s / max(t_cal, 1e-3) * cores * 0.8)))
    m = max(cores, (m // cores) * cores)
    t = run(m, cores)
    evals = m * sum(s.nw for s in sigs)
    m1 = int(max(1, min(lats[0].nk, (target_s / 4) / max(t_cal, 1e-3))))
    t1 = run(m1, 1)
    return {"value": evals / t, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": "N(k) of the first %d k-points of each of the %d iterates over all %d frequencies "
                      "(%d evals, %.1f s); G_loc not formed" % (m, len(lats), sigs[0].nw, evals, t),
            "single_thread": {"value": m1 * sum(s.nw for s in sigs) / t1, "unit": "evals/s",
                              "sample": "first %d k-points of each iterate, %.1f s" % (m1, t1)},
            "host_cpu": host_cpu(), "host_nproc": host_nproc(), "host_cpu_count": os.cpu_count()}


def adjoint_pass(ctx, tune=True):
    """Forward + fused scalar adjoint (N_tot, dN/dmu, dN/dSigma in one pass) on
    the differentiation workload."""
    import torch

    from paper_1111_2157_amd import synth
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = synth.differentiation()
    lat, sig = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
    mu = -0.8
    ctx.dmft_ntot_vjp(lat, sig, mu)  # warm-up
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.dmft_ntot_vjp(lat, sig, mu)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    nb, nc = wl.lattice.nb_max, wl.lattice.nc
    nbp = (nb + 15) // 16 * 16
    evals = wl.lattice.nk * wl.sigma.nw
    var = ctx.get_variant(2, nbp)
    lowrank = var >= 0 and bool(var & 8)
    # dense form: forward (embed + invert + project) plus the adjoint's extra work;
    # low-rank form: X, X2, X3 (3 Nb Nc^2), two inversions, R, R X2 and the four
    # Nc x Nc products of S G^2 S^dag (9 Nc^3)
    dense_fl = 8.0 * (nb ** 3 + 2 * nb * nb * nc + 2 * nb * nc * nc) + 8.0 * (nb * nb * nc + nb * nc * nc + nb * nb)
    fl = 8.0 * (3 * nb * nc * nc + 9 * nc ** 3) if lowrank else dense_fl
    return {"workload": wl.name, "evals_per_s": evals / sec, "ms_per_pass": sec * 1e3,
            "form": "low-rank" if lowrank else "dense", "variant": var, "flop_per_eval": fl,
            "tflops": fl * evals / sec / 1e12, "tflops_dense_count": dense_fl * evals / sec / 1e12}


def general_vjp_pass(ctx):
    """Forward + general vector-Jacobian product (`density_matrix_vjp`: Sigma-bar
    and mu-bar for upstream N(k)-bar and G_loc-bar cotangents, both given) on the
    differentiation workload, in the form the context selects (low-rank by
    default).  Complex multiply-adds per evaluation:
      low-rank: X and X2 (2 Nb Nc^2), Nt D S^dag and Nt D^2 S^dag (2 Nb^2 Nc),
        P1 and P2 (3 Nb Nc^2), fifteen Nc x Nc products and inversions (15 Nc^3);
      dense: the forward (S^dag Sigma' S, the inversion, W = S G, Z = G S^dag,
        M = W Z: Nb^3 + 2 Nb^2 Nc + 2 Nb Nc^2) and the product (Y = Nt W^dag,
        Z^dag Y, X = W S^dag, X^dag Gbar X^dag, Nt G: Nb^3 + Nb^2 Nc + 2 Nb Nc^2
        + 2 Nc^3);
    8 flop each."""
    import numpy as np
    import torch

    from paper_1111_2157_amd import synth
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    wl = synth.differentiation()
    lat, sig = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
    mu = -0.8
    rng = np.random.default_rng(7)
    nbar = np.concatenate([(rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)) for n in wl.lattice.nb])
    gbar = rng.standard_normal(wl.sigma.sigma.shape) + 1j * rng.standard_normal(wl.sigma.sigma.shape)
    nbt, gbt = torch.as_tensor(nbar, device="cuda"), torch.as_tensor(gbar, device="cuda")
    ctx.density_matrix_vjp(lat, sig, mu, nbt, gbt)  # warm-up
    torch.cuda.synchronize()
    ctx.sync_status()
    reps = 3
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.density_matrix_vjp(lat, sig, mu, nbt, gbt)
    e1.record()
    torch.cuda.synchronize()
    ctx.sync_status()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    nb, nc = wl.lattice.nb_max, wl.lattice.nc
    nbp = (nb + 15) // 16 * 16
    var = ctx.get_variant(3, nbp)
    lowrank = var >= 0 and bool(var & 8)
    evals = wl.lattice.nk * wl.sigma.nw
    dense_fl = 8.0 * (2 * nb ** 3 + 3 * nb * nb * nc + 4 * nb * nc * nc + 2 * nc ** 3)
    fl = 8.0 * (2 * nb * nb * nc + 5 * nb * nc * nc + 15 * nc ** 3) if lowrank else dense_fl
    return {"workload": wl.name, "evals_per_s": evals / sec, "ms_per_pass": sec * 1e3,
            "form": "low-rank" if lowrank else "dense", "variant": var, "flop_per_eval": fl,
            "tflops": fl * evals / sec / 1e12, "tflops_dense_count": dense_fl * evals / sec / 1e12}


def adjoint_section(ctx, tune):
    """The fused scalar adjoint and the general VJP on the differentiation
    workload, after autotuning it (as the --extra run does)."""
    from paper_1111_2157_amd import synth
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    if tune:
        w = synth.differentiation()
        ctx.autotune(Lattice.from_host(w.lattice), SelfEnergy.from_host(w.sigma), w.mu)
    return {"fused": adjoint_pass(ctx), "general": general_vjp_pass(ctx)}


def self_consistency(ctx):
    """The DMFT self-consistency step (E_imp and Delta from G_loc) on the d-shell
    and f-shell workloads: microseconds per call from events on the stream it
    runs on, and the rate of its algorithmic HBM bytes (read G_loc and Sigma,
    write Delta: 3 Nw Nc^2 complex; read the projectors and band energies
    once for E_imp)."""
    import torch

    from paper_1111_2157_amd import synth
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    out = {}
    for w in (synth.d_shell(), synth.f_shell()):
        lat, sig = Lattice.from_host(w.lattice), SelfEnergy.from_host(w.sigma)
        gl = ctx.gloc_compute(lat, sig, w.mu)
        ctx.hybridization(lat, sig, w.mu, gl)
        torch.cuda.synchronize()
        ctx.sync_status()
        reps = 50
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ctx.hybridization(lat, sig, w.mu, gl)
        e1.record()
        torch.cuda.synchronize()
        ctx.sync_status()
        us = e0.elapsed_time(e1) * 1e3 / reps
        nk, nc, nw = w.lattice.nk, w.lattice.nc, sig.nw
        nbs = int(w.lattice.nb.astype(np.int64).sum())
        nbytes = 3 * nw * nc * nc * 16 + nbs * (nc * 16 + 8) + nk * 8
        out[w.name] = {"us_per_call": us, "algorithmic_bytes": nbytes, "gbps": nbytes / us / 1e3}
        del gl
    return out


def _event_ms(fn, reps):
    import torch

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def jacobi_step_cost(nb, npl):
    """FP64 flops and LDS bytes of one Jacobi step (every pair rotating) for one
    k with nb bands and npl poles, with the matrix stored as its packed upper
    triangle: m/2 (m/2 - 1)/2 off-diagonal 2x2 blocks (8 complex
    scale-and-rotate updates of 10 flops, 4 reads and 4 writes of 16 B), m/2
    diagonal blocks (3 writes) and m/2 nb eigenvector pairs (2 updates, 2 reads,
    2 writes); m = nb + npl rounded up to even."""
    m = nb + npl
    m += m & 1
    p = m // 2
    flops = p * (p - 1) // 2 * 80 + p * nb * 20
    lds = (p * (p - 1) // 2 * 8 + p * 3 + p * nb * 4) * 16
    return flops, lds, m


def pole_route(ctx, tune=True):
    """The pole-expansion route on the d-shell and f-shell workloads: batched
    pseudo-Hamiltonian eigensystems, exact N(k), the mu search from the
    eigenvalues (Newton and bisection) and a 1001-point DOS/PDOS; the
    eigensolver's rate against the LDS and FP64 peaks (work counted per Jacobi
    step actually taken), and the route's time against one frequency-sum
    density pass of the same workload."""
    import dataclasses

    import torch

    from paper_1111_2157_amd import synth
    from paper_1111_2157_amd.dyson import BISECT, NEWTON, Lattice, PoleSelfEnergy, SelfEnergy

    out = {}
    for w in (synth.d_shell(), synth.f_shell()):
        sig = w.sigma
        sig_abs = dataclasses.replace(sig, poles=[(p + w.mu, v) for p, v in sig.poles])
        lat, pol = Lattice.from_host(w.lattice), PoleSelfEnergy.from_host(sig_abs)
        es = ctx.pole_eig(lat, pol)
        torch.cuda.synchronize()
        ctx.sync_status()
        t_eig = _event_ms(lambda: ctx.pole_eig(lat, pol), 5)
        ctx.sync_status()
        sweeps = ctx.pole_sweeps(lat, pol)
        nb, npl = w.lattice.nb_max, len(sig.poles)
        fl, lb, m = jacobi_step_cost(nb, npl)
        steps = int(sweeps.sum()) * (m - 1)
        t_den = _event_ms(lambda: ctx.pole_density(lat, pol, es, w.mu, 0), 10)
        _, sc = ctx.pole_density(lat, pol, es, w.mu, 0)
        n0 = float(sc[0]) + 0.5
        t0 = time.perf_counter()
        mu_n, pn, _ = ctx.pole_find_mu(lat, pol, es, n0, 1e-8, NEWTON)
        t_newton = time.perf_counter() - t0
        t0 = time.perf_counter()
        mu_b, pb, _ = ctx.pole_find_mu(lat, pol, es, n0, 1e-8, BISECT)
        t_bisect = time.perf_counter() - t0
        t_dos = _event_ms(lambda: ctx.pole_dos(lat, pol, es, w.mu, 0.05, -12.0, 12.0, 1001), 3)
        ctx.sync_status()
        s2 = SelfEnergy.from_host(sig)
        if tune:
            ctx.autotune(lat, s2, w.mu)
        t_mats, _, _ = time_density(ctx, lat, s2, w.mu, 3, 1)
        lds_tbps = steps * lb / (t_eig * 1e-3) / 1e12
        tflops = steps * fl / (t_eig * 1e-3) / 1e12
        out[w.name] = {
            "m": nb + npl, "eig_ms": t_eig, "sweeps_mean": float(sweeps.mean()), "sweeps_max": int(sweeps.max()),
            "density_exact_ms": t_den, "eig_plus_density_ms": t_eig + t_den,
            "frequency_sum_density_ms": t_mats * 1e3,
            "speedup_vs_frequency_sum": t_mats * 1e3 / (t_eig + t_den),
            "find_mu_newton": {"mu": mu_n, "passes": pn, "seconds": t_newton},
            "find_mu_bisect": {"mu": mu_b, "passes": pb, "seconds": t_bisect},
            "dos_1001_points_ms": t_dos,
            "eig_roofline": {"bound": "lds", "achieved": lds_tbps, "peak": LDS_PEAK_TBPS, "unit": "TB/s",
                             "frac": lds_tbps / LDS_PEAK_TBPS, "fp64_tflops": tflops,
                             "fp64_frac": tflops / FP64_PEAK_TFLOPS,
                             "lds_bytes_per_step": lb, "flop_per_step": fl, "steps": steps},
        }
    return out


def atom_section(ctx):
    """Hubbard-I atoms (64 atoms of 10 and of 14 spin-orbitals, U = 6, beta = 40:
    every Fock state of every atom, for every orbital) and the energy-functional
    sums of the pole route on the d-shell and f-shell workloads.  The energy
    kernel reads, per (k, level) entry, E^ps, |u|^2 and |S_a u|^2 (8 (2 + nc) B)
    and the physical eigenvector column (16 Nb B): its HBM rate is priced
    against 8 TB/s."""
    import dataclasses

    import torch

    from paper_1111_2157_amd import synth
    from paper_1111_2157_amd.dyson import Lattice, PoleSelfEnergy

    def dev(x):
        return torch.as_tensor(np.asarray(x, np.float64), device="cuda")

    out = {}
    for nc in (10, 14):
        natoms = 64
        rng = np.random.default_rng(nc)
        eps, U, mu = dev(rng.uniform(-1.0, 0.5, (natoms, nc))), dev(np.full(natoms, 6.0)), dev(np.zeros(natoms))
        ctx.hubbard1(eps, U, mu, 40.0)
        torch.cuda.synchronize()
        ms = _event_ms(lambda: ctx.hubbard1(eps, U, mu, 40.0), 5)
        n = natoms * nc * 2 ** nc
        out["hubbard1-%dx%d" % (natoms, nc)] = {"ms": ms, "state_orbital_evals": n,
                                                "state_orbital_evals_per_s": n / (ms * 1e-3)}
    for w in (synth.d_shell(), synth.f_shell()):
        sig = dataclasses.replace(w.sigma, poles=[(p + w.mu, v) for p, v in w.sigma.poles])
        lat, pol = Lattice.from_host(w.lattice), PoleSelfEnergy.from_host(sig)
        es = ctx.pole_eig(lat, pol)
        ctx.pole_energy(lat, pol, es, w.mu)
        torch.cuda.synchronize()
        ctx.sync_status()
        ms = _event_ms(lambda: ctx.pole_energy(lat, pol, es, w.mu), 10)
        nb, nc = w.lattice.nb_max, w.lattice.nc
        nbytes = w.lattice.nk * (nb + len(sig.poles)) * (8 * (2 + nc) + 16 * nb)
        gbps = nbytes / (ms * 1e-3) / 1e9
        out["energy-" + w.name] = {"ms": ms, "algorithmic_bytes": nbytes, "gbps": gbps,
                                   "roofline": {"bound": "hbm", "achieved": gbps, "peak": 8000.0, "unit": "GB/s",
                                                "frac": gbps / 8000.0}}
    return out


def mu_search(ctx, tune=True):
    import torch

    from paper_1111_2157_amd import synth
    from paper_1111_2157_amd.dyson import BISECT, NEWTON, Lattice, SelfEnergy

    wl = synth.differentiation()
    lat, sig = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
    if tune:
        ctx.autotune(lat, sig, 0.0)
    ctx.dmft_ntot(lat, sig, 0.0)  # warm-up
    torch.cuda.synchronize()
    out = {"workload": wl.name, "n_target": wl.n_target, "tol": 1e-8, "bracket": [-40.0, 40.0]}
    for name, m in (("newton", NEWTON), ("bisect", BISECT)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mu, passes, n = ctx.find_mu(lat, sig, wl.n_target, 1e-8, m, -40.0, 40.0, 0.0, 300)
        dt = time.perf_counter() - t0
        out[name] = {"mu": mu, "passes": passes, "N": n, "seconds": dt}
    out["speedup"] = out["bisect"]["seconds"] / out["newton"]["seconds"]
    return out


def batched_flops(wl):
    """Algorithmic low-rank flops of one batched pass, summed over the ragged windows."""
    fl = 0.0
    for lat, sig in zip(wl.lattices, wl.sigmas):
        fl += sig.nw * float(np.sum(flops_per_eval_lowrank(lat.nb.astype(float), float(lat.nc))))
    return fl


def batched_headline(ctx, steps, warmup, tune=True, plan_candidate=-1):
    """The batched workload: plan (the autotuner picks the form and tiles),
    capture one pass into a hipGraph with kernel timing on, replay it warmup
    times, then time steps replays.  Returns the record's measurement fields."""
    import torch

    from paper_1111_2157_amd import synth
    from paper_1111_2157_amd.dyson import FORM_AUTO, FORM_LOWRANK, Lattice, SelfEnergy

    wl = synth.batched()
    lats = [Lattice.from_host(l) for l in wl.lattices]
    sigs = [SelfEnergy.from_host(s) for s in wl.sigmas]
    ctx.batched_set_form(FORM_AUTO if tune else FORM_LOWRANK)
    ctx.batched_set_tile_candidate(plan_candidate)
    t0 = time.perf_counter()
    ctx.batched_plan(lats, sigs, 2)
    plan_s = time.perf_counter() - t0
    mu_dev = torch.zeros(len(lats), dtype=torch.float64, device="cuda")
    nks, gls = ctx.batched_outputs()
    ctx.timing(True)
    ctx.batched_graph_capture(mu_dev, nks, gls)
    torch.cuda.synchronize()
    ctx.batched_sync_status()
    for _ in range(warmup):
        ctx.batched_graph_launch()
    torch.cuda.synchronize()
    ctx.timing(True)  # reads the warm-up replays and starts counting afresh
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.batched_graph_launch()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    kms, launches = ctx.timing(False)
    ctx.batched_sync_status()
    # per-class kernel durations (overlapping when the plan runs the classes
    # concurrently) from two directly enqueued passes: a graph replay is timed
    # as a whole
    ctx.timing(True)
    for _ in range(2):
        ctx.batched_pass(mu_dev, nks, gls)
    torch.cuda.synchronize()
    direct_ms, npass = ctx.timing(False)
    classes = ctx.batched_classes()
    ctx.batched_sync_status()
    evals = sum(l.nk for l in wl.lattices) * wl.sigmas[0].nw
    fl = batched_flops(wl)
    kavg = kms / max(launches, 1) / 1e3
    for c in classes:
        c["kernel_ms_per_pass"] = c.pop("kernel_ms") / max(npass, 1)
    from paper_1111_2157_amd.dyson import FORM_LOWRANK as LR
    form = "low-rank" if ctx.batched_form() == LR else "dense"
    concurrent = ctx.batched_concurrent() == 1
    tile_candidate = ctx.batched_tile_candidate()
    del nks, gls
    ctx._b_ws = None
    torch.cuda.empty_cache()
    return wl, {"sec": sec, "evals": evals, "flops": fl, "kernel_s": kavg, "launches": launches,
                "classes": classes, "plan_seconds": plan_s, "form": form, "concurrent": concurrent,
                "tile_candidate": tile_candidate,
                "direct_pass_ms": direct_ms / max(npass, 1)}


def density_workload(ctx, wl, steps, tune):
    """One autotuned density pass (N(k), G_loc, scalars) of a single-lattice workload."""
    from paper_1111_2157_amd.dyson import Lattice, SelfEnergy

    lat, sig = Lattice.from_host(wl.lattice), SelfEnergy.from_host(wl.sigma)
    if tune:
        ctx.autotune(lat, sig, wl.mu)
    sec, kms, ln = time_density(ctx, lat, sig, wl.mu, steps, 1)
    nb, nc = wl.lattice.nb_max, wl.lattice.nc
    ev = wl.lattice.nk * sig.nw
    kn, fp = density_kernel(ctx, nb, nc)
    kavg = kms / max(ln, 1) / 1e3
    return {"evals_per_s": ev / sec, "ms_per_pass": sec * 1e3, "kernel": kn, "kernel_ms": kavg * 1e3,
            "flop_per_eval": fp, "kernel_tflops": fp * ev / kavg / 1e12,
            "kernel_frac": fp * ev / kavg / 1e12 / FP64_PEAK_TFLOPS}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; the path shards over k across GPUs "
              "by design, but multi-GPU runs are not part of it (use --gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    from paper_1111_2157_amd.dyson import Context

    ctx = Context(0)
    if args.section:
        from paper_1111_2157_amd import synth as _synth

        rec = {"pole": lambda: pole_route(ctx, not args.no_tune), "sc": lambda: self_consistency(ctx),
               "atom": lambda: atom_section(ctx),
               "adj": lambda: adjoint_section(ctx, not args.no_tune),
               "d-shell": lambda: density_workload(ctx, _synth.d_shell(), args.steps, not args.no_tune),
               "f-shell": lambda: density_workload(ctx, _synth.f_shell(), args.steps, not args.no_tune),
               }[args.section]()
        print(json.dumps({"section": args.section, "result": rec}), flush=True)
        return
    from paper_1111_2157_amd import synth

    wl, m = batched_headline(ctx, args.steps, args.warmup, not args.no_tune, args.plan_candidate)
    achieved = m["flops"] / m["kernel_s"] / 1e12
    traffic = measured_traffic(wl.name, m["form"], m["classes"])
    rec = {
        "metric": "(k,iw) Dyson evals/s",
        "value": m["evals"] / m["sec"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "nk": wl.lattices[0].nk, "iterates": len(wl.lattices),
                   "nb": "U{%d..%d}" % (int(wl.lattices[0].nb.min()), int(wl.lattices[0].nb.max())),
                   "nc": sorted({l.nc for l in wl.lattices}), "nw": wl.sigmas[0].nw, "beta": wl.sigmas[0].beta,
                   "mu": 0.0, "outputs": "N(k) and G_loc of every iterate", "tail_order": 2,
                   "graph": True, "form": m["form"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": traffic["bytes"] if traffic else None,
                     "traffic_unit": "HBM bytes per pass of the class kernels (counters)",
                     "traffic_gbps": traffic["bytes"] / m["kernel_s"] / 1e9 if traffic else None,
                     "traffic_profile": traffic["profile"] if traffic else None,
                     "kernel": "batched low-rank Dyson pass: %d class launches (%s) and the epilogue "
                               "reductions, timed per graph replay"
                               % (len(m["classes"]), "concurrent" if m["concurrent"] else "one after another"),
                     "kernel_ms": m["kernel_s"] * 1e3, "timed_launches": m["launches"],
                     "dyson_section_ms_direct": m["direct_pass_ms"],
                     "flop_per_pass": m["flops"],
                     "flop_count": "8 (Nb^2 Nc + 2 Nb Nc^2 + 5 Nc^3) per (k, i w_n), low-rank form"},
        "batched_classes": m["classes"],
        "plan_seconds": m["plan_seconds"],
        "plan_tile_candidate": m["tile_candidate"],
    }
    if not args.no_mu:
        rec["mu_search"] = mu_search(ctx, not args.no_tune)
    if not args.no_workloads:
        tune = not args.no_tune
        wls = {}
        for maker, steps in ((synth.d_shell, 10), (synth.f_shell, 3)):
            w = maker()
            wls[w.name] = density_workload(ctx, w, steps, tune)
        wls["diff fused forward + adjoint (N_tot, dN/dmu, dN/dSigma)"] = adjoint_pass(ctx)
        rec["workloads"] = wls
    if args.extra:
        extra = {}
        w = synth.plain()
        extra[w.name] = density_workload(ctx, w, 20, not args.no_tune)
        extra["general VJP (Sigma-bar, mu-bar)"] = general_vjp_pass(ctx)
        extra["self-consistency (E_imp, Delta)"] = self_consistency(ctx)
        extra["pole route"] = pole_route(ctx, not args.no_tune)
        extra["atom and energy"] = atom_section(ctx)
        rec["extra"] = extra
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(wl, 0.0, args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
