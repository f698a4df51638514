"""CPU checks of the C-ABI library: it loads and exports every function that
include/dmft.h declares; host-side validation paths need no GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dmft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("gloc_compute", "density_matrix", "find_mu", "density_matrix_vjp", "dmft_ntot",
              "dmft_batched_pass", "dmft_autotune"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1111_2157_amd import _lib

    lib = _lib.load()
    assert sorted(_lib.EXPORTS) == declared_functions()
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_strerror_and_null_handle_validation():
    from paper_1111_2157_amd import _lib

    lib = _lib.load()
    for code, name in _lib.STATUS.items():
        assert lib.dmft_strerror(code)
    # argument checks run before any device work: NULL handle / NULL outputs
    assert lib.dmft_workspace_size(None, None, None, None) == -1
    assert lib.dmft_last_error(None) == b""
    assert lib.dmft_destroy(None) == -1


def test_widened_entry_points_validate_before_device_work():
    """The pole route, the atom, the energy sums and the self-consistency step
    reject a NULL handle or missing arguments on the host (DMFT_EINVAL), before
    any HIP call."""
    from paper_1111_2157_amd import _lib

    lib = _lib.load()
    lat, pol, sig = _lib.DmftLattice(), _lib.DmftPoles(), _lib.DmftSigma()
    ref = ctypes.byref
    assert lib.dmft_pole_workspace_size(None, ref(lat), ref(pol), 0, None) == -1
    assert lib.dmft_pole_eig(None, ref(lat), ref(pol), None, None, None, None, None, 0, None) == -1
    assert lib.dmft_pole_density(None, ref(lat), ref(pol), 0.0, 0, None, None, None, None, None, 0, None) == -1
    mu, passes, n = ctypes.c_double(), ctypes.c_int(), ctypes.c_double()
    assert lib.dmft_pole_find_mu(None, ref(lat), ref(pol), None, None, 1.0, 1e-8, 0, -1.0, 1.0, 10, ref(mu),
                                 ref(passes), ref(n), None, 0, None) == -1
    assert lib.dmft_pole_dos(None, ref(lat), ref(pol), None, None, None, 0.0, 0.1, -1.0, 1.0, 11, None, None,
                             None, 0, None) == -1
    assert lib.dmft_pole_energy(None, ref(lat), ref(pol), 0.0, None, None, None, None, None, None, 0, None) == -1
    assert lib.dmft_hubbard1(None, 1, 2, None, None, None, 10.0, 0.0, None, None, None, None, None, None,
                             None) == -1
    assert lib.dmft_hubbard1_poles(None, 2, 2, 0, None, None, None, None, None, None, None) == -1
    assert lib.dmft_sigma_from_poles(None, 2, ref(pol), 8, 0.0, None, None) == -1
    assert lib.dmft_hybridization(None, ref(lat), ref(sig), 0.0, None, None, None, None, 0, None) == -1


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bench_jacobi_cost_matches_the_hand_count():
    """Per rotating Jacobi step of the d-shell pseudo-Hamiltonian (32 bands, 10
    poles, m = 42, 21 pairs): 210 off-diagonal blocks x 80 flop + 21 x 32
    vector pairs x 20 flop; LDS (210 x 8 + 21 x 3 + 21 x 32 x 4) x 16 B."""
    import importlib.util

    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    fl, lds, m = bench.jacobi_step_cost(32, 10)
    assert (fl, lds, m) == (210 * 80 + 21 * 32 * 20, (210 * 8 + 21 * 3 + 21 * 32 * 4) * 16, 42)
    fl, lds, m = bench.jacobi_step_cost(12, 5)   # odd size: padded to 18
    assert m == 18 and fl == 36 * 80 + 9 * 12 * 20


def test_variant_lists_of_the_adjoint_kinds():
    """Kinds 2 and 3 (fused scalar adjoint, general product) list low-rank codes
    (bit 3) first, the default, then the dense adjoint kernel (code 0) where it
    exists (padded windows up to 48); kind 4 does not exist."""
    from paper_1111_2157_amd import _lib

    lib = _lib.load()
    buf = (ctypes.c_int * 16)()
    for kind in (2, 3):
        for nbp in (16, 32, 48, 64):
            n = lib.dmft_variants(kind, nbp, buf, 16)
            codes = list(buf[:n])
            assert n >= 1 and codes[0] & 8, (kind, nbp, codes)
            assert (0 in codes) == (nbp <= 48), (kind, nbp, codes)
            assert all(c & 8 for c in codes if c != 0)
    assert lib.dmft_variants(4, 32, buf, 16) == 0
