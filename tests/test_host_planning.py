"""CPU tests of the host layer through a planning handle (no device): argument
checks, bucketing of ragged band windows by padded size, workspace sizing, and
refusal of every call that would reach the device."""
import ctypes as C

import numpy as np
import pytest

ref = C.byref


@pytest.fixture(scope="module")
def lib():
    from paper_1111_2157_amd import _lib

    return _lib.load()


@pytest.fixture()
def h(lib):
    hh = C.c_void_p()
    assert lib.dmft_create(ref(hh), -1) == 0
    yield hh
    assert lib.dmft_destroy(hh) == 0


def fake(n, step=256):
    """Distinct, aligned, never-dereferenced addresses standing in for device
    buffers: a planning handle only checks that they are set."""
    return C.c_void_p(0x7f0000000000 + n * step)


def lattice(nk, nc, nb):
    from paper_1111_2157_amd import _lib

    nb = np.ascontiguousarray(nb, np.int32)
    lat = _lib.DmftLattice(nk, nc, int(nb.max()), nb.ctypes.data_as(C.c_void_p), fake(1), fake(2), fake(3))
    lat._keep = nb
    return lat


def sigma(nw, beta=40.0):
    from paper_1111_2157_amd import _lib

    return _lib.DmftSigma(nw, beta, fake(4), None, fake(5))


def last(lib, h):
    return lib.dmft_last_error(h).decode()


def ws_size(lib, h, lat, sig):
    n = C.c_size_t()
    r = lib.dmft_workspace_size(h, ref(lat), ref(sig), ref(n))
    return r, n.value


def test_planning_handle_sizes_ragged_windows_across_every_bucket(lib, h):
    # every window size from nc to 64 in one lattice: all four padded sizes,
    # each with its lowest (NBP - 15) and highest (NBP) member
    nb = np.arange(5, 65, dtype=np.int32)
    r, n = ws_size(lib, h, lattice(len(nb), 5, nb), sigma(64))
    assert r == 0, last(lib, h)
    assert n > 0 and n % 256 == 0
    # uniform and ragged lattices of the same shape: ragged needs no less
    r2, n2 = ws_size(lib, h, lattice(len(nb), 5, np.full(len(nb), 64, np.int32)), sigma(64))
    assert r2 == 0 and n2 > 0


def test_workspace_grows_with_frequencies_and_kpoints(lib, h):
    nb = np.full(16, 32, np.int32)
    sizes = [ws_size(lib, h, lattice(16, 10, nb), sigma(nw))[1] for nw in (16, 256, 4096)]
    assert sizes[0] < sizes[1] < sizes[2]
    sizes = [ws_size(lib, h, lattice(nk, 10, np.full(nk, 32, np.int32)), sigma(256))[1] for nk in (4, 64, 1024)]
    assert sizes[0] < sizes[1] < sizes[2]


@pytest.mark.parametrize("case,needle", [
    ("nk0", "nk must be"), ("nc0", "nc must be"), ("nc17", "nc must be"), ("nbmax65", "nb_max"),
    ("nb_lt_nc", "outside nc..nb_max"), ("nw0", "nw must be"), ("beta0", "beta"), ("betanan", "beta"),
    ("noeps", "eps, wk and proj"), ("nosigma", "sigma and e_dc"),
])
def test_host_checks_reject_bad_shapes(lib, h, case, needle):
    lat, sig = lattice(4, 5, [8, 8, 8, 8]), sigma(16)
    if case == "nk0":
        lat.nk = 0
    elif case == "nc0":
        lat.nc = 0
    elif case == "nc17":
        lat.nc = 17
    elif case == "nbmax65":
        lat = lattice(4, 5, [8, 65, 8, 8])
    elif case == "nb_lt_nc":
        lat = lattice(4, 5, [8, 4, 8, 8])
    elif case == "nw0":
        sig.nw = 0
    elif case == "beta0":
        sig.beta = 0.0
    elif case == "betanan":
        sig.beta = float("nan")
    elif case == "noeps":
        lat.eps = None
    elif case == "nosigma":
        sig.sigma = None
    r, _ = ws_size(lib, h, lat, sig)
    assert r == -1
    assert needle in last(lib, h)


def test_device_calls_refused_after_host_checks(lib, h):
    lat, sig = lattice(4, 5, [8, 9, 16, 17]), sigma(16)
    ws = fake(100)
    out = fake(200)
    # argument errors are reported first ...
    assert lib.density_matrix(h, ref(lat), ref(sig), C.c_double(0.0), 1, out, None, None, ws, C.c_size_t(1 << 30),
                              None) == -1
    assert "tail_order" in last(lib, h)
    assert lib.density_matrix(h, ref(lat), ref(sig), C.c_double(float("inf")), 2, out, None, None, ws,
                              C.c_size_t(1 << 30), None) == -1
    assert "mu is not finite" in last(lib, h)
    # ... then the workspace ...
    _, need = ws_size(lib, h, lat, sig)
    assert lib.density_matrix(h, ref(lat), ref(sig), C.c_double(0.0), 2, out, None, None, ws, C.c_size_t(need - 1),
                              None) == -6
    assert lib.density_matrix(h, ref(lat), ref(sig), C.c_double(0.0), 2, out, None, None, C.c_void_p(0x7f0000000010),
                              C.c_size_t(need), None) == -6
    # ... and only then the missing device
    assert lib.density_matrix(h, ref(lat), ref(sig), C.c_double(0.0), 2, out, None, None, ws, C.c_size_t(need),
                              None) == -1
    assert "planning handle" in last(lib, h)
    assert lib.gloc_compute(h, ref(lat), ref(sig), C.c_double(0.0), out, ws, C.c_size_t(need), None) == -1
    assert "planning handle" in last(lib, h)


def test_find_mu_argument_checks(lib, h):
    lat, sig = lattice(2, 3, [6, 6]), sigma(8)
    mu, p, n = C.c_double(), C.c_int(), C.c_double()
    _, need = ws_size(lib, h, lat, sig)

    def call(lo, hi, tol=1e-8, method=0, max_iter=50, tail=2):
        return lib.find_mu(h, ref(lat), ref(sig), tail, C.c_double(3.0), C.c_double(tol), method, C.c_double(lo),
                           C.c_double(hi), C.c_double(0.0), max_iter, ref(mu), ref(p), ref(n), fake(100),
                           C.c_size_t(need), None)

    assert call(1.0, -1.0) == -1 and "mu_lo < mu_hi" in last(lib, h)
    assert call(-1.0, float("inf")) == -1
    assert call(-1.0, 1.0, tol=0.0) == -1 and "tol_n" in last(lib, h)
    assert call(-1.0, 1.0, max_iter=0) == -1
    assert call(-1.0, 1.0, method=7) == -1 and "method" in last(lib, h)
    assert call(-1.0, 1.0, tail=1) == -1 and "tail_order" in last(lib, h)
    assert call(-1.0, 1.0) == -1 and "planning handle" in last(lib, h)


def test_batched_workspace_size_on_planning_handle(lib, h):
    lats = [lattice(6, 5, [20, 33, 48, 49, 64, 31]), lattice(6, 14, [20, 33, 48, 49, 64, 31])]
    sigs = [sigma(64), sigma(64)]
    lp = (C.c_void_p * 2)(*[C.addressof(x) for x in lats])
    sp = (C.c_void_p * 2)(*[C.addressof(x) for x in sigs])
    n = C.c_size_t()
    assert lib.dmft_batched_workspace_size(h, 2, lp, sp, ref(n)) == 0, last(lib, h)
    assert n.value > 0
    assert lib.dmft_batched_plan(h, 2, lp, sp, 2, fake(100), n, None) == -1
    assert "planning handle" in last(lib, h)


def test_real_device_index_without_gpu_fails_cleanly(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    hh = C.c_void_p()
    assert lib.dmft_create(ref(hh), 0) == -2
    assert not hh.value
