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
