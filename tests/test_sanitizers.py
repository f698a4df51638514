"""AddressSanitizer and UndefinedBehaviorSanitizer on the host code (CPU only):
the C oracle and the library's C-ABI host layer are built by gcc / g++ with
the sanitizers (no device code is involved) and driven by the small programs
in tests/sanitize/; a memory or undefined-behaviour error aborts the program."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, **kw)
    return r.returncode, r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    rc, out = _run(["gcc", "-std=gnu11"] + SAN + [os.path.join(ROOT, "oracle", "dmft_oracle.c"),
                                                 os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                                                 "-lm", "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe], env=ENV)
    assert rc == 0 and "oracle driver ok" in out, out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists("/opt/rocm/lib/libamdhip64.so"),
                    reason="g++ or the HIP runtime library not available")
def test_host_layer_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_san")
    csrc = os.path.join(ROOT, "paper_1111_2157_amd", "csrc")
    rc, out = _run(["g++", "-std=c++17"] + SAN + [
        "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + csrc,
        os.path.join(csrc, "dmft_host.cpp"), os.path.join(ROOT, "tests", "sanitize", "host_stubs.cpp"),
        os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe], env=ENV)
    assert rc == 0 and "host driver ok" in out, out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
