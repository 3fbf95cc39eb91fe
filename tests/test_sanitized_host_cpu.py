"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

`python -m paper_1212_4560_amd.build --sanitize` compiles the host side of every source with
both sanitizers (device code unoptimized, never run here), and `tests/host/abi_host_checks.c`,
built with the same compiler and sanitizers, drives the C ABI's host paths: argument checks of
every entry point, context creation without a usable device, the status strings, the fixed
scratch limit of the allocation-free entry point.  Any sanitizer report aborts the program
(halt_on_error), so the test passes only when every check holds and no report was raised.
"""
import os
import shutil
import subprocess

import pytest

from paper_1212_4560_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"


@pytest.fixture(scope="module")
def checks_exe(tmp_path_factory):
    if shutil.which(B.hipcc()) is None or not os.path.exists(CLANG):
        pytest.skip("no ROCm clang for the sanitizer build")
    lib = B.build_sanitized()
    exe = str(tmp_path_factory.mktemp("san") / "abi_host_checks")
    libdir = os.path.dirname(lib)
    subprocess.run([CLANG, "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host", "abi_host_checks.c"),
                    "-L", libdir, "-lgenp_san", f"-Wl,-rpath,{libdir}", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                   check=True, capture_output=True, text=True)
    return exe


def test_sanitized_library_is_instrumented(checks_exe):
    nm = subprocess.run(["nm", "-D", os.path.join(os.path.dirname(B.LIB_SAN), "libgenp_san.so")],
                        capture_output=True, text=True, check=True).stdout
    assert "__asan_report" in nm and "__ubsan_handle" in nm


def test_host_paths_clean_under_asan_and_ubsan(checks_exe):
    env = dict(os.environ)
    # the ROCm runtime's own allocations at exit are not the library's: no leak report;
    # every other report is fatal
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([checks_exe], capture_output=True, text=True, env=env, timeout=120)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "all host checks passed" in r.stdout or "device present" in r.stdout
    assert "runtime error" not in out and "ERROR: AddressSanitizer" not in out
