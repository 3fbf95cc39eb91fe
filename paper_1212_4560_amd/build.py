"""Build the HIP library ``libgenp.so`` in-tree for gfx950 with hipcc.

Every ``csrc/*.hip`` file is compiled to an object in ``_build/`` (in
parallel), then linked into ``paper_1212_4560_amd/libgenp.so``.  Always
recompiles: the build is the "does it compile" check and takes well under a
minute.  Usage: ``python -m paper_1212_4560_amd.build``.

``python -m paper_1212_4560_amd.build --sanitize`` builds the host-checking
variant ``_build_san/libgenp_san.so`` instead: the library's host code under
AddressSanitizer and UndefinedBehaviorSanitizer (the flags apply to the host
compilation only; device code is compiled unoptimized and never run there),
for the CPU tests of the C ABI's host paths.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shlex
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libgenp.so")

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-pass-failed",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    return obj


BUILD_SAN = os.path.join(os.path.dirname(HERE), "_build_san")
LIB_SAN = os.path.join(BUILD_SAN, "libgenp_san.so")
# host-only sanitizer flags (each -fsanitize= right after -Xarch_host: no device code is built with them)
SAN_HOST = shlex.split("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
                       "-Xarch_host -fno-omit-frame-pointer")


def build_sanitized(verbose: bool = False) -> str:
    """The host-sanitized library (see the module docstring); rebuilt every call."""
    os.makedirs(BUILD_SAN, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    flags = [f"--offload-arch={ARCH}", "-g", "-fPIC", "-std=c++17", "-Xarch_host", "-O1", "-Xarch_device", "-O0",
             "-Wno-unused-result", "-Wno-pass-failed", *SAN_HOST]

    def one(src: str) -> str:
        obj = os.path.join(BUILD_SAN, os.path.basename(src) + ".o")
        r = subprocess.run([hipcc(), *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc (sanitized) failed for {src}:\n{r.stderr[-4000:]}")
        return obj

    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(one, srcs))
    r = subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *SAN_HOST[:4], "-o", LIB_SAN, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link (sanitized) failed:\n{r.stderr[-4000:]}")
    if verbose:
        print(f"built {LIB_SAN} from {len(srcs)} sources")
    return LIB_SAN


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    if not srcs:
        raise RuntimeError("no HIP sources found")
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources")
    return LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv[1:]:
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
