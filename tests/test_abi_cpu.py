"""The C-ABI library loads and exports every entry point of include/genp.h (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1212_4560_amd import genp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "genp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(genp_[a-z_0-9]+)\s*\(", src)))


def _lib():
    if not os.path.exists(genp.LIB_PATH):
        pytest.fail("libgenp.so is not built: run `python -m paper_1212_4560_amd.build`")
    return genp.load()


def test_header_declares_the_abi():
    assert _declared() == sorted(genp.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib()
    for name in _declared():
        assert hasattr(L, name), name
    nm = os.popen(f"nm -D --defined-only {genp.LIB_PATH}").read()
    exported = set(re.findall(r" T (genp_[a-z_0-9]+)", nm))
    assert set(_declared()) <= exported


def test_strerror_covers_codes():
    _lib()
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7):
        s = genp.strerror(code)
        assert s and "unknown" not in s
    assert "unknown" in genp.strerror(99)


@pytest.mark.parametrize("cname,pyname", [("genp_info", "GenpInfo"), ("genp_lr_info", "GenpLrInfo"),
                                          ("genp_nrank_info", "GenpNrankInfo"),
                                          ("genp_refine_opts", "GenpRefineOpts")])
def test_info_struct_layout_matches_header(tmp_path, cname, pyname):
    """The binding's mirrors of the info structs have the C structs' sizes and field offsets."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    cls = getattr(genp, pyname)
    fields = [f for f, _ in cls._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'    printf("{f} %zu\\n", offsetof({cname}, {f}));\n' for f in fields)
    src.write_text(f'#include <stddef.h>\n#include <stdio.h>\n#include "genp.h"\nint main(void) {{\n'
                   f'    printf("sizeof %zu\\n", sizeof({cname}));\n{body}    return 0;\n}}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.splitlines())
    assert int(out["sizeof"]) == ctypes.sizeof(cls)
    for f in fields:
        assert int(out[f]) == getattr(cls, f).offset, f


def test_invalid_arguments_rejected_before_device():
    L = _lib()
    h = ctypes.c_void_p()
    assert L.genp_create(ctypes.byref(h), 0, 0, 256, None) == genp.EINVAL
    assert L.genp_create(ctypes.byref(h), 10, 7, 256, None) == genp.EINVAL
    assert L.genp_create(ctypes.byref(h), 10, 0, 96, None) == genp.EINVAL
    assert L.genp_create(None, 10, 0, 256, None) == genp.EINVAL
    assert L.genp_destroy(None) == genp.OK
    for fn, args in (("genp_factor", (None, 0.0, None)), ("genp_get_info", (None, None)),
                     ("genp_copy_work", (None, None, 1)), ("genp_condest", (None, None, None, None)),
                     ("genp_refine_ex", (None, None, 1, 1, None, 1, None, None)),
                     ("genp_solve_backward_ex", (None, None, 1, None, 1, 1, None, 1, None, 1, None, None))):
        assert getattr(L, fn)(*args) == genp.EINVAL


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = _lib()
    h = ctypes.c_void_p()
    assert L.genp_create(ctypes.byref(h), 16, 0, 64, None) == genp.EDEVICE
    assert not h.value


def test_noalloc_rejects_oversize_before_device_work():
    """The allocation-free numerical rank checks its scratch need on the host first: a problem
    larger than the fixed array is refused with GENP_ESCRATCH (the pointers are never used)."""
    L = _lib()
    info = genp.GenpNrankInfo()
    p = ctypes.c_void_p(256)
    m = n = 200000
    st = L.genp_numerical_rank_noalloc(p, m, n, n, p, 64, 0, 64, 1e6, p, 64, ctypes.byref(info), None)
    assert st == genp.ESCRATCH
    assert L.genp_numerical_rank_noalloc(None, 10, 10, 10, p, 4, 0, 4, 1e6, p, 4, ctypes.byref(info),
                                         None) == genp.EINVAL
