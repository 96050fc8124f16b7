"""Host-side checks of the C ABI: the built library loads and exports every
function that include/dst.h declares; struct layouts match the binding."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1309_5609_amd import dst

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dst.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int|const char\s*\*)\s+(dst_\w+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert set(declared()) == set(dst.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(dst.LIB_PATH):
        pytest.skip("libdst.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", dst.LIB_PATH], capture_output=True, text=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared():
        assert name in syms, name
    lib = dst.library()
    assert lib.dst_version() == 2


def test_struct_layouts():
    # offsets fixed by include/dst.h (x86-64 SysV)
    assert ctypes.sizeof(dst.dst_problem) == 96
    assert dst.dst_problem.pix.offset == 40 and dst.dst_problem.weight.offset == 64
    assert ctypes.sizeof(dst.dst_solve_opts) == 32 and dst.dst_solve_opts.a0.offset == 24
    assert ctypes.sizeof(dst.dst_solve_info) == 136
    assert ctypes.sizeof(dst.dst_scan) == 64


def test_layouts_agree_with_the_c_compiler(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "dst.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(dst_problem),'
                   ' offsetof(dst_problem, pix), offsetof(dst_problem, weight), sizeof(dst_solve_opts),'
                   ' offsetof(dst_solve_opts, a0), sizeof(dst_solve_info)); printf("%zu %zu\\n", sizeof(dst_scan),'
                   ' offsetof(dst_scan, sidereal_day_s)); return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert got == ["96", "40", "64", "32", "24", "136", "64", "56"]
    assert dst.dst_scan.sidereal_day_s.offset == 56


def test_no_device_is_reported_not_crashed():
    """Without a visible GPU, dst_create fails cleanly with DST_EINVAL."""
    if not os.path.exists(dst.LIB_PATH):
        pytest.skip("libdst.so not built")
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = dst.library()
    h = ctypes.c_void_p()
    assert lib.dst_create(ctypes.byref(h), 0) == -1
    assert lib.dst_destroy(None) == 0
