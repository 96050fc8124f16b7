"""Accuracy of the library's FP64 sincos (cos 2psi, sin 2psi of Eqs. 3-6),
compiled for the host from the same header the kernels include, against
long-double libm."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fast_sincos_accuracy(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    exe = tmp_path / "trig_check"
    src = os.path.join(ROOT, "tests", "trig_check.hip")
    inc = os.path.join(ROOT, "paper_1309_5609_amd", "csrc")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", f"-I{inc}", src, "-o", str(exe)], check=True,
                   capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    n, es, ec = int(out[0]), float(out[1]), float(out[2])
    assert n > 2_000_000
    # |sin|, |cos| <= 1: absolute error of a few units of 2^-53
    assert es < 4e-16 and ec < 4e-16, (es, ec)
