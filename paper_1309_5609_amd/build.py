"""Compile the HIP sources of the destriping library for gfx950 into ``libdst.so``.

The library is built in-tree (next to this file) with hipcc; nothing is
installed.  Each source is compiled to an object of its own (in parallel, no
relocatable device code: every kernel and device function lives in the file
that launches it) and the objects are linked into the shared library.
``python -m paper_1309_5609_amd.build`` rebuilds it.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdst.so")
SOURCES = ["dst_kernels.hip", "dst_pixel.hip", "dst_runs.hip", "dst_multi.hip", "dst_pointing.hip", "dst_noise.hip",
           "dst_gmres.hip", "dst_comp.hip", "dst_api.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # hardware FP64 atomics on coarse-grained (hipMalloc) memory
    "-munsafe-fp-atomics",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (set HIPCC or install ROCm)")


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}): {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source and link ``libdst.so`` (always recompiles)."""
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    objs, cmds = [], []
    for s in SOURCES:
        o = os.path.join(OBJ, os.path.splitext(s)[0] + ".o")
        objs.append(o)
        cmds.append([cc, *HIPCC_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-c", os.path.join(CSRC, s), "-o", o])
    jobs = jobs or min(len(cmds), max(1, os.cpu_count() or 1), 8)
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_run, cmds))
    link = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    _run(link)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
