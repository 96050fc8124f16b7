"""All-core FP64 CPU destriper (C++17 + OpenMP), the timing baseline.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: the tests pin it to
the NumPy oracle and the benchmark times it on the host cores; nothing in
the library calls it.  ``build()`` compiles ``cpu_baseline.cpp`` with g++
into ``libcpu_destripe.so`` next to this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_baseline.cpp")
LIB = os.path.join(HERE, "libcpu_destripe.so")
STREAMS = {"T": 1, "QU": 6, "TQU": 7}
_lib = None


def build() -> str:
    cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", SRC, "-o", LIB + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"g++ failed: {res.stderr}")
    os.replace(LIB + ".tmp", LIB)
    return LIB


def library():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is not built; run oracle.cpu_baseline.build()")
        lib = ctypes.CDLL(LIB)
        i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
        lib.cpu_destripe_max_threads.restype = i32
        lib.cpu_destripe_solve.argtypes = [i64, i64, i64, i32, vp, vp, vp, vp, dbl, dbl, i32, i32, vp, vp, vp, vp]
        lib.cpu_destripe_solve.restype = i32
        lib.cpu_destripe_apply.argtypes = [i64, i64, i64, i32, vp, vp, vp, dbl, i32, vp, i32, vp, vp]
        lib.cpu_destripe_apply.restype = i32
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _inputs(pix, psi, streams, weights):
    pix = np.ascontiguousarray(pix, dtype=np.int32)
    psi = None if psi is None else np.ascontiguousarray(psi, dtype=np.float64)
    if streams != "T" and psi is None:
        raise ValueError("psi is needed")
    w = np.ascontiguousarray(weights, dtype=np.float64)
    return pix, psi, w


def solve(pix, psi, tod, n_pix, L, streams, weights, tol=1e-10, max_iter=1000, rcond_cut=1e-3, threads=0,
          maps=True) -> dict:
    """Destripe on the host cores; returns baselines [n_streams][n_b], destriped map [n_pix][3], hits and timings."""
    lib = library()
    pix, psi, w = _inputs(pix, psi, streams, weights)
    tod = np.ascontiguousarray(tod, dtype=np.float64)
    n_t = pix.size
    n_b = -(-n_t // int(L))
    ns = tod.shape[0]
    a = np.zeros((ns, n_b))
    m = np.zeros((int(n_pix), 3)) if maps else None
    h = np.zeros(int(n_pix), dtype=np.int64)
    info = np.zeros(6)
    rc = lib.cpu_destripe_solve(n_t, int(n_pix), int(L), STREAMS[streams], _p(pix), _p(psi), _p(tod), _p(w),
                                float(rcond_cut), float(tol), int(max_iter), int(threads), _p(a), _p(m), _p(h),
                                _p(info))
    return dict(status=rc, baselines=a, destriped_map=m, hits=h, setup_s=info[0], loop_s=info[1], total_s=info[2],
                iterations=int(info[3]), rel_residual=info[4], threads=int(info[5]))


def apply_K(pix, psi, n_pix, L, streams, weights, v, reps=1, rcond_cut=1e-3, threads=0):
    """K v (Eq. 13 operator) on the host cores, repeated ``reps`` times; returns (K v, seconds per application,
    setup seconds, threads)."""
    lib = library()
    pix, psi, w = _inputs(pix, psi, streams, weights)
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros_like(v)
    info = np.zeros(3)
    lib.cpu_destripe_apply(pix.size, int(n_pix), int(L), STREAMS[streams], _p(pix), _p(psi), _p(w),
                           float(rcond_cut), int(threads), _p(v), int(reps), _p(out), _p(info))
    return out, info[1], info[0], int(info[2])


def max_threads() -> int:
    return int(library().cpu_destripe_max_threads())
