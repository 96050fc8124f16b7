"""Python binding of the destriping C ABI (``include/dst.h``).

Argument marshalling only: every computation runs in the HIP kernels of
``libdst.so``.  PyTorch supplies device memory and the current stream.
Functions carry the C names (``dst_bin``, ``dst_unbin``,
``dst_baseline_reduce``, ``dst_solve``, ...).  Arrays are torch tensors on the
context's GPU with the layouts the header states.

Importing this module does not need a GPU; loading the library does need the
built ``libdst.so`` and raises ``RuntimeError`` when it is missing.  There is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdst.so")

DST_OK, DST_ENOCONV = 0, 1
STATUS = {0: "DST_OK", 1: "DST_ENOCONV", -1: "DST_EINVAL", -2: "DST_ENOMEM", -3: "DST_EHIP", -4: "DST_ENAN",
          -5: "DST_EDEGENERATE", -6: "DST_EBOUNDS", -7: "DST_EBREAKDOWN"}
DST_F32, DST_F64 = 1, 2
STREAMS = {"T": 1, "QU": 6, "TQU": 7, "IQU": 8}
N_STREAMS = {"T": 1, "QU": 2, "TQU": 3, "IQU": 1}
DST_BIN_USE_TOD, DST_BIN_MAP = 1, 2
DST_SOLVE_NO_CANON, DST_SOLVE_PROFILE, DST_SOLVE_NO_GRAPH, DST_SOLVE_PER_SAMPLE = 1, 2, 4, 8
DST_SOLVE_AUTOTUNE = 16
DST_SOLVE_GMRES = 32
DST_NOISE_ACCUMULATE = 1

EXPORTS = ("dst_version", "dst_create", "dst_destroy", "dst_last_error", "dst_synchronize", "dst_pixel_setup",
           "dst_bin", "dst_bin_noalloc", "dst_unbin",
           "dst_baseline_reduce", "dst_residual", "dst_apply_operator", "dst_solve", "dst_solve_batched",
           "dst_pointing_expand", "dst_noise_generate")


class dst_problem(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int64), ("n_pix", ctypes.c_int64), ("baseline_length", ctypes.c_int64),
                ("streams", ctypes.c_uint32), ("tod_dtype", ctypes.c_int32), ("psi_dtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("pix", ctypes.c_void_p), ("psi", ctypes.c_void_p),
                ("tod", ctypes.c_void_p), ("weight", ctypes.c_double * 3), ("rcond_cut", ctypes.c_double)]


class dst_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("restart", ctypes.c_int32), ("a0", ctypes.c_void_p)]


class dst_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("true_rel_residual", ctypes.c_double), ("b_norm", ctypes.c_double),
                ("n_valid_pix", ctypes.c_int64 * 2), ("n_valid_samples", ctypes.c_int64 * 2),
                ("t_setup_ms", ctypes.c_double), ("t_iter_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("t_bin_ms", ctypes.c_double), ("t_apply_ms", ctypes.c_double), ("t_unbin_ms", ctypes.c_double),
                ("t_update_ms", ctypes.c_double), ("n_runs", ctypes.c_int64), ("n_components", ctypes.c_int64)]


SCAN_FIELDS = ("sample_rate_hz", "spin_period_s", "elevation_deg", "latitude_deg", "az0_deg", "lst0_rad",
               "psi0_deg", "sidereal_day_s")


class dst_scan(ctypes.Structure):
    _fields_ = [(name, ctypes.c_double) for name in SCAN_FIELDS]


class DstError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load ``libdst.so`` (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_1309_5609_amd.build.build() first")
    try:
        import torch  # noqa: F401  -- loads the HIP runtime the library will bind to
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, u32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER(dst_problem)
    sig = {
        "dst_version": ([], i32),
        "dst_create": ([ctypes.POINTER(vp), i32], i32),
        "dst_destroy": ([vp], i32),
        "dst_last_error": ([vp], ctypes.c_char_p),
        "dst_synchronize": ([vp, vp], i32),
        "dst_pixel_setup": ([vp, P, vp, vp, vp, vp], i32),
        "dst_bin": ([vp, P, vp, u32, vp, vp, vp], i32),
        "dst_bin_noalloc": ([vp, P, vp, u32, vp, vp, vp], i32),
        "dst_unbin": ([vp, P, vp, vp, vp], i32),
        "dst_baseline_reduce": ([vp, P, vp, vp, vp], i32),
        "dst_residual": ([vp, P, vp, vp, vp], i32),
        "dst_apply_operator": ([vp, P, vp, vp, vp], i32),
        "dst_solve": ([vp, P, ctypes.POINTER(dst_solve_opts), vp, vp, vp, vp, ctypes.POINTER(dst_solve_info), vp],
                      i32),
        "dst_solve_batched": ([vp, i32, P, ctypes.POINTER(dst_solve_opts), vp, vp, vp, vp,
                               ctypes.POINTER(dst_solve_info), vp], i32),
        "dst_pointing_expand": ([vp, ctypes.POINTER(dst_scan), i64, i64, i64, vp, vp, i32, vp], i32),
        "dst_noise_generate": ([vp, ctypes.c_uint64, ctypes.c_uint64, i64, i64, dbl, dbl, dbl, dbl, vp, i32, u32, vp],
                               i32),
    }
    for name, (argtypes, restype) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = restype
    _ = (i64, dbl)
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """A library context on one GPU (``dst_create`` / ``dst_destroy``)."""

    def __init__(self, device: int = 0):
        self.lib = library()
        self.device = device
        h = ctypes.c_void_p()
        rc = self.lib.dst_create(ctypes.byref(h), device)
        if rc != DST_OK:
            raise DstError(rc, f"dst_create(device={device}) failed")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.dst_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int, allow=(DST_OK,)) -> int:
        if rc not in allow:
            raise DstError(rc, self.lib.dst_last_error(self.handle).decode())
        return rc


def _is_float(t) -> bool:
    import torch
    return t.dtype in (torch.float32, torch.float64)


def _dev_index(t) -> int:
    return t.device.index if t.device.index is not None else 0


def _tensor(name: str, t, shape=None, dtypes=None, device=None, min_numel=None):
    """Check a tensor argument: a contiguous torch tensor on GPU ``device`` of an allowed dtype and shape."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor (got {type(t).__name__})")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU (got {t.device})")
    if device is not None and _dev_index(t) != device:
        raise ValueError(f"{name} is on cuda:{_dev_index(t)}, the context on cuda:{device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtypes is not None and t.dtype not in dtypes:
        raise ValueError(f"{name} must have dtype {' or '.join(str(d) for d in dtypes)} (got {t.dtype})")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name} must hold at least {min_numel} elements (got {t.numel()})")
    return t


def _floats():
    import torch
    return (torch.float32, torch.float64)


def _f64():
    import torch
    return (torch.float64,)


@dataclass
class Problem:
    """Device-side problem: torch tensors kept alive with the C struct.

    ``pix`` int32 [n_samples]; ``psi`` float32/float64 [n_samples] (None for
    streams "T"); ``tod`` float32/float64 [n_streams][n_samples] or None; all
    contiguous on one GPU.
    """

    pix: object
    psi: object
    tod: object
    n_pix: int
    baseline_length: int
    streams: str
    weights: tuple
    rcond_cut: float = 1e-3

    @property
    def n_samples(self) -> int:
        return int(self.pix.shape[0])

    @property
    def n_baselines(self) -> int:
        return -(-self.n_samples // self.baseline_length)

    @property
    def n_streams(self) -> int:
        return N_STREAMS[self.streams]

    def validate(self, device=None, need_tod: bool = False) -> None:
        """Raise ValueError unless the arrays have the dtypes, shapes and device the C ABI reads."""
        import torch
        if self.streams not in STREAMS:
            raise ValueError(f"streams must be one of {sorted(STREAMS)} (got {self.streams!r})")
        _tensor("pix", self.pix, dtypes=(torch.int32,), device=device)
        if self.pix.dim() != 1:
            raise ValueError(f"pix must be 1-D (got shape {tuple(self.pix.shape)})")
        dev = _dev_index(self.pix) if device is None else device
        n = self.n_samples
        if self.psi is not None:
            _tensor("psi", self.psi, shape=(n,), dtypes=_floats(), device=dev)
        elif self.streams != "T":
            raise ValueError(f"psi is needed for streams {self.streams!r}")
        if self.tod is not None:
            _tensor("tod", self.tod, shape=(self.n_streams, n), dtypes=_floats(), device=dev)
        elif need_tod:
            raise ValueError("tod is needed by this call")

    def c_struct(self, device=None, need_tod: bool = False) -> dst_problem:
        import torch
        self.validate(device, need_tod)
        s = dst_problem()
        s.n_samples = self.n_samples
        s.n_pix = int(self.n_pix)
        s.baseline_length = int(self.baseline_length)
        s.streams = STREAMS[self.streams]
        s.tod_dtype = 0 if self.tod is None else (DST_F32 if self.tod.dtype == torch.float32 else DST_F64)
        s.psi_dtype = 0 if self.psi is None else (DST_F32 if self.psi.dtype == torch.float32 else DST_F64)
        s.reserved = 0
        s.pix = self.pix.data_ptr()
        s.psi = None if self.psi is None else self.psi.data_ptr()
        s.tod = None if self.tod is None else self.tod.data_ptr()
        for k in range(3):
            s.weight[k] = float(self.weights[k])
        s.rcond_cut = float(self.rcond_cut)
        return s


def to_device(p, device="cuda:0", tod_dtype=None, psi_dtype=None, rcond_cut: float = 1e-3) -> Problem:
    """Copy a host problem (``synth.Problem``-like: numpy pix/psi/tod) to the GPU."""
    import numpy as np
    import torch
    pix = torch.from_numpy(np.ascontiguousarray(p.pix, dtype=np.int32)).to(device)
    psi = None
    if p.psi is not None:
        arr = np.ascontiguousarray(p.psi)
        if psi_dtype is not None:
            arr = arr.astype(psi_dtype)
        psi = torch.from_numpy(arr).to(device)
    arr = np.ascontiguousarray(p.tod)
    if tod_dtype is not None:
        arr = arr.astype(tod_dtype)
    tod = torch.from_numpy(arr).to(device)
    return Problem(pix, psi, tod, p.n_pix, p.baseline_length, p.streams, tuple(p.weights), rcond_cut)


def _empty(shape, dtype, device):
    import torch
    return torch.empty(shape, dtype=dtype, device=device)


def dst_synchronize(ctx: Context) -> None:
    """Wait for the current stream; raise DstError (DST_EBOUNDS) for a device-detected error since the last report."""
    ctx.check(ctx.lib.dst_synchronize(ctx.handle, _stream()))


def dst_pixel_setup(ctx: Context, prob: Problem):
    """Hits [n_pix] int32, blocks [n_pix][4] f64 (M_II, M_QQ, M_QU, M_UU), valid [n_pix] uint8 (asynchronous)."""
    import torch
    s = prob.c_struct(ctx.device)
    dev = prob.pix.device
    hits = _empty((prob.n_pix,), torch.int32, dev)
    blocks = _empty((prob.n_pix, 4), torch.float64, dev)
    valid = _empty((prob.n_pix,), torch.uint8, dev)
    ctx.check(ctx.lib.dst_pixel_setup(ctx.handle, ctypes.byref(s), _ptr(hits), _ptr(blocks), _ptr(valid), _stream()))
    return hits, blocks, valid


def dst_bin(ctx: Context, prob: Problem, baselines=None, use_tod: bool = True, as_map: bool = False):
    """Sum maps s = A^T W (d - F a) (or the map M^-1 s with ``as_map``) [n_pix][3], and hits (asynchronous)."""
    import torch
    s = prob.c_struct(ctx.device, need_tod=use_tod)
    if baselines is not None:
        _tensor("baselines", baselines, shape=(prob.n_streams, prob.n_baselines), dtypes=_f64(), device=ctx.device)
    dev = prob.pix.device
    out = _empty((prob.n_pix, 3), torch.float64, dev)
    hits = _empty((prob.n_pix,), torch.int32, dev)
    flags = (DST_BIN_USE_TOD if use_tod else 0) | (DST_BIN_MAP if as_map else 0)
    ctx.check(ctx.lib.dst_bin(ctx.handle, ctypes.byref(s), _ptr(baselines), flags, _ptr(out), _ptr(hits), _stream()))
    return out, hits


def dst_bin_noalloc(ctx: Context, prob: Problem, map_out, hits_out=None, baselines=None, use_tod: bool = True,
                    as_map: bool = False):
    """As ``dst_bin``, into caller-given ``map_out`` [n_pix][3] f64 (and ``hits_out`` [n_pix] int32), with the
    library's fixed scratch: the call allocates no device memory (n_pix <= 786432)."""
    import torch
    s = prob.c_struct(ctx.device, need_tod=use_tod)
    if baselines is not None:
        _tensor("baselines", baselines, shape=(prob.n_streams, prob.n_baselines), dtypes=_f64(), device=ctx.device)
    _tensor("map_out", map_out, shape=(prob.n_pix, 3), dtypes=_f64(), device=ctx.device)
    if hits_out is not None:
        _tensor("hits_out", hits_out, shape=(prob.n_pix,), dtypes=(torch.int32,), device=ctx.device)
    flags = (DST_BIN_USE_TOD if use_tod else 0) | (DST_BIN_MAP if as_map else 0)
    ctx.check(ctx.lib.dst_bin_noalloc(ctx.handle, ctypes.byref(s), _ptr(baselines), flags, _ptr(map_out),
                                      _ptr(hits_out), _stream()))
    return map_out, hits_out


def dst_unbin(ctx: Context, prob: Problem, m):
    """Timelines A m [n_streams][n_samples] f64 from a map [n_pix][3] f64 (asynchronous)."""
    import torch
    s = prob.c_struct(ctx.device)
    _tensor("map", m, shape=(prob.n_pix, 3), dtypes=_f64(), device=ctx.device)
    out = _empty((prob.n_streams, prob.n_samples), torch.float64, prob.pix.device)
    ctx.check(ctx.lib.dst_unbin(ctx.handle, ctypes.byref(s), _ptr(m), _ptr(out), _stream()))
    return out


def dst_baseline_reduce(ctx: Context, prob: Problem, x):
    """F^T W x over valid samples, [n_streams][n_b] f64; x float32/float64 [n_streams][n_samples] (asynchronous)."""
    import torch
    s = prob.c_struct(ctx.device)
    _tensor("x", x, shape=(prob.n_streams, prob.n_samples), dtypes=_floats(), device=ctx.device)
    out = _empty((prob.n_streams, prob.n_baselines), torch.float64, prob.pix.device)
    s.tod_dtype = DST_F32 if x.dtype == torch.float32 else DST_F64
    ctx.check(ctx.lib.dst_baseline_reduce(ctx.handle, ctypes.byref(s), _ptr(x), _ptr(out), _stream()))
    return out


def dst_residual(ctx: Context, prob: Problem, a=None, use_tod: bool = True):
    """F^T Z (d - F a), [n_streams][n_b] f64 (d = 0 without ``use_tod``; asynchronous)."""
    import torch
    s = prob.c_struct(ctx.device, need_tod=use_tod)
    if a is not None:
        _tensor("a", a, shape=(prob.n_streams, prob.n_baselines), dtypes=_f64(), device=ctx.device)
    out = _empty((prob.n_streams, prob.n_baselines), torch.float64, prob.pix.device)
    if not use_tod:
        s.tod = None
    ctx.check(ctx.lib.dst_residual(ctx.handle, ctypes.byref(s), _ptr(a), _ptr(out), _stream()))
    return out


def dst_apply_operator(ctx: Context, prob: Problem, v):
    """K v = F^T Z F v, [n_streams][n_b] f64."""
    import torch
    s = prob.c_struct(ctx.device)
    _tensor("v", v, shape=(prob.n_streams, prob.n_baselines), dtypes=_f64(), device=ctx.device)
    out = _empty((prob.n_streams, prob.n_baselines), torch.float64, prob.pix.device)
    ctx.check(ctx.lib.dst_apply_operator(ctx.handle, ctypes.byref(s), _ptr(v), _ptr(out), _stream()))
    return out


def _opts(tol, max_iter, check_every, flags, restart, a0):
    opts = dst_solve_opts()
    opts.tol = tol
    opts.max_iter = max_iter
    opts.check_every = check_every
    opts.flags = flags
    opts.restart = restart
    opts.a0 = None if a0 is None else a0.data_ptr()
    return opts


def _info_dict(info) -> dict:
    out = {k: getattr(info, k) for k, _ in dst_solve_info._fields_}
    out["n_valid_pix"] = tuple(info.n_valid_pix)
    out["n_valid_samples"] = tuple(info.n_valid_samples)
    return out


def dst_solve(ctx: Context, prob: Problem, tol: float = 1e-10, max_iter: int = 1000, a0=None, flags: int = 0,
              check_every: int = 0, maps: bool = True, allow_noconv: bool = True, restart: int = 0) -> dict:
    """Destripe: baselines, destriped and binned maps, hits and solver info."""
    import torch
    s = prob.c_struct(ctx.device, need_tod=True)
    if a0 is not None:
        _tensor("a0", a0, shape=(prob.n_streams, prob.n_baselines), dtypes=_f64(), device=ctx.device)
    dev = prob.pix.device
    a = _empty((prob.n_streams, prob.n_baselines), torch.float64, dev)
    m = _empty((prob.n_pix, 3), torch.float64, dev) if maps else None
    mb = _empty((prob.n_pix, 3), torch.float64, dev) if maps else None
    hits = _empty((prob.n_pix,), torch.int32, dev)
    opts = _opts(tol, max_iter, check_every, flags, restart, a0)
    info = dst_solve_info()
    allow = (DST_OK, DST_ENOCONV) if allow_noconv else (DST_OK,)
    rc = ctx.check(ctx.lib.dst_solve(ctx.handle, ctypes.byref(s), ctypes.byref(opts), _ptr(a), _ptr(m), _ptr(mb),
                                     _ptr(hits), ctypes.byref(info), _stream()), allow)
    out = _info_dict(info)
    out.update(status=rc, baselines=a, destriped_map=m, binned_map=mb, hits=hits)
    return out


def dst_solve_batched(ctx: Context, probs, tol: float = 1e-10, max_iter: int = 1000, flags: int = 0,
                      check_every: int = 0, maps: bool = True, allow_noconv: bool = True):
    """Destripe a list of problems in one call; problems sharing pix/psi/weights are solved together.

    Returns (status, [dict per problem]) with the keys of ``dst_solve``'s result.
    """
    import torch
    n = len(probs)
    structs = (dst_problem * n)(*[p.c_struct(ctx.device, need_tod=True) for p in probs])
    outs = []
    for p in probs:
        dev = p.pix.device
        outs.append(dict(
            baselines=_empty((p.n_streams, p.n_baselines), torch.float64, dev),
            destriped_map=_empty((p.n_pix, 3), torch.float64, dev) if maps else None,
            binned_map=_empty((p.n_pix, 3), torch.float64, dev) if maps else None,
            hits=_empty((p.n_pix,), torch.int32, dev)))

    def ptrs(key):
        if not maps and key in ("destriped_map", "binned_map"):
            return None
        return (ctypes.c_void_p * n)(*[o[key].data_ptr() for o in outs])

    opts = _opts(tol, max_iter, check_every, flags, 0, None)
    infos = (dst_solve_info * n)()
    allow = (DST_OK, DST_ENOCONV) if allow_noconv else (DST_OK,)
    b, m, mb, h = ptrs("baselines"), ptrs("destriped_map"), ptrs("binned_map"), ptrs("hits")
    rc = ctx.check(ctx.lib.dst_solve_batched(ctx.handle, n, structs, ctypes.byref(opts), b, m, mb, h, infos,
                                             _stream()), allow)
    res = []
    for o, info in zip(outs, infos):
        d = _info_dict(info)
        d.update(o)
        res.append(d)
    return rc, res


def dst_pointing_expand(ctx: Context, spec, nside: int, n_samples: int, start: int = 0, psi_dtype=None,
                        with_psi: bool = True, device=None):
    """Pointing of samples start .. start + n_samples - 1 of a scan, computed on the GPU.

    ``spec`` is any object with the ``dst_scan`` field names (``synth.ScanSpec``).
    Returns (pix int32 [n], psi [n] float64 / float32 or None).
    """
    import torch
    device = device or f"cuda:{ctx.device}"
    sc = dst_scan(*[float(getattr(spec, f)) for f in SCAN_FIELDS])
    pix = _empty((n_samples,), torch.int32, device)
    dt = torch.float32 if psi_dtype in ("float32", torch.float32) or getattr(psi_dtype, "__name__", "") == "float32" \
        else torch.float64
    psi = _empty((n_samples,), dt, device) if with_psi else None
    code = DST_F32 if dt == torch.float32 else DST_F64
    ctx.check(ctx.lib.dst_pointing_expand(ctx.handle, ctypes.byref(sc), int(nside), int(start), int(n_samples),
                                          _ptr(pix), _ptr(psi), code, _stream()))
    return pix, psi


def dst_noise_generate(ctx: Context, seed: int, stream_id: int, n_samples: int, segment: int,
                       sample_rate_hz: float, sigma: float, fknee_hz: float, alpha: float, out=None,
                       dtype=None, accumulate: bool = False, device=None):
    """White + 1/f noise timeline on the GPU (into ``out`` when given; added to it with ``accumulate``).

    ``out``: contiguous float32/float64 tensor on the context's GPU with at least n_samples elements.
    """
    import torch
    device = device or f"cuda:{ctx.device}"
    if out is None:
        out = torch.zeros((n_samples,), dtype=dtype or torch.float64, device=device)
    _tensor("out", out, dtypes=_floats(), device=ctx.device, min_numel=int(n_samples))
    code = DST_F32 if out.dtype == torch.float32 else DST_F64
    ctx.check(ctx.lib.dst_noise_generate(ctx.handle, int(seed), int(stream_id), int(n_samples), int(segment),
                                         float(sample_rate_hz), float(sigma), float(fknee_hz), float(alpha),
                                         _ptr(out), code, DST_NOISE_ACCUMULATE if accumulate else 0, _stream()))
    return out
