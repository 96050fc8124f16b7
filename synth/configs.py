"""Seeded synthetic destriping problems with the shapes of the benchmark workloads.

A problem is what the paper's destriper consumes (Algorithm section, data
model and Eqs. 2-8): per-sample HEALPix pixel indices, the polarisation angle
psi, and calibrated timelines for the streams of one channel, T (intensity),
q and u, in kelvin, plus the fixed baseline length in samples (Polarimeters
data section) and the white-noise weights ``1/sigma^2``.

Timelines follow the data model with pointing rows ``A_T = (1, 0, 0)``,
``A_q = (0, cos 2psi, sin 2psi)`` and ``A_u = (0, -sin 2psi, cos 2psi)``
(Eqs. 3-6):

    d_T = I[p] + n_T,   d_q = Q[p] cos2psi + U[p] sin2psi + n_q,
    d_u = -Q[p] sin2psi + U[p] cos2psi + n_u,

with the sky an i.i.d. Gaussian map per pixel and ``n`` white + 1/f noise
(Eq. 1).  Optional injected offsets add ``a_true[k][t // L]`` to stream k.

Seeds: ``SeedSequence([1309, 5609, cfg, role, channel, realization, stream])``
with role 0 = sky, 1 = noise, PCG64 bit generator.

The named workloads (sizes are the benchmark's):

* ``workload(0)``: 6 h at 50 Hz (1,080,000 samples), N_side 64, L = 3000,
  f_k = 50 mHz, alpha = 1.7, sigma = 1 mK, FP64.
* ``workload(1, fknee_hz=...)``: 30 days at 50 Hz (129,600,000 samples),
  N_side 256, L = 3000, f_k in {20, 50, 200} mHz, alpha = 1.7, FP64.
* ``workload(2)``: workload 1's data with timelines and angles rounded to FP32.
* ``realizations(...)``: independent noise realizations over one pointing.

This module is input synthesis, shared by both sides of every comparison.  It
holds no step of the destriping method.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from .healpix_ring import nside2npix
from .noise import segmented
from .scan import ScanSpec, pointing

# "r": one stream of a polarisation-sensitive radiometer, d = I + Q cos 2psi + U sin 2psi
STREAM_INDEX = {"T": 0, "q": 1, "u": 2, "r": 0}
STREAM_SETS = {"TQU": ("T", "q", "u"), "QU": ("q", "u"), "T": ("T",), "IQU": ("r",)}

DAY_S = 86400.0


@dataclass
class Problem:
    """One channel's destriping input, host arrays (numpy)."""

    pix: np.ndarray  # int32 [n_t], -1 = masked sample
    psi: np.ndarray | None  # float64/float32 [n_t] radians, None for T-only
    tod: np.ndarray  # float64/float32 [n_streams][n_t], kelvin
    n_pix: int
    baseline_length: int
    streams: str  # "TQU", "QU" or "T"
    weights: tuple  # (w_T, w_q, w_u), 1/K^2
    nside: int = 0
    sky: np.ndarray | None = None  # float64 [n_pix][3] (I, Q, U)
    offsets: np.ndarray | None = None  # injected offsets [n_streams][n_b] or None
    meta: dict = field(default_factory=dict)

    @property
    def n_samples(self) -> int:
        return int(self.pix.shape[0])

    @property
    def n_baselines(self) -> int:
        return -(-self.n_samples // self.baseline_length)

    def astype(self, tod_dtype, psi_dtype) -> "Problem":
        """Copy with timelines / angles rounded to other float types."""
        return Problem(self.pix, None if self.psi is None else self.psi.astype(psi_dtype),
                       self.tod.astype(tod_dtype), self.n_pix, self.baseline_length, self.streams,
                       self.weights, self.nside, self.sky, self.offsets, dict(self.meta))


def _rng(*words) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1309, 5609, *words])))


def gaussian_sky(n_pix: int, cfg: int, sigma_i: float = 1e-3, sigma_pol: float = 1e-4) -> np.ndarray:
    """i.i.d. Gaussian I/Q/U map, float64 [n_pix][3] in kelvin."""
    sky = np.empty((n_pix, 3), dtype=np.float64)
    for k, sg in enumerate((sigma_i, sigma_pol, sigma_pol)):
        sky[:, k] = _rng(cfg, 0, 0, 0, k).standard_normal(n_pix) * sg
    return sky


def signal_timelines(sky: np.ndarray, pix: np.ndarray, psi, streams: str, out: np.ndarray,
                     chunk: int = 1 << 22) -> None:
    """Add the sky seen through the pointing to ``out`` [n_streams][n_t] (Eqs. 2-6)."""
    names = STREAM_SETS[streams]
    n = pix.shape[0]

    def work(c0):
        c1 = min(n, c0 + chunk)
        p = pix[c0:c1]
        good = p >= 0
        pp = np.where(good, p, 0)
        if psi is not None:
            two = 2.0 * psi[c0:c1].astype(np.float64)
            c, s = np.cos(two), np.sin(two)
        for row, name in enumerate(names):
            if name == "T":
                sig = sky[pp, 0]
            elif name == "r":
                sig = sky[pp, 0] + sky[pp, 1] * c + sky[pp, 2] * s
            elif name == "q":
                sig = sky[pp, 1] * c + sky[pp, 2] * s
            else:
                sig = -sky[pp, 1] * s + sky[pp, 2] * c
            out[row, c0:c1] += np.where(good, sig, 0.0)

    starts = list(range(0, n, chunk))
    if len(starts) > 1:
        with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            list(ex.map(work, starts))
    else:
        for c0 in starts:
            work(c0)


def make_problem(*, nside: int, n_samples: int, baseline_length: int, streams: str = "TQU",
                 sigma=1e-3, fknee_hz=0.05, alpha=1.7, sample_rate_hz: float = 50.0,
                 scan: ScanSpec | None = None, cfg: int = 100, channel: int = 0, realization: int = 0,
                 signal: bool = True, noise: bool = True, offsets_rms: float = 0.0,
                 weights=None, mask_fraction: float = 0.0, noise_segment: int | None = None,
                 sky: np.ndarray | None = None, pointing_arrays=None, threads: int = 3) -> Problem:
    """Build one seeded problem.

    ``sigma`` / ``fknee_hz`` / ``alpha`` may be scalars or 3-tuples per stream
    (T, q, u).  ``weights`` defaults to ``1/sigma^2`` per stream.
    ``mask_fraction`` > 0 marks random samples as masked (pix = -1).
    """
    if streams not in STREAM_SETS:
        raise ValueError(streams)
    scan = scan or ScanSpec(sample_rate_hz=sample_rate_hz)
    n_pix = nside2npix(nside)
    names = STREAM_SETS[streams]

    def per_stream(v):
        return tuple(v) if np.ndim(v) else (v, v, v)

    sig3, fk3, al3 = per_stream(sigma), per_stream(fknee_hz), per_stream(alpha)
    if weights is None:
        weights = tuple(1.0 / (s * s) for s in sig3)

    if pointing_arrays is None:
        pix, psi = pointing(scan, nside, n_samples)
    else:
        pix, psi = pointing_arrays
    if mask_fraction > 0:
        pix = pix.copy()
        m = _rng(cfg, 2, channel, realization, 9).random(n_samples) < mask_fraction
        pix[m] = -1
    if streams == "T":
        psi_out = None
    else:
        psi_out = psi

    if sky is None:
        sky = gaussian_sky(n_pix, cfg)
    tod = np.zeros((len(names), n_samples), dtype=np.float64)

    seg = noise_segment if noise_segment else n_samples

    def gen_noise(row_name):
        row, name = row_name
        k = STREAM_INDEX[name]
        segmented([cfg, 1, channel, realization, k], n_samples, seg, scan.sample_rate_hz, sig3[k], fk3[k], al3[k],
                  out=tod[row])

    if noise:
        with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
            list(ex.map(gen_noise, list(enumerate(names))))
    if signal:
        signal_timelines(sky, pix, psi, streams, tod)
    offsets = None
    L = int(baseline_length)
    n_b = -(-n_samples // L)
    if offsets_rms > 0:
        offsets = np.empty((len(names), n_b), dtype=np.float64)
        for row, name in enumerate(names):
            offsets[row] = _rng(cfg, 3, channel, realization, STREAM_INDEX[name]).standard_normal(n_b) * offsets_rms
            tod[row] += np.repeat(offsets[row], L)[:n_samples]
    return Problem(pix=pix, psi=psi_out, tod=tod, n_pix=n_pix, baseline_length=L, streams=streams,
                   weights=tuple(float(w) for w in weights), nside=nside, sky=sky, offsets=offsets,
                   meta=dict(cfg=cfg, sigma=sig3, fknee_hz=fk3, alpha=al3, sample_rate_hz=scan.sample_rate_hz))


WORKLOADS = {
    0: dict(nside=64, n_samples=1_080_000, baseline_length=3000, fknee_hz=0.05, alpha=1.7),
    1: dict(nside=256, n_samples=129_600_000, baseline_length=3000, fknee_hz=0.05, alpha=1.7),
}


def workload(cfg: int, fknee_hz: float | None = None, n_samples: int | None = None, **kw) -> Problem:
    """Benchmark workload ``cfg`` (0, 1 or 2), optionally truncated to ``n_samples``."""
    base = 1 if cfg == 2 else cfg
    spec = dict(WORKLOADS[base])
    if fknee_hz is not None:
        spec["fknee_hz"] = fknee_hz
    if n_samples is not None:
        spec["n_samples"] = int(n_samples)
    spec.update(kw)
    prob = make_problem(cfg=base, sigma=1e-3, streams="TQU", **spec)
    prob.meta["workload"] = cfg
    if cfg == 2:
        prob = prob.astype(np.float32, np.float32)
        prob.meta["workload"] = 2
    return prob


def realizations(n_real: int, *, nside: int, n_samples: int, baseline_length: int, fknee_hz: float = 0.05,
                 alpha: float = 1.7, sigma: float = 1e-3, cfg: int = 3, tod_dtype=np.float32):
    """``n_real`` noise realizations sharing one pointing and sky.

    Returns ``(pix, psi, tod[n_real][3][n_t], sky, weights)``.
    """
    pix, psi = pointing(ScanSpec(), nside, n_samples)
    n_pix = nside2npix(nside)
    sky = gaussian_sky(n_pix, 1)
    tod = np.empty((n_real, 3, n_samples), dtype=tod_dtype)
    sig = np.zeros((3, n_samples), dtype=np.float64)
    signal_timelines(sky, pix, psi, "TQU", sig)
    for r in range(n_real):
        for k in range(3):
            n = segmented([cfg, 1, 0, r, k], n_samples, n_samples, 50.0, sigma, fknee_hz, alpha)
            tod[r, k] = (sig[k] + n).astype(tod_dtype)
    w = 1.0 / (sigma * sigma)
    return pix, psi.astype(tod_dtype), tod, sky, (w, w, w)
