"""Synthetic spinning ground scan: telescope pointing -> (pixel, polarisation angle).

Stands in for the B-Machine pointing the paper destripes (Polarimeters data
section; scanning strategy paragraph of the simulation section), which is not
available: a telescope at fixed elevation spins about its vertical axis while
the sky turns overhead, so every revolution draws a circle on the sky that
drifts slowly in right ascension and produces the crossing points destriping
relies on (Introduction).

Spherical astronomy used (textbook alt-az -> equatorial transform):

* ``sin(dec) = sin(el) sin(lat) + cos(el) cos(lat) cos(az)``
* hour angle ``H = atan2(-sin(az) cos(el), cos(lat) sin(el) - sin(lat) cos(el) cos(az))``
* ``RA = LST - H``
* parallactic angle ``q = atan2(sin H, tan(lat) cos(dec) - sin(dec) cos H)``

The polarisation angle of a channel is ``psi = q + psi0`` (the footnote on the
parallactic angle in the Algorithm section).  Because declination, hour
angle and parallactic angle depend on azimuth only, they repeat every spin
period; only the right ascension advances with sidereal time.

This module is input synthesis, shared by both sides of every comparison.  It
holds no step of the destriping method.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

from .healpix_ring import ang2pix_ring_z

SIDEREAL_DAY_S = 86164.0905


@dataclass(frozen=True)
class ScanSpec:
    sample_rate_hz: float = 50.0
    spin_period_s: float = 60.0
    elevation_deg: float = 60.0
    latitude_deg: float = 37.5
    az0_deg: float = 0.0
    lst0_rad: float = 0.0
    psi0_deg: float = 0.0
    sidereal_day_s: float = SIDEREAL_DAY_S


def one_period(spec: ScanSpec, n_period: int):
    """Declination, hour angle and polarisation angle over one spin period.

    Returns ``(dec, hour_angle, psi)`` float64 arrays of length ``n_period``
    for samples ``i = 0..n_period-1`` at ``t = i / sample_rate``.  Evaluated
    element by element with the C library's functions (``math``), in the
    order written, so that any consumer calling the same library on the same
    expressions gets the same bits (the table is only ``n_period`` long).
    """
    el = math.radians(spec.elevation_deg)
    lat = math.radians(spec.latitude_deg)
    az0 = math.radians(spec.az0_deg)
    psi0 = math.radians(spec.psi0_deg)
    dec = np.empty(n_period)
    ha = np.empty(n_period)
    psi = np.empty(n_period)
    for i in range(n_period):
        t = float(i) / spec.sample_rate_hz
        az = az0 + 2.0 * math.pi * t / spec.spin_period_s
        sin_dec = math.sin(el) * math.sin(lat) + math.cos(el) * math.cos(lat) * math.cos(az)
        d = math.asin(min(1.0, max(-1.0, sin_dec)))
        h = math.atan2(-math.sin(az) * math.cos(el), math.cos(lat) * math.sin(el) - math.sin(lat) * math.cos(el) * math.cos(az))
        q = math.atan2(math.sin(h), math.tan(lat) * math.cos(d) - math.sin(d) * math.cos(h))
        dec[i], ha[i], psi[i] = d, h, q + psi0
    return dec, ha, psi


def period_z(dec: np.ndarray) -> np.ndarray:
    """cos(colatitude) of each table entry, element by element with ``math``."""
    return np.array([math.cos(0.5 * math.pi - d) for d in dec])


def samples_per_period(spec: ScanSpec) -> int:
    n = spec.sample_rate_hz * spec.spin_period_s
    if abs(n - round(n)) > 1e-9:
        raise ValueError("spin period must hold a whole number of samples")
    return int(round(n))


def pointing(spec: ScanSpec, nside: int, n_samples: int, start: int = 0, chunk: int = 1 << 22):
    """Pixel index (int32, RING) and polarisation angle (float64) per sample.

    Samples ``start .. start + n_samples - 1`` of the scan.  Work is chunked so
    peak memory stays near ``chunk`` samples of temporaries.
    """
    n_per = samples_per_period(spec)
    dec, ha, psi_per = one_period(spec, n_per)
    z_per = period_z(dec)
    pix = np.empty(n_samples, dtype=np.int32)
    psi = np.empty(n_samples, dtype=np.float64)

    def work(c0):
        c1 = min(n_samples, c0 + chunk)
        idx = np.arange(start + c0, start + c1, dtype=np.int64)
        ph = idx % n_per
        t = idx.astype(np.float64) / spec.sample_rate_hz
        lst = spec.lst0_rad + 2.0 * np.pi * t / spec.sidereal_day_s
        ra = lst - ha[ph]
        pix[c0:c1] = ang2pix_ring_z(nside, z_per[ph], ra).astype(np.int32)
        psi[c0:c1] = psi_per[ph]

    starts = list(range(0, n_samples, chunk))
    if len(starts) > 1:
        # chunks are independent; NumPy releases the GIL inside its kernels
        with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            list(ex.map(work, starts))
    else:
        for c0 in starts:
            work(c0)
    return pix, psi
