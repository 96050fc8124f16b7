"""Small seeded problems shared by the oracle pins and the GPU parity tests."""
import numpy as np

from synth import ScanSpec, make_problem

# A fast toy scan: 6 s spin (300 samples at 50 Hz) and a sky that turns once
# every 1800 s, so successive circles drift and cross.
TOY_SCAN = ScanSpec(spin_period_s=6.0, sidereal_day_s=1800.0)


def toy(n_samples=9100, L=250, nside=8, streams="TQU", cfg=300, **kw):
    kw.setdefault("fknee_hz", 0.5)
    kw.setdefault("alpha", 1.5)
    return make_problem(nside=nside, n_samples=n_samples, baseline_length=L, streams=streams, cfg=cfg,
                        scan=kw.pop("scan", TOY_SCAN), **kw)


def tiny(n_samples=1500, L=110, nside=4, streams="TQU", cfg=301, **kw):
    kw.setdefault("fknee_hz", 0.5)
    kw.setdefault("alpha", 1.5)
    return make_problem(nside=nside, n_samples=n_samples, baseline_length=L, streams=streams, cfg=cfg,
                        scan=kw.pop("scan", ScanSpec(spin_period_s=2.0, sidereal_day_s=120.0)), **kw)


def args(p):
    """Positional arguments for the oracle's entry points."""
    return p.pix, p.psi, p.tod, p.n_pix, p.baseline_length, p.streams, p.weights
