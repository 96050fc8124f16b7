"""White plus 1/f noise timelines by FFT filtering (Introduction, Eq. 1).

The paper gives the correlated-noise spectrum only up to a constant,
``P(f) ~ sigma^2 [1 + (f_k / f)^alpha]``.  The reading used here: draw white
Gaussian noise ``w ~ N(0, sigma^2)`` and multiply its discrete Fourier
transform by ``sqrt(1 + (f_k / f)^alpha)``, leaving the zero-frequency bin
untouched (factor 1), so the white level stays ``sigma`` and the correlated
part has zero mean.  ``f_k = 0`` returns the white noise unchanged.

Long timelines can be generated in independent segments (each segment is one
FFT), which keeps host memory bounded for multi-day inputs.

This module is input synthesis, shared by both sides of every comparison.  It
holds no step of the destriping method.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft


def one_over_f(rng: np.random.Generator, n: int, sample_rate_hz: float, sigma: float, fknee_hz: float,
               alpha: float, workers: int = -1) -> np.ndarray:
    """One timeline of ``n`` float64 samples with the spectrum of Eq. (1)."""
    w = rng.standard_normal(n) * sigma
    if fknee_hz <= 0.0 or n < 2:
        return w
    spec = sfft.rfft(w, workers=workers)
    del w
    f = np.fft.rfftfreq(n, d=1.0 / sample_rate_hz)
    gain = np.ones_like(f)
    gain[1:] = np.sqrt(1.0 + (fknee_hz / f[1:]) ** alpha)
    spec *= gain
    del gain, f
    return sfft.irfft(spec, n=n, workers=workers)


def segmented(seed_words, n: int, segment: int, sample_rate_hz: float, sigma: float, fknee_hz: float,
              alpha: float, out: np.ndarray | None = None, dtype=np.float64) -> np.ndarray:
    """Timeline of ``n`` samples made of independent segments of ``segment`` samples.

    Segment ``j`` is drawn from ``SeedSequence(list(seed_words) + [j])``.  With
    ``segment >= n`` this is a single FFT over the whole timeline.
    """
    if out is None:
        out = np.empty(n, dtype=dtype)
    segment = max(1, min(int(segment), n)) if n > 0 else 1
    for j, s0 in enumerate(range(0, n, segment)):
        s1 = min(n, s0 + segment)
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed_words) + [j])))
        out[s0:s1] = one_over_f(rng, s1 - s0, sample_rate_hz, sigma, fknee_hz, alpha)
    return out


def one_over_f_torch(gen, n: int, sample_rate_hz: float, sigma: float, fknee_hz: float, alpha: float,
                     device="cuda"):
    """``one_over_f`` on a torch device (same spectrum, torch's generator ``gen``).

    Used where many long realizations are needed at once (the batched Monte
    Carlo benchmark); the draws differ from the NumPy generator's, the
    recipe and spectrum are the same.  Returns float64 on ``device``.
    """
    import torch
    w = torch.randn(n, generator=gen, dtype=torch.float64, device=device) * sigma
    if fknee_hz <= 0.0 or n < 2:
        return w
    spec = torch.fft.rfft(w)
    del w
    f = torch.fft.rfftfreq(n, d=1.0 / sample_rate_hz, dtype=torch.float64, device=device)
    gain = torch.ones_like(f)
    gain[1:] = torch.sqrt(1.0 + (fknee_hz / f[1:]) ** alpha)
    spec *= gain
    del gain, f
    return torch.fft.irfft(spec, n=n)
