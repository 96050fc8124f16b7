"""Oracle of the on-GPU Monte Carlo noise generator: white + 1/f noise (Eq. 1).

TEST INFRASTRUCTURE ONLY: imported by tests/ (and nothing in the product path).

Definition of the generated timeline (the recipe the library's
``dst_noise_generate`` implements, written out plainly here):

* Random bits: Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random
  numbers: as easy as 1, 2, 3", SC 2011): 10 rounds of
  ``(X0, X1, X2, X3) -> (hi(M1 X2) ^ X1 ^ K0, lo(M1 X2), hi(M0 X0) ^ X3 ^ K1,
  lo(M0 X0))`` with the key bumped by the Weyl constants between rounds.
  Block ``b`` of segment ``j`` uses counter ``(b, j, 0, 0)`` and key
  ``(seed, stream)``.
* Uniforms from the top 53 bits: ``u1 = (w0 >> 11 + 1) 2^-53`` in (0, 1],
  ``u2 = (w1 >> 11) 2^-53`` in [0, 1); Box-Muller gives
  ``sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2)``; a block's four words give
  four normals in order; sample ``k`` of a segment is normal ``k`` of it.
* Each segment of ``S`` samples (S a power of two; the last segment of a
  timeline is drawn at full length and cut) is ``sigma`` times those
  normals, filtered in the Fourier domain by ``sqrt(1 + (f_k / |f|)^alpha)``
  with the zero-frequency bin left unchanged (the reading of Eq. 1 the input
  generator uses: white level ``sigma``, zero-mean correlated part).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
MASK32 = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)


def mulhilo64(a, b):
    """(high, low) 64-bit words of the 128-bit product of uint64 arrays."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a0, a1 = a & MASK32, a >> S32
    b0, b1 = b & MASK32, b >> S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> S32) + (p01 & MASK32) + (p10 & MASK32)
    hi = p11 + (p01 >> S32) + (p10 >> S32) + (mid >> S32)
    return hi, a * b


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds on counters ``ctr`` (..., 4) and keys ``key`` (..., 2); uint64."""
    x = [np.asarray(ctr, dtype=np.uint64)[..., i].copy() for i in range(4)]
    k0 = np.asarray(key, dtype=np.uint64)[..., 0].copy()
    k1 = np.asarray(key, dtype=np.uint64)[..., 1].copy()
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = mulhilo64(M0, x[0])
            hi1, lo1 = mulhilo64(M1, x[2])
            x = [hi1 ^ x[1] ^ k0, lo1, hi0 ^ x[3] ^ k1, lo0]
    return np.stack(x, axis=-1)


def white_segment(seed: int, stream: int, segment: int, n: int) -> np.ndarray:
    """The first ``n`` unit normals of segment ``segment`` (n a multiple of 4 or not)."""
    nb = -(-n // 4)
    ctr = np.zeros((nb, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(nb, dtype=np.uint64)
    ctr[:, 1] = np.uint64(segment)
    key = np.empty((nb, 2), dtype=np.uint64)
    key[:, 0] = np.uint64(seed)
    key[:, 1] = np.uint64(stream)
    w = philox4x64_10(ctr, key)
    scale = 2.0 ** -53
    out = np.empty((nb, 4))
    for pair in (0, 1):
        u1 = ((w[:, 2 * pair] >> np.uint64(11)).astype(np.float64) + 1.0) * scale
        u2 = (w[:, 2 * pair + 1] >> np.uint64(11)).astype(np.float64) * scale
        r = np.sqrt(-2.0 * np.log(u1))
        out[:, 2 * pair] = r * np.cos(2.0 * np.pi * u2)
        out[:, 2 * pair + 1] = r * np.sin(2.0 * np.pi * u2)
    return out.reshape(-1)[:n]


def filter_gain(S: int, sample_rate_hz: float, fknee_hz: float, alpha: float) -> np.ndarray:
    """Real-FFT gains of a segment of S samples: 1 at f = 0, sqrt(1 + (f_k/f)^alpha) elsewhere."""
    f = np.fft.rfftfreq(S, d=1.0 / sample_rate_hz)
    g = np.ones_like(f)
    if fknee_hz > 0.0:
        g[1:] = np.sqrt(1.0 + (fknee_hz / f[1:]) ** alpha)
    return g


def noise_timeline(seed: int, stream: int, n: int, S: int, sample_rate_hz: float, sigma: float, fknee_hz: float,
                   alpha: float) -> np.ndarray:
    """``n`` samples of white + 1/f noise: segments of S samples, each filtered on its own."""
    if S < 4 or S & (S - 1):
        raise ValueError("segment length must be a power of two >= 4")
    g = filter_gain(S, sample_rate_hz, fknee_hz, alpha)
    out = np.empty(n)
    for j, s0 in enumerate(range(0, n, S)):
        w = sigma * white_segment(seed, stream, j, S)
        x = np.fft.irfft(np.fft.rfft(w) * g, n=S)
        out[s0:s0 + S] = x[:min(S, n - s0)]
    return out
