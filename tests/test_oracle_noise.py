"""Pins of the noise oracle (oracle/noise.py) against references outside it.

* Philox4x64-10 against NumPy's own Philox bit generator (the published
  generator as a library routine; NumPy increments the counter before each
  block, so its first block for counter c is the block of c + 1).
* Box-Muller normals: moments and a Kolmogorov-Smirnov test against the
  normal law; a cosine through the filter comes out scaled by exactly the
  Eq. 1 gain at its frequency; band powers of a long timeline follow Eq. 1.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import noise as N


def plus_one(c):
    c = [int(x) for x in c]
    for i in range(4):
        c[i] = (c[i] + 1) % (1 << 64)
        if c[i] != 0:
            break
    return c


@pytest.mark.parametrize("seed", range(6))
def test_philox_matches_numpy(seed):
    rng = np.random.default_rng(seed)
    ctr = [int(x) for x in rng.integers(0, 2 ** 63, size=4, dtype=np.int64)]
    if seed == 1:
        ctr[0] = (1 << 64) - 1  # carry into the second word
    if seed == 2:
        ctr = [(1 << 64) - 1] * 3 + [5]
    key = [int(x) for x in rng.integers(0, 2 ** 63, size=2, dtype=np.int64)]
    ref = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array(key, dtype=np.uint64)).random_raw(8)
    c1 = plus_one(ctr)
    c2 = plus_one(c1)
    got = N.philox4x64_10(np.array([c1, c2], dtype=np.uint64), np.array([key, key], dtype=np.uint64))
    assert np.array_equal(got.reshape(-1), ref)


def test_mulhilo_against_python_integers():
    rng = np.random.default_rng(7)
    a = rng.integers(0, 2 ** 63, size=1000, dtype=np.int64).astype(np.uint64) * np.uint64(2) + np.uint64(1)
    b = rng.integers(0, 2 ** 63, size=1000, dtype=np.int64).astype(np.uint64) * np.uint64(2)
    hi, lo = N.mulhilo64(a, b)
    for x, y, h, l in zip(a[:200], b[:200], hi[:200], lo[:200]):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l) == p & ((1 << 64) - 1)


def test_white_is_standard_normal():
    x = np.concatenate([N.white_segment(11, 3, j, 1 << 16) for j in range(4)])
    n = x.size
    assert abs(x.mean()) < 5 / np.sqrt(n)
    assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(stats.kurtosis(x)) < 0.05
    assert stats.kstest(x, "norm").pvalue > 1e-3
    # different segments / streams / seeds are different draws
    a, b, c = N.white_segment(11, 3, 0, 4096), N.white_segment(11, 4, 0, 4096), N.white_segment(12, 3, 0, 4096)
    for u, v in ((a, b), (a, c), (b, c)):
        assert abs(np.corrcoef(u, v)[0, 1]) < 5 / np.sqrt(4096)
    # a prefix is the same draw
    assert np.array_equal(N.white_segment(11, 3, 2, 1000), N.white_segment(11, 3, 2, 4096)[:1000])


def test_filter_gain_on_a_cosine():
    S, fs, fk, al = 1 << 12, 50.0, 0.7, 1.6
    g = N.filter_gain(S, fs, fk, al)
    t = np.arange(S)
    for k0 in (1, 3, 100, S // 2 - 1):
        x = np.cos(2 * np.pi * k0 * t / S)
        y = np.fft.irfft(np.fft.rfft(x) * g, n=S)
        f0 = k0 * fs / S
        assert np.allclose(y, np.sqrt(1.0 + (fk / f0) ** al) * x, rtol=0, atol=1e-11 * (fk / f0) ** (al / 2) + 1e-12)
    assert g[0] == 1.0


def test_timeline_spectrum_follows_eq1():
    S, fs, sigma, fk, al = 1 << 16, 50.0, 2e-3, 0.5, 1.7
    x = N.noise_timeline(5, 0, 8 * S, S, fs, sigma, fk, al)
    acc = np.zeros(S // 2 + 1)
    for j in range(8):
        acc += np.abs(np.fft.rfft(x[j * S:(j + 1) * S])) ** 2 / S
    acc /= 8
    f = np.fft.rfftfreq(S, 1.0 / fs)
    ratio = acc[1:] / (sigma ** 2 * (1.0 + (fk / f[1:]) ** al))
    for lo, hi in ((0.01, 0.1), (0.1, 1.0), (1.0, 10.0), (10.0, 25.0)):
        band = (f[1:] >= lo) & (f[1:] < hi)
        assert abs(ratio[band].mean() - 1.0) < 0.1, (lo, hi)


def test_timeline_cut_is_a_prefix():
    a = N.noise_timeline(1, 2, 3000, 1024, 50.0, 1e-3, 0.1, 1.5)
    b = N.noise_timeline(1, 2, 3072, 1024, 50.0, 1e-3, 0.1, 1.5)
    assert np.array_equal(a, b[:3000])
