"""Pins of the input generators: HEALPix RING geometry, scan geometry, 1/f noise."""
import numpy as np
import pytest

from synth import ScanSpec, ang2pix_ring, make_problem, nside2npix, pix2ang_ring, pointing
from synth.healpix_ring import ring_of_pixel_counts
from synth.noise import one_over_f, segmented
from synth.scan import one_period


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 64, 256, 512])
def test_ring_round_trip_all_centres(nside):
    p = np.arange(nside2npix(nside))
    th, ph = pix2ang_ring(nside, p)
    assert np.array_equal(ang2pix_ring(nside, th, ph), p)


@pytest.mark.parametrize("nside", [1, 4, 16, 256, 512])
def test_ring_structure(nside):
    counts = ring_of_pixel_counts(nside)
    assert counts.sum() == 12 * nside * nside
    assert counts.size == 4 * nside - 1
    # pixels of one ring share z; z decreases ring by ring
    p = np.arange(nside2npix(nside))
    th, _ = pix2ang_ring(nside, p)
    starts = np.concatenate([[0], np.cumsum(counts)])
    zs = []
    for i in range(counts.size):
        z = np.cos(th[starts[i]:starts[i + 1]])
        assert np.ptp(z) < 1e-12
        zs.append(z[0])
    assert np.all(np.diff(zs) < 0)
    # closed forms: polar ring i at z = 1 - i^2/(3N^2); belt rings at 4/3 - 2i/(3N)
    for i in range(1, nside):
        assert abs(zs[i - 1] - (1 - i * i / (3.0 * nside * nside))) < 1e-12
    for i in range(nside, 3 * nside + 1):
        assert abs(zs[i - 1] - (4.0 / 3.0 - 2.0 * i / (3.0 * nside))) < 1e-12


@pytest.mark.parametrize("nside", [256, 512])
def test_points_near_a_centre_fall_in_its_pixel(nside):
    """Directions a small fraction of a pixel away from a centre map to that pixel (the benchmark resolutions)."""
    rng = np.random.default_rng(nside)
    p = rng.integers(0, nside2npix(nside), 200000)
    th, ph = pix2ang_ring(nside, p)
    size = np.sqrt(4 * np.pi / nside2npix(nside))
    dth = rng.uniform(-0.05, 0.05, p.size) * size
    dph = rng.uniform(-0.05, 0.05, p.size) * size / np.maximum(np.sin(th), 1e-12)
    # stay clear of the poles, where the phi jitter is not small in angle
    keep = np.sin(th) > 4 * size
    got = ang2pix_ring(nside, np.clip(th + dth, 0, np.pi), np.mod(ph + dph, 2 * np.pi))
    assert np.array_equal(got[keep], p[keep])


def test_poles_and_boundaries():
    n = 8
    assert set(ang2pix_ring(n, np.zeros(4) + 1e-9, np.array([0.1, 1.7, 3.3, 4.9]))) == {0, 1, 2, 3}
    npix = nside2npix(n)
    assert set(ang2pix_ring(n, np.full(4, np.pi - 1e-9), np.array([0.1, 1.7, 3.3, 4.9]))) == {npix - 4, npix - 3,
                                                                                            npix - 2, npix - 1}
    # continuity across z = 2/3 and phi = 0 / 2 pi: nearby points land on neighbouring pixels
    eps = 1e-10
    th = np.arccos(2.0 / 3.0)
    for ph in np.linspace(0.01, 6.2, 25):
        a = ang2pix_ring(n, np.array([th - eps]), np.array([ph]))[0]
        b = ang2pix_ring(n, np.array([th + eps]), np.array([ph]))[0]
        ta, pa = pix2ang_ring(n, [a])
        tb, pb = pix2ang_ring(n, [b])
        # both centres lie within one pixel size of the query point
        assert abs(ta[0] - th) < 2.5 / n and abs(tb[0] - th) < 2.5 / n
    assert ang2pix_ring(n, np.array([1.0]), np.array([2 * np.pi - 1e-13]))[0] == \
        ang2pix_ring(n, np.array([1.0]), np.array([-1e-13]))[0]


def test_equal_area_poisson():
    """Uniform directions fill every pixel with Poisson counts (equal-area property)."""
    n = 4
    npix = nside2npix(n)
    rng = np.random.default_rng(5)
    N = 400_000
    z = rng.uniform(-1, 1, N)
    ph = rng.uniform(0, 2 * np.pi, N)
    c = np.bincount(ang2pix_ring(n, np.arccos(z), ph), minlength=npix)
    lam = N / npix
    chi2 = np.sum((c - lam) ** 2 / lam)
    dof = npix - 1
    assert abs(chi2 - dof) < 5 * np.sqrt(2 * dof)


def test_scan_geometry():
    spec = ScanSpec()
    dec, ha, psi = one_period(spec, 3000)
    # fixed elevation 60 deg at latitude 37.5 deg spans dec in [lat - 30, lat + 30]
    assert abs(np.rad2deg(dec.max()) - 67.5) < 1e-6
    assert abs(np.rad2deg(dec.min()) - 7.5) < 1e-3
    # at az = 0 (north, between zenith and pole) the hour angle is 0 and the
    # parallactic angle is 180 deg
    assert abs(ha[0]) < 1e-12 and abs(abs(psi[0]) - np.pi) < 1e-12
    pix, ps = pointing(spec, 64, 12000)
    # declination, hour angle and psi repeat each spin period; pixels drift with sidereal time
    assert np.array_equal(ps[:3000], ps[3000:6000])
    assert pix.min() >= 0 and pix.max() < nside2npix(64)


def test_noise_white_and_psd():
    rng = np.random.Generator(np.random.PCG64(1))
    w = one_over_f(rng, 1 << 18, 50.0, 2e-3, 0.0, 1.7)
    assert abs(w.std() / 2e-3 - 1) < 0.01
    # periodogram of 1/f noise follows sigma^2 (1 + (fk/f)^alpha) up to chi^2_2 scatter
    n, fs, sg, fk, al = 1 << 20, 50.0, 1e-3, 0.5, 1.5
    x = segmented([7, 7], n, n, fs, sg, fk, al)
    X = np.fft.rfft(x)
    f = np.fft.rfftfreq(n, 1 / fs)
    per = np.abs(X[1:]) ** 2 / n  # E = sigma^2 (1 + (fk/f)^alpha)
    model = sg * sg * (1 + (fk / f[1:]) ** al)
    ratio = per / model
    # average over log-spaced bands: mean 1 within statistical error
    edges = np.unique(np.geomspace(1, ratio.size, 20).astype(int))
    for a, b in zip(edges[:-1], edges[1:]):
        if b - a < 50:
            continue
        seg = ratio[a:b]
        assert abs(seg.mean() - 1) < 5 / np.sqrt(seg.size)


def test_problem_reproducible_and_signal_only():
    kw = dict(nside=8, n_samples=9000, baseline_length=300, cfg=150,
              scan=ScanSpec(spin_period_s=6.0))
    a = make_problem(**kw)
    b = make_problem(**kw)
    assert np.array_equal(a.pix, b.pix) and np.array_equal(a.tod, b.tod)
    s = make_problem(noise=False, **kw)
    c, sn = np.cos(2 * s.psi), np.sin(2 * s.psi)
    sky = s.sky[s.pix]
    assert np.allclose(s.tod[0], sky[:, 0], rtol=0, atol=1e-18)
    assert np.allclose(s.tod[1], sky[:, 1] * c + sky[:, 2] * sn, rtol=0, atol=1e-18)
    assert np.allclose(s.tod[2], -sky[:, 1] * sn + sky[:, 2] * c, rtol=0, atol=1e-18)


def test_one_over_f_torch_spectrum():
    """The torch generator follows the same spectrum: band powers / (sigma^2 (1 + (f_k/f)^alpha)) near 1."""
    import torch
    from synth.noise import one_over_f_torch
    n, fs, sigma, fk, alpha = 2 ** 18, 50.0, 1e-3, 0.5, 1.7
    acc = np.zeros(n // 2 + 1)
    for s in range(8):
        g = torch.Generator(device="cpu")
        g.manual_seed(100 + s)
        x = one_over_f_torch(g, n, fs, sigma, fk, alpha, device="cpu").numpy()
        acc += np.abs(np.fft.rfft(x)) ** 2 / n
    acc /= 8
    f = np.fft.rfftfreq(n, 1.0 / fs)
    model = sigma ** 2 * (1.0 + (fk / f[1:]) ** alpha)
    ratio = acc[1:] / model
    for lo, hi in ((0.01, 0.1), (0.1, 1.0), (1.0, 10.0), (10.0, 25.0)):
        band = (f[1:] >= lo) & (f[1:] < hi)
        assert abs(ratio[band].mean() - 1.0) < 0.1, (lo, hi, ratio[band].mean())
