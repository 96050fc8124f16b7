"""On-GPU noise (dst_noise_generate) against the noise oracle.

Same Philox words on both sides, so the white normals agree to the rounding
of log / sqrt / sin / cos (bar 1e-13 of the RMS); the filtered timelines to
the rounding of two FFTs (bar 1e-12 of the RMS), for odd and even log2 of the
segment length, ragged ends, an odd number of segments, FP32 output and
accumulation onto an existing timeline.
"""
import numpy as np
import pytest

from oracle import noise as N

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1309_5609_amd import dst
    c = dst.Context(0)
    yield c
    c.close()


def rms(x):
    return float(np.sqrt(np.mean(np.square(x))))


CASES = [
    # seed, stream, n, S, rate, sigma, fknee, alpha
    (1, 0, 4096, 4096, 50.0, 1.0, 0.0, 1.0),
    (2, 5, 1000, 16, 50.0, 1e-3, 0.5, 1.7),
    (3, 1, 3 * 1024 + 7, 1024, 50.0, 1e-3, 0.05, 1.7),
    (4, 2, 5 * 2048, 2048, 100.0, 2e-3, 1.0, 2.0),
    (5, 3, (1 << 15) * 3 - 11, 1 << 15, 50.0, 1e-3, 0.02, 1.0),
    (6, 7, (1 << 20) * 2 + 3, 1 << 20, 50.0, 1e-3, 0.05, 1.7),
    (7, 0, 10, 4, 50.0, 1.0, 3.0, 1.5),
]


@pytest.mark.parametrize("case", CASES)
def test_noise_matches_oracle(ctx, case):
    from paper_1309_5609_amd import dst
    seed, stream, n, S, rate, sigma, fk, al = case
    ref = N.noise_timeline(seed, stream, n, S, rate, sigma, fk, al)
    got = dst.dst_noise_generate(ctx, seed, stream, n, S, rate, sigma, fk, al).cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * rms(ref), (np.max(np.abs(got - ref)), rms(ref))


def test_noise_fp32_and_accumulate(ctx):
    from paper_1309_5609_amd import dst
    import torch
    n, S = 50_000, 1 << 13
    ref = N.noise_timeline(9, 4, n, S, 50.0, 1e-3, 0.05, 1.7)
    got32 = dst.dst_noise_generate(ctx, 9, 4, n, S, 50.0, 1e-3, 0.05, 1.7, dtype=torch.float32)
    assert got32.dtype == torch.float32
    assert np.max(np.abs(got32.cpu().numpy().astype(np.float64) - ref)) <= 1e-6 * rms(ref)
    base = torch.linspace(-1.0, 1.0, n, dtype=torch.float64, device="cuda")
    acc = dst.dst_noise_generate(ctx, 9, 4, n, S, 50.0, 1e-3, 0.05, 1.7, out=base.clone(), accumulate=True)
    assert np.max(np.abs(acc.cpu().numpy() - (base.cpu().numpy() + ref))) <= 1e-12 * (1.0 + rms(ref))


def test_noise_errors(ctx):
    from paper_1309_5609_amd import dst
    import torch
    out = torch.zeros(16, dtype=torch.float64, device="cuda")
    for kw in (dict(segment=12), dict(segment=2), dict(sigma=-1.0), dict(rate=0.0)):
        a = dict(segment=16, sigma=1.0, rate=50.0)
        a.update(kw)
        with pytest.raises(dst.DstError) as e:
            dst.dst_noise_generate(ctx, 1, 0, 16, a["segment"], a["rate"], a["sigma"], 0.1, 1.0, out=out)
        assert e.value.code == -1
