"""On-GPU pointing expansion (dst_pointing_expand) against the generator.

The generator (synth.scan.pointing, NumPy) and the HIP kernel evaluate the
same expressions from the same per-period table (C library functions on both
sides), so pixel indices must agree bit for bit and angles exactly, at every
resolution, for sample ranges starting anywhere in a year-long scan.
"""
import numpy as np
import pytest

from synth import ScanSpec, pointing
from problems import TOY_SCAN

pytestmark = pytest.mark.gpu

SPECS = {
    "default": ScanSpec(),
    "toy": TOY_SCAN,
    "south_fast": ScanSpec(spin_period_s=2.0, sidereal_day_s=120.0, elevation_deg=45.0, latitude_deg=-20.0,
                           az0_deg=17.3, lst0_rad=1.1, psi0_deg=12.5),
    "steep": ScanSpec(sample_rate_hz=100.0, spin_period_s=30.0, elevation_deg=80.0, latitude_deg=60.0,
                      az0_deg=-40.0, lst0_rad=-2.0, psi0_deg=-90.0),
}


@pytest.fixture(scope="module")
def ctx():
    from paper_1309_5609_amd import dst
    c = dst.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("name", list(SPECS))
@pytest.mark.parametrize("nside", [1, 8, 64, 256, 512, 2048])
def test_expand_bit_exact(ctx, name, nside):
    from paper_1309_5609_amd import dst
    spec = SPECS[name]
    for start, n in ((0, 600_000), (1_576_800_000 - 250_000, 250_001), (123_457, 1)):
        pix_ref, psi_ref = pointing(spec, nside, n, start=start)
        pix, psi = dst.dst_pointing_expand(ctx, spec, nside, n, start=start)
        p = pix.cpu().numpy()
        bad = np.flatnonzero(p != pix_ref)
        assert bad.size == 0, (name, nside, start, bad[:5], p[bad[:5]], pix_ref[bad[:5]])
        assert np.array_equal(psi.cpu().numpy(), psi_ref)


def test_expand_fp32_angle_and_no_angle(ctx):
    from paper_1309_5609_amd import dst
    import torch
    spec = SPECS["default"]
    pix_ref, psi_ref = pointing(spec, 256, 100_000, start=77)
    pix, psi = dst.dst_pointing_expand(ctx, spec, 256, 100_000, start=77, psi_dtype=torch.float32)
    assert psi.dtype == torch.float32
    assert np.array_equal(psi.cpu().numpy(), psi_ref.astype(np.float32))
    pix2, none = dst.dst_pointing_expand(ctx, spec, 256, 100_000, start=77, with_psi=False)
    assert none is None and np.array_equal(pix2.cpu().numpy(), pix_ref)


def test_expand_errors(ctx):
    from paper_1309_5609_amd import dst
    bad = ScanSpec(spin_period_s=60.01)  # not a whole number of samples per period
    for spec, nside, n in ((bad, 64, 10), (ScanSpec(), 0, 10), (ScanSpec(), 64, 0),
                           (ScanSpec(latitude_deg=90.0), 64, 10)):
        with pytest.raises(dst.DstError) as e:
            dst.dst_pointing_expand(ctx, spec, nside, n)
        assert e.value.code == -1
