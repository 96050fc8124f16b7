"""Mixed precision: FP32 timelines and angles, FP64 accumulators, inverse and CG.

Error statement against the FP64 oracle, per stream and per map component:
  * total error: GPU on FP32 inputs vs the oracle on the FP64 inputs;
  * arithmetic-only error: GPU on FP32 inputs vs the oracle on the same
    FP32-rounded inputs promoted to FP64.
Bounds (stated in the design notes): baseline RMS error <= 1e-3 sigma / sqrt(L)
per stream; map RMS error <= 1e-3 RMS_p(sigma / sqrt(h_p)) per component; and
the destriped map's error against the sky equals the FP64 one to 1e-3
("equal map RMS accuracy").
"""
import numpy as np
import pytest

from oracle import destripe as O
from problems import args, toy

pytestmark = pytest.mark.gpu
SIGMA = 1e-3


@pytest.fixture(scope="module")
def ctx():
    from paper_1309_5609_amd import dst
    c = dst.Context(0)
    yield c
    c.close()


def rms(x):
    return float(np.sqrt(np.mean(np.square(x))))


def error_statement(p, gpu, ref, sigma=SIGMA):
    """RMS errors of baselines (per stream) and maps (per component)."""
    obs = ref.hits > 0
    L = p.baseline_length
    base = [rms(gpu["baselines"][k] - ref.baselines[k]) / (sigma / np.sqrt(L)) for k in range(ref.baselines.shape[0])]
    noise_rms = rms(sigma / np.sqrt(ref.hits[obs]))
    maps = [rms(gpu["destriped_map"][obs, c] - ref.destriped_map[obs, c]) / noise_rms for c in range(3)]
    return np.array(base), np.array(maps)


def run_mixed(ctx, p, form="runs"):
    from paper_1309_5609_amd import dst
    dp = dst.to_device(p, tod_dtype=np.float32, psi_dtype=np.float32)
    flags = dst.DST_SOLVE_PER_SAMPLE if form == "samples" else 0
    out = dst.dst_solve(ctx, dp, tol=1e-12, max_iter=3000, flags=flags)
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


@pytest.mark.parametrize("form", ["runs", "samples"])
def test_mixed_error_statement_toy(ctx, form):
    p = toy(n_samples=60000, nside=16, L=500)
    gpu = run_mixed(ctx, p, form)
    ref64 = O.solve(*args(p), tol=1e-12, max_iter=3000)
    p32 = p.astype(np.float32, np.float32)
    ref32 = O.solve(p32.pix, p32.psi.astype(np.float64), p32.tod.astype(np.float64), p.n_pix, p.baseline_length,
                    p.streams, p.weights, tol=1e-12, max_iter=3000)
    b_tot, m_tot = error_statement(p, gpu, ref64)
    b_ari, m_ari = error_statement(p, gpu, ref32)
    assert np.all(b_tot <= 1e-3) and np.all(m_tot <= 1e-3), (b_tot, m_tot)
    # the arithmetic alone (FP32 run records, FP64 accumulation) stays far below the input rounding
    assert np.all(b_ari <= 1e-4) and np.all(m_ari <= 1e-4), (b_ari, m_ari)
    assert np.array_equal(gpu["hits"], ref64.hits)


def test_mixed_equal_map_accuracy_workload0(ctx):
    """Workload 0 at full size: FP32-input map error vs the sky equals the FP64 one."""
    from paper_1309_5609_amd import dst
    from synth import workload
    p = workload(0)
    gpu32 = run_mixed(ctx, p)
    out64 = dst.dst_solve(ctx, dst.to_device(p), tol=1e-12, max_iter=3000)
    m64 = out64["destriped_map"].cpu().numpy()
    obs = out64["hits"].cpu().numpy() > 0
    for c in range(3):
        e32 = rms(gpu32["destriped_map"][obs, c] - p.sky[obs, c])
        e64 = rms(m64[obs, c] - p.sky[obs, c])
        assert abs(e32 / e64 - 1) <= 1e-3, (c, e32, e64)
    ref64 = O.solve(*args(p), tol=1e-12, max_iter=3000)
    b_tot, m_tot = error_statement(p, gpu32, ref64)
    assert np.all(b_tot <= 1e-3) and np.all(m_tot <= 1e-3), (b_tot, m_tot)
