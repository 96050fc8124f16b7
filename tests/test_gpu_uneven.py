"""Uneven batches: independent problems with their own pointing solved together.

dst_solve_batched advances problems that share no operator (the channels of
a survey: different scans, lengths, baseline lengths, stream sets, resolutions)
with one launch per PCG phase over all of them.  Each problem must meet the
single solve's bars against the FP64 oracle (hits bit-exact, baselines and
destriped maps within 1e-9 relative at tolerance 1e-13, binned maps within
1e-12), stop on its own, and replay from the captured graph with the same bits
as launches one by one.
"""
import numpy as np
import pytest

from oracle import destripe as O
from problems import TOY_SCAN, args, toy
from synth import ScanSpec, make_problem

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def ctx():
    from paper_1309_5609_amd import dst
    c = dst.Context(0)
    yield c
    c.close()


def survey():
    """Five problems: different scans (spin phase, angle offset), lengths, L, N_side and stream sets."""
    return [
        toy(n_samples=30000, L=300, nside=16, cfg=320, scan=ScanSpec(spin_period_s=6.0, sidereal_day_s=1800.0,
                                                                      az0_deg=45.0, psi0_deg=22.5)),
        toy(n_samples=12011, L=211, nside=8, cfg=321, streams="T"),
        toy(n_samples=20000, L=500, nside=16, cfg=322, streams="QU",
            scan=ScanSpec(spin_period_s=6.0, sidereal_day_s=1800.0, az0_deg=90.0, psi0_deg=45.0)),
        toy(n_samples=20000, L=400, nside=8, cfg=323, streams="IQU"),
        toy(n_samples=9100, L=250, nside=8, cfg=324, mask_fraction=0.05),
    ]


def check(p, out, tol=1e-13):
    ref = O.solve(*args(p), tol=tol, max_iter=3000)
    assert out["converged"] == 1
    assert np.array_equal(out["hits"].cpu().numpy(), ref.hits)
    assert rel(out["baselines"].cpu().numpy(), ref.baselines) < 1e-9
    ok = ref.valid_T if p.streams in ("T", "IQU") else (ref.hits > 0)
    if p.streams == "QU":
        ok = ref.valid_QU
    m = out["destriped_map"].cpu().numpy()
    assert rel(m[ok], ref.destriped_map[ok]) < 1e-9
    assert rel(out["binned_map"].cpu().numpy()[ok], ref.binned_map[ok]) < 1e-12
    assert out["true_rel_residual"] < 1e-11
    return ref


def test_uneven_batch_matches_oracle(ctx):
    from paper_1309_5609_amd import dst
    ps = survey()
    rc, res = dst.dst_solve_batched(ctx, [dst.to_device(p) for p in ps], tol=1e-13, max_iter=3000)
    assert rc == 0
    for p, out in zip(ps, res):
        check(p, out)
    # at the benchmark tolerance every problem takes its own number of steps, as the oracle does
    rc, res10 = dst.dst_solve_batched(ctx, [dst.to_device(p) for p in ps], tol=1e-10, max_iter=3000)
    its = []
    for p, out in zip(ps, res10):
        ref = O.solve(*args(p), tol=1e-10, max_iter=3000)
        assert abs(out["iterations"] - ref.iterations) <= 1
        its.append(out["iterations"])
    assert len(set(its)) > 1


def test_uneven_graph_replay_is_bit_identical(ctx):
    from paper_1309_5609_amd import dst
    ps = survey()
    dps = [dst.to_device(p) for p in ps]
    _, a = dst.dst_solve_batched(ctx, dps, tol=1e-12, max_iter=3000)
    _, b = dst.dst_solve_batched(ctx, dps, tol=1e-12, max_iter=3000, flags=dst.DST_SOLVE_NO_GRAPH)
    _, c = dst.dst_solve_batched(ctx, dps, tol=1e-12, max_iter=3000, flags=dst.DST_SOLVE_PROFILE)
    for x, y, z in zip(a, b, c):
        assert x["iterations"] == y["iterations"] == z["iterations"]
        assert np.array_equal(x["baselines"].cpu().numpy(), y["baselines"].cpu().numpy())
        assert np.array_equal(x["destriped_map"].cpu().numpy(), y["destriped_map"].cpu().numpy())
        assert np.array_equal(x["baselines"].cpu().numpy(), z["baselines"].cpu().numpy())
    assert c[0]["t_bin_ms"] > 0 and c[0]["t_unbin_ms"] > 0 and c[0]["t_update_ms"] > 0


def test_uneven_batch_matches_single_solves(ctx):
    from paper_1309_5609_amd import dst
    ps = survey()
    dps = [dst.to_device(p) for p in ps]
    _, res = dst.dst_solve_batched(ctx, dps, tol=1e-10, max_iter=3000)
    for d, out in zip(dps, res):
        one = dst.dst_solve(ctx, d, tol=1e-10, max_iter=3000)
        assert out["iterations"] == one["iterations"]
        assert rel(out["baselines"].cpu().numpy(), one["baselines"].cpu().numpy()) < 1e-12


def test_uneven_fp32_and_stopped_problem(ctx):
    """FP32 channels with an intensity stream; one problem has no signal and no noise (b = 0: stops at once)."""
    from paper_1309_5609_amd import dst
    ps = survey()[:3]
    zero = toy(n_samples=8000, L=200, nside=8, cfg=325, noise=False, signal=False)
    dps = [dst.to_device(p, tod_dtype=np.float32, psi_dtype=np.float32 if p.psi is not None else None)
           for p in ps + [zero]]
    rc, res = dst.dst_solve_batched(ctx, dps, tol=1e-12, max_iter=3000)
    assert rc == 0
    assert res[3]["iterations"] == 0 and np.all(res[3]["baselines"].cpu().numpy() == 0.0)
    sigma = 1e-3
    for p, out in zip(ps, res[:3]):
        q = p.astype(np.float32, np.float32)
        psi = None if q.psi is None else q.psi.astype(np.float64)
        ref = O.solve(q.pix, psi, q.tod.astype(np.float64), p.n_pix, p.baseline_length, p.streams, p.weights,
                      tol=1e-12, max_iter=3000)
        for k in range(ref.baselines.shape[0]):
            err = np.sqrt(np.mean((out["baselines"].cpu().numpy()[k] - ref.baselines[k]) ** 2))
            assert err <= 1e-4 * sigma / np.sqrt(p.baseline_length)
        assert np.array_equal(out["hits"].cpu().numpy(), ref.hits)


def test_uneven_with_split_graph_member(ctx):
    from paper_1309_5609_amd import dst
    from test_gpu_components import split_problem
    ps = [split_problem("TQU"), survey()[0], split_problem("T", realization=1)]
    rc, res = dst.dst_solve_batched(ctx, [dst.to_device(p) for p in ps], tol=1e-13, max_iter=3000)
    assert rc == 0
    assert res[0]["n_components"] == 3 and res[1]["n_components"] == 1 and res[2]["n_components"] == 3
    for p, out in zip(ps, res):
        check(p, out)


@pytest.mark.parametrize("env", [("DST_BIN_LPP", "4"), ("DST_BIN_LPP", "8"), ("DST_BIN_LPP", "16"),
                                 ("DST_BIN_LPP", "32"), ("DST_UNBIN_BPW", "1"), ("DST_UNBIN_BPW", "2"),
                                 ("DST_UNBIN_BPW", "8")])
def test_uneven_launch_shapes_agree(ctx, env):
    """Every lanes-per-pixel of the group binning and baselines-per-wavefront of the group rescan gives the
    solve of the default shapes (chosen from each kind's runs per pixel), summation order aside."""
    import os
    from paper_1309_5609_amd import dst
    ps = survey()
    dps = [dst.to_device(p) for p in ps]
    _, ref = dst.dst_solve_batched(ctx, dps, tol=1e-13, max_iter=3000)
    os.environ[env[0]] = env[1]
    try:
        c = dst.Context(0)
    finally:
        del os.environ[env[0]]
    try:
        _, res = dst.dst_solve_batched(c, dps, tol=1e-13, max_iter=3000)
    finally:
        c.close()
    for x, y in zip(res, ref):
        assert abs(x["iterations"] - y["iterations"]) <= 1
        assert rel(x["baselines"].cpu().numpy(), y["baselines"].cpu().numpy()) < 1e-10
