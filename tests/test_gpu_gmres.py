"""Restarted GMRES on the GPU (DST_SOLVE_GMRES) against the oracle's GMRES and PCG.

The two implementations orthogonalise differently (the library: classical
Gram-Schmidt twice; the oracle: modified Gram-Schmidt), so iterates agree to
rounding and iteration counts within two; solutions meet the FP64 bar (1e-9
relative to the oracle at tolerance 1e-13).
"""
import numpy as np
import pytest

from oracle import destripe as O
from problems import args, toy

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


VARIANTS = {
    "plain": dict(),
    "masked": dict(mask_fraction=0.07),
    "ragged": dict(n_samples=9037, L=211),
    "unequal": dict(weights=(2.0e6, 5.0e6, 0.7e6)),
    "QU": dict(streams="QU"),
    "T": dict(streams="T"),
}


@pytest.mark.parametrize("restart", [30, 6])
@pytest.mark.parametrize("name", list(VARIANTS))
def test_gmres_matches_oracle(ctx, name, restart):
    from paper_1309_5609_amd import dst
    p = toy(**VARIANTS[name])
    ref = O.solve(*args(p), tol=1e-13, max_iter=3000, solver="gmres", restart=restart)
    out = dst.dst_solve(ctx, dst.to_device(p), tol=1e-13, max_iter=3000, flags=dst.DST_SOLVE_GMRES, restart=restart)
    assert out["converged"] == 1
    assert abs(out["iterations"] - ref.iterations) <= 2, (out["iterations"], ref.iterations)
    assert rel(out["baselines"].cpu().numpy(), ref.baselines) < 1e-9
    obs = ref.hits > 0
    assert rel(out["destriped_map"].cpu().numpy()[obs], ref.destriped_map[obs]) < 1e-9
    assert out["true_rel_residual"] < 1e-11


def test_gmres_equals_pcg(ctx):
    from paper_1309_5609_amd import dst
    d = dst.to_device(toy(n_samples=30000, nside=16))
    g = dst.dst_solve(ctx, d, tol=1e-12, flags=dst.DST_SOLVE_GMRES)
    c = dst.dst_solve(ctx, d, tol=1e-12)
    assert rel(g["baselines"].cpu().numpy(), c["baselines"].cpu().numpy()) < 1e-9


def test_gmres_workload0(ctx):
    from paper_1309_5609_amd import dst
    from synth import workload
    p = workload(0)
    ref = O.solve(*args(p), tol=1e-12, max_iter=2000, solver="gmres", restart=50)
    out = dst.dst_solve(ctx, dst.to_device(p), tol=1e-12, max_iter=2000, flags=dst.DST_SOLVE_GMRES)
    assert abs(out["iterations"] - ref.iterations) <= 2
    assert rel(out["baselines"].cpu().numpy(), ref.baselines) < 1e-9


def test_gmres_limits_and_errors(ctx):
    from paper_1309_5609_amd import dst
    d = dst.to_device(toy())
    out = dst.dst_solve(ctx, d, tol=1e-14, max_iter=3, flags=dst.DST_SOLVE_GMRES)
    assert out["status"] == 1 and out["iterations"] == 3 and out["converged"] == 0
    for kw in (dict(restart=5), dict(restart=200, flags=dst.DST_SOLVE_GMRES)):
        with pytest.raises(dst.DstError) as e:
            dst.dst_solve(ctx, d, **kw)
        assert e.value.code == -1
    # resume from a previous GMRES solution
    first = dst.dst_solve(ctx, d, tol=1e-12, flags=dst.DST_SOLVE_GMRES | dst.DST_SOLVE_NO_CANON)
    again = dst.dst_solve(ctx, d, tol=1e-6, flags=dst.DST_SOLVE_GMRES, a0=first["baselines"])
    assert again["iterations"] <= 1
