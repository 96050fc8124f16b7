"""IQU radiometer rows (streams DST_IQU) on the GPU against the FP64 oracle.

One stream per detector with pointing row (1, cos 2psi, sin 2psi): the full
3x3 per-pixel block and its eigenvalue cut, the operator, the solve (PCG and
GMRES), and the maps, at the same bars as the polarimeter streams.
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
    "plain": dict(n_samples=20000, L=400),
    "masked": dict(n_samples=20000, L=400, mask_fraction=0.07),
    "ragged": dict(n_samples=19037, L=311),
    "L37": dict(n_samples=6001, L=37),
    "nside16": dict(n_samples=60000, L=500, nside=16),
}


def make(name):
    return toy(streams="IQU", **VARIANTS[name])


@pytest.mark.parametrize("name", list(VARIANTS))
def test_iqu_operator(ctx, name):
    from paper_1309_5609_amd import dst
    import torch
    p = make(name)
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    v = np.random.default_rng(4).standard_normal((1, p.n_baselines))
    Kv = dst.dst_apply_operator(ctx, dst.to_device(p), torch.from_numpy(v).cuda()).cpu().numpy()
    assert rel(Kv, O.K_compact(st, v)) < 1e-12


@pytest.mark.parametrize("solver", ["pcg", "gmres"])
@pytest.mark.parametrize("name", list(VARIANTS))
def test_iqu_solve(ctx, name, solver):
    from paper_1309_5609_amd import dst
    p = make(name)
    ref = O.solve(*args(p), tol=1e-13, max_iter=3000, solver=solver)
    flags = dst.DST_SOLVE_GMRES if solver == "gmres" else 0
    out = dst.dst_solve(ctx, dst.to_device(p), tol=1e-13, max_iter=3000, flags=flags)
    assert out["converged"] == 1
    assert np.array_equal(out["hits"].cpu().numpy(), ref.hits)
    assert out["n_valid_pix"][0] == int(ref.valid_T.sum())
    assert out["n_valid_pix"][0] < int((ref.hits > 0).sum())  # the 3x3 cut drops pixels here
    # with few valid pixels the baseline-pixel graph splits into components, each with its own
    # null vector; both sides report zero mean per component, so they compare directly
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    _, lab = O.t_components(st)
    assert out["n_components"] == len(np.unique(lab[lab >= 0]))
    assert rel(out["baselines"].cpu().numpy(), ref.baselines) < 1e-9
    ok = ref.valid_T
    assert rel(out["destriped_map"].cpu().numpy()[ok], ref.destriped_map[ok]) < 1e-9
    assert rel(out["binned_map"].cpu().numpy()[ok], ref.binned_map[ok]) < 1e-12
    assert np.all(out["destriped_map"].cpu().numpy()[~ok] == 0.0)
    assert abs(out["iterations"] - ref.iterations) <= 2


def test_iqu_signal_only_null_baselines(ctx):
    from paper_1309_5609_amd import dst
    p = toy(streams="IQU", noise=False, n_samples=20000, L=400)
    out = dst.dst_solve(ctx, dst.to_device(p), tol=1e-10)
    assert np.max(np.abs(out["baselines"].cpu().numpy())) <= 1e-12 * np.sqrt(np.mean(p.tod ** 2))
    ref = O.solve(*args(p), tol=1e-10)
    ok = ref.valid_T
    assert rel(out["destriped_map"].cpu().numpy()[ok], p.sky[ok]) < 1e-11


def test_iqu_in_batched_call_and_errors(ctx):
    from paper_1309_5609_amd import dst
    pa, pb = make("plain"), toy(streams="IQU", n_samples=20000, L=400, realization=1,
                                pointing_arrays=(make("plain").pix, make("plain").psi))
    da = dst.to_device(pa)
    db = dst.Problem(da.pix, da.psi, dst.to_device(pb).tod, da.n_pix, da.baseline_length, "IQU", da.weights)
    rc, res = dst.dst_solve_batched(ctx, [da, db], tol=1e-13, max_iter=3000)
    assert rc == 0
    for p, out in zip((pa, pb), res):
        ref = O.solve(*args(p), tol=1e-13, max_iter=3000)
        assert rel(out["baselines"].cpu().numpy(), ref.baselines) < 1e-9
    for call in (lambda: dst.dst_bin(ctx, da), lambda: dst.dst_pixel_setup(ctx, da),
                 lambda: dst.dst_solve(ctx, da, flags=dst.DST_SOLVE_PER_SAMPLE)):
        with pytest.raises(dst.DstError) as e:
            call()
        assert e.value.code == -1
