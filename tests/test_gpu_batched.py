"""Batched solve (dst_solve_batched) against the FP64 oracle.

Realizations that share the pointing are solved together by the
multi-right-hand-side kernels; every realization must meet the same bars as
the single solve (hits bit-exact, baselines and destriped maps within 1e-9
relative, binned maps within 1e-12), stop on its own, and agree with the
library's single-problem solve.
"""
import numpy as np
import pytest

from oracle import destripe as O
from problems import TOY_SCAN, args, tiny, toy
from synth import pointing

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


def family(n_real, make=toy, scan=TOY_SCAN, freeze_every=0, **kw):
    """n_real problems on one pointing and sky; realization r draws its own noise.  freeze_every > 0: one fixed
    angle on every freeze_every-th observed pixel (shared by all realizations)."""
    base = make(**kw)
    psi = base.psi if base.psi is not None else pointing(scan, base.nside, base.n_samples)[1]
    if freeze_every:
        psi = np.array(psi, copy=True)
        psi[np.isin(base.pix, np.unique(base.pix[base.pix >= 0])[::freeze_every])] = 0.4
        base.psi = psi
    kw2 = {k: v for k, v in kw.items() if k != "mask_fraction"}
    out = [base]
    for r in range(1, n_real):
        out.append(make(realization=r, pointing_arrays=(base.pix, psi), sky=base.sky, **kw2))
    return out


def on_device(probs, **kw):
    """Device problems sharing the first one's pix / psi tensors."""
    from paper_1309_5609_amd import dst
    d0 = dst.to_device(probs[0], **kw)
    out = [d0]
    for p in probs[1:]:
        d = dst.to_device(p, **kw)
        out.append(dst.Problem(d0.pix, d0.psi, d.tod, d0.n_pix, d0.baseline_length, d0.streams, d0.weights,
                               d0.rcond_cut))
    return out


def check_against_oracle(p, out, tol=1e-13):
    ref = O.solve(*args(p), tol=tol, max_iter=3000)
    assert out["converged"] == 1
    assert np.array_equal(out["hits"].cpu().numpy(), ref.hits)
    assert rel(out["baselines"].cpu().numpy(), ref.baselines) < 1e-9
    obs = ref.hits > 0
    assert rel(out["destriped_map"].cpu().numpy()[obs], ref.destriped_map[obs]) < 1e-9
    assert rel(out["binned_map"].cpu().numpy()[obs], ref.binned_map[obs]) < 1e-12
    assert out["true_rel_residual"] < 1e-11
    return ref


VARIANTS = {
    "plain": (4, dict()),
    "masked": (3, dict(mask_fraction=0.07)),
    "ragged": (5, dict(n_samples=9037, L=211)),
    "unequal": (3, dict(weights=(2.0e6, 5.0e6, 0.7e6))),
    "QU": (3, dict(streams="QU")),
    "T": (2, dict(streams="T")),
    "L37": (3, dict(n_samples=3001, L=37)),
    # about 100 runs per pixel: the binning goes through several 63-run windows per pixel
    "dense": (3, dict(n_samples=60000, L=16, nside=2)),
    # a weak u stream and one fixed angle on every fifth pixel: 22 of 88 q/u blocks fail the cut
    "qucut": (3, dict(weights=(1.0e6, 1.0e6, 1.0e2), freeze_every=5)),
}


@pytest.mark.parametrize("name", list(VARIANTS))
def test_batched_matches_oracle(ctx, name):
    from paper_1309_5609_amd import dst
    n, kw = VARIANTS[name]
    probs = family(n, **kw)
    rc, res = dst.dst_solve_batched(ctx, on_device(probs), tol=1e-13, max_iter=3000)
    assert rc == 0
    for p, out in zip(probs, res):
        check_against_oracle(p, out)


def test_batched_equals_single(ctx):
    """The batch and one-at-a-time solves agree and take the same number of steps."""
    from paper_1309_5609_amd import dst
    probs = family(4)
    dps = on_device(probs)
    rc, res = dst.dst_solve_batched(ctx, dps, tol=1e-10)
    assert rc == 0
    for d, out in zip(dps, res):
        one = dst.dst_solve(ctx, d, tol=1e-10)
        assert abs(out["iterations"] - one["iterations"]) <= 1
        assert rel(out["baselines"].cpu().numpy(), one["baselines"].cpu().numpy()) < 1e-8
        assert rel(out["binned_map"].cpu().numpy(), one["binned_map"].cpu().numpy()) < 1e-13
        assert np.array_equal(out["hits"].cpu().numpy(), one["hits"].cpu().numpy())


def test_batched_per_rhs_stop(ctx):
    """Each right-hand side stops on its own: an all-zero one at once (its baselines stay exactly
    zero while the others iterate), the others at the step their single solves stop at."""
    from paper_1309_5609_amd import dst
    import torch
    probs = family(3, fknee_hz=(0.5, 0.5, 0.5))
    probs[1] = toy(realization=1, fknee_hz=0.02, pointing_arrays=(probs[0].pix, probs[0].psi), sky=probs[0].sky)
    dps = on_device(probs)
    zero = dst.Problem(dps[0].pix, dps[0].psi, torch.zeros_like(dps[0].tod), dps[0].n_pix, dps[0].baseline_length,
                       dps[0].streams, dps[0].weights)
    rc, res = dst.dst_solve_batched(ctx, [dps[0], zero, dps[1], dps[2]], tol=1e-12, max_iter=3000)
    assert rc == 0
    assert res[1]["iterations"] == 0 and res[1]["converged"] == 1
    assert torch.count_nonzero(res[1]["baselines"]).item() == 0
    its = []
    for k, p in ((0, probs[0]), (2, probs[1]), (3, probs[2])):
        check_against_oracle(p, res[k], tol=1e-12)
        one = dst.dst_solve(ctx, dps[[0, None, 1, 2][k]], tol=1e-12, max_iter=3000)
        assert abs(res[k]["iterations"] - one["iterations"]) <= 1
        its.append(res[k]["iterations"])
    assert min(its) > 0, its


def test_batched_graph_equals_eager(ctx):
    """Replaying the captured iteration graph gives the same bits as launching each kernel."""
    from paper_1309_5609_amd import dst
    dps = on_device(family(3))
    _, g = dst.dst_solve_batched(ctx, dps, tol=1e-12, check_every=3)
    _, e = dst.dst_solve_batched(ctx, dps, tol=1e-12, check_every=3, flags=dst.DST_SOLVE_NO_GRAPH)
    _, g2 = dst.dst_solve_batched(ctx, dps, tol=1e-12, check_every=3)
    for x, y, z in zip(g, e, g2):
        assert x["iterations"] == y["iterations"] == z["iterations"]
        assert torch_equal(x["baselines"], y["baselines"]) and torch_equal(x["baselines"], z["baselines"])
        assert torch_equal(x["destriped_map"], y["destriped_map"])


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))


def test_single_solve_graph_equals_eager(ctx):
    from paper_1309_5609_amd import dst
    d = on_device([toy()])[0]
    g = dst.dst_solve(ctx, d, tol=1e-12, check_every=4)
    e = dst.dst_solve(ctx, d, tol=1e-12, check_every=4, flags=dst.DST_SOLVE_NO_GRAPH)
    assert g["iterations"] == e["iterations"]
    assert torch_equal(g["baselines"], e["baselines"])
    assert torch_equal(g["destriped_map"], e["destriped_map"])


def test_batched_mixed_groups(ctx):
    """Problems on two pointings plus a lone one: grouped by shared operator, order kept."""
    from paper_1309_5609_amd import dst
    fa = family(3)
    fb = family(2, n_samples=7000, L=300, nside=8, cfg=310)
    lone = toy(n_samples=5000, L=199, cfg=320)
    da, db, dl = on_device(fa), on_device(fb), on_device([lone])
    order = [("a", 0), ("b", 0), ("a", 1), ("l", 0), ("b", 1), ("a", 2)]
    host = {"a": fa, "b": fb, "l": [lone]}
    devs = {"a": da, "b": db, "l": dl}
    rc, res = dst.dst_solve_batched(ctx, [devs[f][i] for f, i in order], tol=1e-13, max_iter=3000)
    assert rc == 0
    for (f, i), out in zip(order, res):
        check_against_oracle(host[f][i], out)


def test_batched_mixed_precision(ctx):
    """FP32 timelines and angles: the error statement of the single mixed solve holds per realization."""
    from paper_1309_5609_amd import dst
    probs = family(3, n_samples=60000, nside=16, L=500)
    rc, res = dst.dst_solve_batched(ctx, on_device(probs, tod_dtype=np.float32, psi_dtype=np.float32), tol=1e-12,
                                    max_iter=3000)
    assert rc == 0
    sigma = 1e-3
    for p, out in zip(probs, res):
        ref = O.solve(*args(p), tol=1e-12, max_iter=3000)
        obs = ref.hits > 0
        L = p.baseline_length
        for k in range(ref.baselines.shape[0]):
            e = np.sqrt(np.mean((out["baselines"][k].cpu().numpy() - ref.baselines[k]) ** 2))
            assert e / (sigma / np.sqrt(L)) <= 1e-3
        noise = np.sqrt(np.mean(sigma ** 2 / ref.hits[obs]))
        m = out["destriped_map"].cpu().numpy()
        for c in range(3):
            e = np.sqrt(np.mean((m[obs, c] - ref.destriped_map[obs, c]) ** 2))
            assert e / noise <= 1e-3


def test_batched_more_than_64(ctx):
    """65 realizations: a group of 64 and the remaining one, each matching the oracle."""
    from paper_1309_5609_amd import dst
    probs = family(65, make=tiny, scan=None)
    rc, res = dst.dst_solve_batched(ctx, on_device(probs), tol=1e-13, max_iter=3000)
    assert rc == 0
    for k in (0, 1, 31, 63, 64):
        check_against_oracle(probs[k], res[k])


def test_batched_errors(ctx):
    from paper_1309_5609_amd import dst
    dps = on_device(family(2))
    with pytest.raises(dst.DstError) as e:
        dst.dst_solve_batched(ctx, [])
    assert e.value.code == -1
    bad = dst.Problem(dps[1].pix, dps[1].psi, dps[1].tod, dps[1].n_pix, dps[1].baseline_length, dps[1].streams,
                      (1.0, -1.0, 1.0))
    with pytest.raises(dst.DstError) as e:
        dst.dst_solve_batched(ctx, [dps[0], bad])
    assert e.value.code == -1 and "problem 1" in str(e.value)
    with pytest.raises(dst.DstError) as e:
        dst.dst_solve_batched(ctx, dps, flags=dst.DST_SOLVE_PER_SAMPLE)
    assert e.value.code == -1
    rc, res = dst.dst_solve_batched(ctx, dps, tol=1e-14, max_iter=2)
    assert rc == 1
    assert all(r["iterations"] == 2 and r["converged"] == 0 for r in res)


def test_batched_workload0(ctx):
    """Three realizations of the 6 h, N_side 64 workload at full size."""
    from paper_1309_5609_amd import dst
    from synth.configs import WORKLOADS, make_problem
    spec = dict(WORKLOADS[0])
    base = make_problem(cfg=0, sigma=1e-3, streams="TQU", **spec)
    probs = [base] + [make_problem(cfg=0, sigma=1e-3, streams="TQU", realization=r,
                                   pointing_arrays=(base.pix, base.psi), sky=base.sky, **spec) for r in (1, 2)]
    rc, res = dst.dst_solve_batched(ctx, on_device(probs), tol=1e-13, max_iter=2000)
    assert rc == 0
    for p, out in zip(probs, res):
        check_against_oracle(p, out)
