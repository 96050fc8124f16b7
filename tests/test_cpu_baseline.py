"""The all-core C++ CPU baseline against the NumPy oracle (host only).

The benchmark times it beside the GPU library, so it must compute the same
thing: the operator of Eq. 13 within 1e-12 relative, and the solve
(baselines canonical per connected part, destriped map, hits) within 1e-9
at tolerance 1e-13 with the same number of CG steps.
"""
import numpy as np
import pytest

from oracle import cpu_baseline as C
from oracle import destripe as O
from problems import args, toy


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module", autouse=True)
def built():
    C.build()


VARIANTS = {
    "plain": dict(),
    "masked": dict(mask_fraction=0.07),
    "ragged": dict(n_samples=9037, L=211),
    "unequal": dict(weights=(2.0e6, 5.0e6, 0.7e6)),
    "QU": dict(streams="QU"),
    "T": dict(streams="T"),
}


@pytest.mark.parametrize("name", list(VARIANTS))
def test_operator_matches_oracle(name):
    p = toy(**VARIANTS[name])
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    v = np.random.default_rng(7).standard_normal((p.tod.shape[0], p.n_baselines))
    for threads in (1, 3):
        Kv, _, _, nth = C.apply_K(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights, v, threads=threads)
        assert nth == threads
        assert rel(Kv, O.K_compact(st, v)) < 1e-12


@pytest.mark.parametrize("name", list(VARIANTS))
def test_solve_matches_oracle(name):
    p = toy(**VARIANTS[name])
    ref = O.solve(*args(p), tol=1e-13, max_iter=3000)
    out = C.solve(*args(p), tol=1e-13, max_iter=3000, threads=4)
    assert out["status"] == 0
    assert np.array_equal(out["hits"], ref.hits)
    assert rel(out["baselines"], ref.baselines) < 1e-9
    obs = ref.hits > 0
    assert rel(out["destriped_map"][obs], ref.destriped_map[obs]) < 1e-9
    ref10 = O.solve(*args(p), tol=1e-10, max_iter=3000)
    out10 = C.solve(*args(p), tol=1e-10, max_iter=3000, threads=2)
    assert abs(out10["iterations"] - ref10.iterations) <= 1


def test_split_graph_canonical_per_part():
    from test_gpu_components import split_problem
    p = split_problem("TQU")
    ref = O.solve(*args(p), tol=1e-13, max_iter=3000)
    out = C.solve(*args(p), tol=1e-13, max_iter=3000)
    assert rel(out["baselines"], ref.baselines) < 1e-9
