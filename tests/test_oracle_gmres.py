"""Pins of the oracle's GMRES against references outside it.

* Generic operators: a diagonal operator with three distinct eigenvalues is
  solved exactly in three steps; a random nonsymmetric system matches
  numpy.linalg.solve (full and restarted); within a cycle the residual never
  grows (GMRES minimises it); the exit estimate equals the true residual.
* Destriping: GMRES and PCG reach the dense solution of Eq. 13 on a toy.
"""
import numpy as np
import pytest

from oracle import dense as D
from oracle import destripe as O
from problems import args, tiny, toy


def test_three_distinct_eigenvalues_three_steps():
    d = np.repeat([1.0, 3.0, 7.5], [10, 7, 5])
    b = np.random.default_rng(0).standard_normal(d.size)
    x, it, conv, rel, hist = O.gmres_core(lambda v: d * v, b, np.ones_like(d), 1e-13, 50, 100)
    assert conv and it == 3
    assert np.allclose(x, b / d, rtol=0, atol=1e-12 * np.abs(b / d).max())


@pytest.mark.parametrize("restart", [40, 7])
def test_random_nonsymmetric(restart):
    rng = np.random.default_rng(1)
    A = np.eye(40) * 4.0 + rng.standard_normal((40, 40)) * 0.3
    b = rng.standard_normal(40)
    Mdiag = 1.0 / np.diag(A)
    x, it, conv, rel, hist = O.gmres_core(lambda v: A @ v, b, Mdiag, 1e-13, restart, 2000)
    ref = np.linalg.solve(A, b)
    assert conv
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)
    if restart == 40:
        assert all(h1 <= h0 * (1 + 1e-12) for h0, h1 in zip(hist, hist[1:]))
    true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert abs(true - rel) <= 1e-10


@pytest.mark.parametrize("make", [tiny, toy])
def test_gmres_destriping_matches_dense_and_pcg(make):
    p = make()
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    b = O.rhs(st, O._full(st.pt, p.tod))
    g = O.gmres(st, b, 1e-13, 2000, restart=30)
    c = O.pcg(st, b, 1e-13, 2000)
    assert g.converged and g.true_rel_residual < 1e-11
    ga, ca = O.canonicalise(st, g.a), O.canonicalise(st, c.a)
    assert np.linalg.norm(ga - ca) <= 1e-9 * np.linalg.norm(ca)
    K, bb = D.eliminated(p.pix, p.psi, p.tod, p.n_pix, p.baseline_length, p.streams, p.weights)[:2]
    x = np.linalg.lstsq(K, bb, rcond=None)[0]
    ref = O.canonicalise(st, O._full(st.pt, x.reshape(len(O.ROWS[p.streams]), -1)))
    assert np.linalg.norm(ga - ref) <= 1e-8 * np.linalg.norm(ref)


def test_gmres_solve_entry_point():
    p = toy()
    a = O.solve(*args(p), tol=1e-13, solver="gmres", restart=20)
    c = O.solve(*args(p), tol=1e-13)
    assert a.converged
    assert np.linalg.norm(a.baselines - c.baselines) <= 1e-9 * np.linalg.norm(c.baselines)
