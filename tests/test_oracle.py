"""Pins of the FP64 oracle against things other than itself.

* hand-solved cases (tests/golden/hand_cases.json, each citing its equation);
* brute-force loops over samples on tiny inputs;
* closed forms stated by the paper (QU block = w h I for a polarimeter);
* the explicit dense operator and the joint least-squares definition;
* invariants (symmetry, positive semi-definiteness, the T null vector);
* physics checks (pure offsets recovered, null baselines on signal only,
  white-noise chi^2 of the destriped map);
* planted mistakes: a mutated oracle must fail the pins.
"""
import json
import os

import numpy as np
import pytest

from oracle import dense as D
from oracle import destripe as O
from problems import args, tiny, toy

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# --------------------------------------------------------------------------- golden

def test_golden_hand_cases():
    cases = json.load(open(GOLDEN))["cases"]
    for c in cases:
        pix = np.array(c["pix"])
        psi = None if c["psi"] is None else np.array(c["psi"])
        tod = np.array(c["tod"])
        st = O.prepare(pix, psi, c["n_pix"], c["baseline_length"], c["streams"], c["weights"])
        assert np.array_equal(st.hits, c["hits"])
        assert np.allclose(O.map_compact(st, tod), c["binned_map"], atol=1e-14)
        if "baselines" in c:
            sol = O.solve(pix, psi, tod, c["n_pix"], c["baseline_length"], c["streams"], c["weights"], tol=1e-15)
            assert np.allclose(sol.baselines, c["baselines"], atol=1e-13)
            assert np.allclose(sol.destriped_map, c["destriped_map"], atol=1e-13)
        if "components" in c:
            _, lab = O.t_components(st)
            groups = sorted(sorted(np.nonzero(lab == g)[0].tolist()) for g in np.unique(lab[lab >= 0]))
            assert groups == sorted(c["components"])


def test_two_islands_need_one_mean_each():
    """A single mean over all valid baselines (instead of one per island) fails the two-island hand case."""
    c = [x for x in json.load(open(GOLDEN))["cases"] if x["name"] == "T_two_islands_and_an_empty_baseline"][0]
    st = O.prepare(np.array(c["pix"]), None, c["n_pix"], c["baseline_length"], "T", c["weights"])
    a = np.array(c["baselines"], dtype=float)
    shifted = a.copy()
    shifted[0, :2] += 1.0
    shifted[0, 2:4] -= 1.0  # global mean unchanged, island means moved
    assert np.allclose(O.canonical_compact(st, shifted), a, atol=1e-14)
    # the same null vectors for K: adding the shift changes no residual
    tod = np.array(c["tod"])
    assert np.allclose(O.K_compact(st, shifted - a), 0.0, atol=1e-12)
    assert np.allclose(O.rhs_compact(st, tod) - O.K_compact(st, a), 0.0, atol=1e-12)


# --------------------------------------------------------------------------- setup pins

@pytest.mark.parametrize("kw", [dict(), dict(mask_fraction=0.08), dict(streams="T"), dict(streams="QU"),
                                dict(weights=(2.0e6, 5.0e6, 0.7e6)), dict(streams="IQU", n_samples=20000, L=400)])
def test_jacobi_is_inverse_diagonal_of_FtWF(kw):
    """The preconditioner is 1 / diag(F^T W F) over valid samples (0 for empty baselines), checked against the
    explicit entries of the dense route and against a loop over samples."""
    p = toy(**kw)
    st = O.prepare(*[args(p)[i] for i in (0, 1, 3, 4, 5, 6)])
    J = O._compact(st.pt, O.jacobi(st))
    d = D.baseline_weights(*[args(p)[i] for i in (0, 1, 3, 4, 5, 6)])
    want = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
    assert np.allclose(J, want, rtol=1e-15, atol=0)
    # loop: every valid (sample, stream) adds w_k to its baseline
    rows = O.ROWS[p.streams]
    brute = np.zeros_like(d)
    for t in range(p.n_samples):
        q = p.pix[t]
        if q < 0:
            continue
        for r, k in enumerate(rows):
            ok = st.valid_T[q] if (k == 0 or p.streams == "IQU") else st.valid_QU[q]
            if ok:
                brute[r, t // p.baseline_length] += p.weights[k]
    assert np.array_equal(brute, d)
    assert np.any(d == 0) == bool(np.any(J == 0))

def test_hits_brute_force():
    p = toy(mask_fraction=0.05)
    st = O.prepare(*[args(p)[i] for i in (0, 1, 3, 4, 5, 6)])
    h = np.zeros(p.n_pix, dtype=np.int64)
    for q in p.pix:
        if q >= 0:
            h[q] += 1
    assert np.array_equal(st.hits, h)
    assert st.hits.sum() == np.count_nonzero(p.pix >= 0)


def test_blocks_closed_form_equal_weights():
    """Polarimeter with equal q/u weights: QU block = w h I_2, T block = w h."""
    p = toy(weights=(3.0, 2.0, 2.0))
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    h = st.hits.astype(float)
    assert np.allclose(st.M[:, 0, 0], 3.0 * h, rtol=0, atol=1e-12)
    assert np.allclose(st.M[:, 1, 1], 2.0 * h, rtol=1e-14, atol=1e-12)
    assert np.allclose(st.M[:, 2, 2], 2.0 * h, rtol=1e-14, atol=1e-12)
    assert np.allclose(st.M[:, 1, 2], 0.0, atol=1e-11)
    assert np.allclose(st.M[:, 0, 1:], 0.0, atol=0)


def test_blocks_brute_force_unequal_weights():
    p = tiny(weights=(1.0, 4.0, 0.5))
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    M = np.zeros((p.n_pix, 3, 3))
    for t in range(p.n_samples):
        c, s = np.cos(2 * p.psi[t]), np.sin(2 * p.psi[t])
        for w, row in zip(p.weights, ([1, 0, 0], [0, c, s], [0, -s, c])):
            row = np.array(row)
            M[p.pix[t]] += w * np.outer(row, row)
    assert np.allclose(st.M, M, rtol=1e-13, atol=1e-12)
    # block inverse against numpy's 3x3 inverse of the brute-force matrix
    obs = st.hits > 0
    assert np.allclose(st.Minv[obs], np.linalg.inv(M[obs]), rtol=1e-12, atol=1e-14)


def test_binned_map_is_pixel_average():
    """a = 0: the I map is the per-pixel mean of d_T (Eqs. 10-11 with h^-1)."""
    p = toy()
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    m = O.map_compact(st, p.tod)
    acc = np.zeros(p.n_pix)
    cnt = np.zeros(p.n_pix)
    for t in range(p.n_samples):
        acc[p.pix[t]] += p.tod[0, t]
        cnt[p.pix[t]] += 1
    obs = cnt > 0
    assert np.allclose(m[obs, 0], acc[obs] / cnt[obs], rtol=1e-12, atol=1e-18)
    assert np.all(m[~obs] == 0)


def test_signal_only_map_equals_sky():
    p = toy(noise=False)
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    m = O.map_compact(st, p.tod)
    obs = st.hits > 0
    assert rel(m[obs], p.sky[obs]) < 1e-13


# --------------------------------------------------------------------------- operator pins

@pytest.mark.parametrize("variant", ["plain", "masked", "ragged", "unequal", "QU", "T", "IQU"])
def test_operator_matches_dense(variant):
    kw = {}
    if variant == "masked":
        kw["mask_fraction"] = 0.1
    if variant == "ragged":
        kw["n_samples"] = 1457
    if variant == "unequal":
        kw["weights"] = (2.0, 5.0, 0.7)
    if variant in ("QU", "T", "IQU"):
        kw["streams"] = variant
    p = tiny(**kw)
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    K, b, a = D.eliminated(*args(p))
    rng = np.random.default_rng(3)
    v = rng.standard_normal((len(O.ROWS[p.streams]), p.n_baselines))
    Kv = O.K_compact(st, v)
    assert rel(Kv.ravel(), K @ v.ravel()) < 1e-12
    assert rel(O.rhs_compact(st, p.tod).ravel(), b) < 1e-12


def test_operator_invariants():
    p = toy(mask_fraction=0.02, weights=(1.0, 2.0, 0.5))
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    rng = np.random.default_rng(11)
    u = rng.standard_normal((3, p.n_baselines))
    v = rng.standard_normal((3, p.n_baselines))
    Ku, Kv = O.K_compact(st, u), O.K_compact(st, v)
    # symmetric and positive semi-definite
    assert abs(np.sum(u * Kv) - np.sum(v * Ku)) <= 1e-12 * np.linalg.norm(Ku) * np.linalg.norm(v)
    assert np.sum(v * Kv) >= -1e-12 * np.linalg.norm(Kv) * np.linalg.norm(v)
    # constant T offset is invisible to the destriper; the RHS is orthogonal to it
    one = np.zeros((3, p.n_baselines))
    one[0] = 1.0
    assert np.linalg.norm(O.K_compact(st, one)) <= 1e-10 * np.linalg.norm(Kv)
    b = O.rhs_compact(st, p.tod)
    assert abs(np.sum(b[0])) <= 1e-10 * np.linalg.norm(b)
    # Z W^-1 is a projector: applying the signal removal twice changes nothing
    x = O._full(st.pt, p.tod)
    z1 = O.apply_Z(st, x) / np.where(st.pt.w[:, None] > 0, st.pt.w[:, None], 1)
    z2 = O.apply_Z(st, z1) / np.where(st.pt.w[:, None] > 0, st.pt.w[:, None], 1)
    assert rel(z2, z1) < 1e-12


def test_dense_K_psd_and_null_space():
    p = tiny()
    K, b, a = D.eliminated(*args(p))
    ev = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert ev[0] > -1e-10 * ev[-1]
    assert np.sum(np.abs(ev) < 1e-9 * ev[-1]) == 1  # one T component -> one null vector


# --------------------------------------------------------------------------- solve pins

@pytest.mark.parametrize("variant", ["plain", "masked", "ragged", "unequal", "QU", "T", "IQU"])
def test_solve_matches_dense_and_joint(variant):
    kw = {}
    if variant == "masked":
        kw["mask_fraction"] = 0.1
    if variant == "ragged":
        kw["n_samples"] = 1457
    if variant == "unequal":
        kw["weights"] = (2.0, 5.0, 0.7)
    if variant in ("QU", "T", "IQU"):
        kw["streams"] = variant
    p = tiny(**kw)
    sol = O.solve(*args(p), tol=1e-14, max_iter=2000)
    assert sol.converged
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    _, _, a_el = D.eliminated(*args(p))
    assert rel(sol.baselines, O.canonical_compact(st, a_el)) < 1e-9
    m_j, a_j = D.joint_lstsq(*args(p))
    a_jc = O.canonical_compact(st, a_j)
    assert rel(sol.baselines, a_jc) < 1e-9
    # the destriped map is the joint fit's map once both use canonical baselines
    m_jc = O.map_compact(st, p.tod, a_jc)
    obs = st.hits > 0
    assert rel(sol.destriped_map[obs], m_jc[obs]) < 1e-9


def test_solve_config0_matches_dense():
    """Full-size 6 h workload: PCG against the explicitly formed 1080 x 1080 system."""
    from synth import workload
    p = workload(0)
    sol = O.solve(*args(p), tol=1e-13, max_iter=2000)
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    K, b, a_el = D.eliminated(*args(p))
    assert K.shape == (1080, 1080)
    assert rel(sol.baselines, O.canonical_compact(st, a_el)) < 1e-9


def test_pure_offsets_recovered():
    """d = A m_sky + F a_true: q/u baselines recovered exactly, T up to a constant."""
    p = toy(noise=False, offsets_rms=1e-3)
    sol = O.solve(*args(p), tol=1e-14, max_iter=2000)
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    a_true = O.canonical_compact(st, p.offsets)
    assert rel(sol.baselines, a_true) < 1e-9
    obs = st.hits > 0
    # destriped map = sky + the T constant removed by canonicalisation
    shift = np.mean(p.offsets[0]) - 0.0
    assert np.allclose(sol.destriped_map[obs, 1:], p.sky[obs, 1:], atol=1e-12)
    assert np.allclose(sol.destriped_map[obs, 0] - p.sky[obs, 0], shift, atol=1e-12)


def test_signal_only_null_baselines():
    """Signal generated from a map: baselines vanish to rounding (simulation section)."""
    p = toy(noise=False)
    sol = O.solve(*args(p), tol=1e-10, max_iter=2000)
    rms = np.sqrt(np.mean(p.tod ** 2))
    assert np.max(np.abs(sol.baselines)) <= 1e-12 * rms
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    obs = st.hits > 0
    assert rel(sol.destriped_map[obs], p.sky[obs]) < 1e-12


def test_white_noise_chi2():
    """White noise only: the destriped residual map stays at the white-noise level.

    Statistical check (the simulation section's reduced chi^2 near 1): per-pixel
    variance sigma^2 / h for I and for Q, U (each sample's (q, u) pair is a
    rotation of two independent measurements).  Fitting the baselines adds a
    little noise, so the bound is loose; the binned map must sit at 1 within
    its sampling error.
    """
    sigma = 1e-3
    p = toy(n_samples=200000, nside=16, fknee_hz=0.0, sigma=sigma, L=1500, cfg=301)
    sol = O.solve(*args(p), tol=1e-12, max_iter=2000)
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    obs = st.hits > 20
    n = int(obs.sum())
    var = sigma ** 2 / st.hits[obs]
    for m, bound in ((sol.binned_map, 5 * np.sqrt(2.0 / n)), (sol.destriped_map, 0.15)):
        res = m[obs] - p.sky[obs]
        # the T map absorbs one constant (canonicalisation); remove the weighted mean
        res[:, 0] -= np.sum(res[:, 0] / var) / np.sum(1 / var)
        for comp in range(3):
            chi2 = np.mean(res[:, comp] ** 2 / var)
            assert abs(chi2 - 1) < bound, (comp, chi2)


# --------------------------------------------------------------------------- planted mistakes

def _mutated_K_error(monkeypatch, mutate):
    p = tiny(weights=(2.0, 5.0, 0.7))
    K, b, _ = D.eliminated(*args(p))
    with monkeypatch.context() as mp:
        mutate(mp)
        st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
        v = np.random.default_rng(3).standard_normal((3, p.n_baselines))
        return rel(O.K_compact(st, v).ravel(), K @ v.ravel())


def test_planted_sign_error_in_u_row_is_caught(monkeypatch):
    orig = O.make_pointing

    def bad(*a, **k):
        pt = orig(*a, **k)
        z, ms, c = pt.rows[2]
        pt.rows[2] = (z, -ms, c)  # +sin instead of -sin in A_u
        return pt

    assert _mutated_K_error(monkeypatch, lambda mp: mp.setattr(O, "make_pointing", bad)) > 1e-3


def test_planted_missing_weight_is_caught(monkeypatch):
    orig = O.apply_Z

    def bad(st, x3):
        m = O.map_from(st, x3)
        return st.v * (x3 - O.scan(st, m))  # dropped W

    assert _mutated_K_error(monkeypatch, lambda mp: mp.setattr(O, "apply_Z", bad)) > 1e-3


def test_planted_transposed_binning_is_caught(monkeypatch):
    """Eq. 12 taken literally (R instead of R^T) must not pass."""
    orig = O.make_pointing

    def bad(*a, **k):
        pt = orig(*a, **k)
        zq, c, s = pt.rows[1]
        zu, ms, c2 = pt.rows[2]
        pt.rows[1] = (zq, c, ms)
        pt.rows[2] = (zu, s, c2)
        return pt

    assert _mutated_K_error(monkeypatch, lambda mp: mp.setattr(O, "make_pointing", bad)) > 1e-3


# --------------------------------------------------------------------------- radiometer rows

def test_iqu_block_cut_bites():
    """A pixel seen at only two angles has a rank-2 3x3 block: it is cut and its samples leave the stream."""
    pix = np.array([0, 0, 0, 0, 1, 1, 1, 1, 1, 1])
    psi = np.array([0.0, 0.3, 0.0, 0.3, 0.0, 0.4, 0.9, 1.3, 0.2, 0.7])
    st = O.prepare(pix, psi, 2, 5, "IQU", (4.0, 0.0, 0.0))
    assert not st.valid_T[0] and st.valid_T[1]
    assert np.array_equal(st.v[0], [0, 0, 0, 0, 1, 1, 1, 1, 1, 1])
    # brute-force block of pixel 1 and its eigenvalue ratio
    M = np.zeros((3, 3))
    for t in range(4, 10):
        a = np.array([1.0, np.cos(2 * psi[t]), np.sin(2 * psi[t])])
        M += 4.0 * np.outer(a, a)
    assert np.allclose(st.M[1], M, rtol=0, atol=1e-13)
    assert np.allclose(st.Minv[1] @ M, np.eye(3), atol=1e-12)
    lam = np.linalg.eigvalsh(st.M[0])
    assert lam[0] <= 1e-12 * lam[-1]
    # a cut that rejects pixel 1 as well
    lam1 = np.linalg.eigvalsh(M)
    st2 = O.prepare(pix, psi, 2, 5, "IQU", (4.0, 0.0, 0.0), rcond_cut=1.01 * lam1[0] / lam1[-1])
    assert not st2.valid_T.any()


def test_iqu_signal_only_map_and_null_baselines():
    p = toy(streams="IQU", noise=False, n_samples=20000, L=400)
    st = O.prepare(p.pix, p.psi, p.n_pix, p.baseline_length, p.streams, p.weights)
    m = O.map_compact(st, p.tod)
    ok = st.valid_T
    assert ok.sum() > 20 and (~ok & (st.hits > 0)).sum() > 20  # the cut keeps some pixels and drops others
    assert rel(m[ok], p.sky[ok]) < 1e-12
    sol = O.solve(*args(p), tol=1e-12)
    assert np.max(np.abs(sol.baselines)) <= 1e-12 * np.sqrt(np.mean(p.tod ** 2))
