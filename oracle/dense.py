"""Dense direct references for the destriping solution (small problems only).

TEST INFRASTRUCTURE ONLY (see ``oracle.destripe``).  These routes build the
matrices explicitly from per-sample entries and share no code with the
iterative oracle, so they pin it independently.

* ``joint_lstsq``: the plain definition.  Destriping is the maximum-likelihood
  fit of the model of Eq. 8 (Algorithm section): minimise over the sky map m
  and the baselines a the weighted squared residual
  ``sum_t sum_k v_k(t) w_k (d_k(t) - A_k(t) m_p(t) - a_k[t // L])^2``.
  Solved with ``numpy.linalg.lstsq`` on the explicit design matrix ``[A | F]``.
* ``eliminated``: the destriping equation (Eq. 13) with the operator formed
  explicitly, ``K = F^T W F - G^T M^+ G`` with ``G = A^T W F`` and ``M^+`` the
  pseudo-inverse of each pixel's 3x3 block, solved by a minimum-norm
  least-squares solve.

The per-pixel validity rule (hits > 0 for T; eigenvalue ratio of the QU block
>= rcond_cut for Q/U) is applied here with its own code.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_ROWS = {"TQU": (0, 1, 2), "QU": (1, 2), "T": (0,), "IQU": (0,)}


def _entries(pix, psi, n_pix, streams, weights, rcond_cut):
    """Explicit per-(sample, stream) pointing entries and their validity.

    Returns a dict with flat arrays over (sample, stream) pairs:
    ``t``, ``k`` (stream), ``row`` (position of k in the stream list),
    ``p`` (pixel), ``A`` [n][3] (row of the pointing matrix), ``w``, ``ok``.
    """
    pix = np.asarray(pix).astype(np.int64)
    n_t = pix.size
    present = _ROWS[streams]
    ts, ks, rs, As = [], [], [], []
    for row, k in enumerate(present):
        A = np.zeros((n_t, 3))
        if streams == "IQU":  # radiometer row (1, cos 2psi, sin 2psi)
            ang = 2.0 * np.asarray(psi, dtype=np.float64)
            A[:, 0], A[:, 1], A[:, 2] = 1.0, np.cos(ang), np.sin(ang)
        elif k == 0:
            A[:, 0] = 1.0
        else:
            ang = 2.0 * np.asarray(psi, dtype=np.float64)
            if k == 1:
                A[:, 1], A[:, 2] = np.cos(ang), np.sin(ang)
            else:
                A[:, 1], A[:, 2] = -np.sin(ang), np.cos(ang)
        ts.append(np.arange(n_t))
        ks.append(np.full(n_t, k))
        rs.append(np.full(n_t, row))
        As.append(A)
    t = np.concatenate(ts)
    k = np.concatenate(ks)
    row = np.concatenate(rs)
    A = np.concatenate(As)
    p = pix[t]
    w = np.asarray(weights, dtype=np.float64)[k]
    good = p >= 0
    # per-pixel 3x3 normal matrices, summed entry by entry
    M = np.zeros((n_pix, 3, 3))
    for i in range(3):
        for j in range(3):
            np.add.at(M[:, i, j], p[good], (w * A[:, i] * A[:, j])[good])
    hits = np.bincount(pix[pix >= 0], minlength=n_pix)
    okT = hits > 0
    okQU = np.zeros(n_pix, dtype=bool)
    if 1 in present:
        obs = np.nonzero(hits > 0)[0]
        for q in obs:
            ev = np.linalg.eigvalsh(M[q, 1:, 1:])
            okQU[q] = ev[0] > 0 and ev[0] / ev[1] >= rcond_cut
    if streams == "IQU":
        okT = np.zeros(n_pix, dtype=bool)
        for q in np.nonzero(hits > 0)[0]:
            ev = np.linalg.eigvalsh(M[q])
            okT[q] = ev[0] > 0 and ev[0] / ev[2] >= rcond_cut
        okQU = okT.copy()
    pp = np.where(good, p, 0)
    ok = good & np.where(k == 0, okT[pp], okQU[pp])
    return dict(t=t, k=k, row=row, p=p, A=A, w=w, ok=ok, present=present, M=M, okT=okT, okQU=okQU)


def baseline_weights(pix, psi, n_pix, L, streams, weights, rcond_cut=1e-3):
    """Diagonal of ``F^T W F`` over valid entries, [n_streams][n_b]: ``w_k`` times the number of valid
    samples of stream k in each baseline, summed entry by entry from the explicit pointing entries."""
    e = _entries(pix, psi, n_pix, streams, weights, rcond_cut)
    n_t = np.asarray(pix).size
    n_b = -(-n_t // L)
    ns = len(e["present"])
    sel = np.nonzero(e["ok"])[0]
    out = np.zeros(ns * n_b)
    np.add.at(out, e["row"][sel] * n_b + e["t"][sel] // L, e["w"][sel])
    return out.reshape(ns, n_b)


def joint_lstsq(pix, psi, tod, n_pix, L, streams, weights, rcond_cut=1e-3):
    """Minimum-norm joint weighted LS over (m, a), tiny problems only.

    Returns ``(m [n_pix][3], a [n_streams][n_b])`` -- raw, not canonicalised.
    Unknowns: map components ``3 p + i``, then baselines
    ``3 n_pix + row * n_b + beta``.
    """
    e = _entries(pix, psi, n_pix, streams, weights, rcond_cut)
    n_t = np.asarray(pix).size
    n_b = -(-n_t // L)
    ns = len(e["present"])
    tod = np.asarray(tod, dtype=np.float64)
    sel = np.nonzero(e["ok"])[0]
    n_eq = sel.size
    sw = np.sqrt(e["w"][sel])
    D = np.zeros((n_eq, 3 * n_pix + ns * n_b))
    eq = np.arange(n_eq)
    for i in range(3):
        D[eq, 3 * e["p"][sel] + i] += sw * e["A"][sel, i]
    D[eq, 3 * n_pix + e["row"][sel] * n_b + e["t"][sel] // L] += sw
    y = sw * tod[e["row"][sel], e["t"][sel]]
    x = np.linalg.lstsq(D, y, rcond=1e-12)[0]
    return x[: 3 * n_pix].reshape(n_pix, 3), x[3 * n_pix:].reshape(ns, n_b)


def eliminated(pix, psi, tod, n_pix, L, streams, weights, rcond_cut=1e-3):
    """Explicit ``K`` and ``b`` of Eq. 13 and their minimum-norm solution.

    Returns ``(K [nu][nu], b [nu], a [n_streams][n_b])`` with
    ``nu = n_streams * n_b``; feasible for ``nu`` up to a few thousand.
    """
    e = _entries(pix, psi, n_pix, streams, weights, rcond_cut)
    n_t = np.asarray(pix).size
    n_b = -(-n_t // L)
    ns = len(e["present"])
    tod = np.asarray(tod, dtype=np.float64)
    sel = np.nonzero(e["ok"])[0]
    w = e["w"][sel]
    p = e["p"][sel]
    A = e["A"][sel]
    col = e["row"][sel] * n_b + e["t"][sel] // L
    dv = tod[e["row"][sel], e["t"][sel]]
    nu = ns * n_b
    # G = A^T W F as a sparse (3 n_pix x nu) matrix, duplicates summed
    G = sp.coo_matrix((np.concatenate([w * A[:, i] for i in range(3)]),
                       (np.concatenate([3 * p + i for i in range(3)]), np.tile(col, 3))),
                      shape=(3 * n_pix, nu)).tocsr()
    Ddiag = np.bincount(col, weights=w, minlength=nu)
    f_d = np.bincount(col, weights=w * dv, minlength=nu)
    s_d = np.zeros(3 * n_pix)
    for i in range(3):
        np.add.at(s_d, 3 * p + i, w * A[:, i] * dv)
    # per-pixel 3x3 normal matrix of the valid entries, then its pseudo-inverse
    Mv = np.zeros((n_pix, 3, 3))
    for i in range(3):
        for j in range(3):
            np.add.at(Mv[:, i, j], p, w * A[:, i] * A[:, j])
    obs = np.unique(p)
    Mp = np.zeros_like(Mv)
    for q in obs:
        Mp[q] = np.linalg.pinv(Mv[q], rcond=1e-12, hermitian=True)
    Minv = sp.block_diag([Mp[q] for q in range(n_pix)], format="csr") if n_pix <= 4096 else None
    if Minv is None:
        blocks_r, blocks_c, blocks_v = [], [], []
        for i in range(3):
            for j in range(3):
                blocks_r.append(3 * obs + i)
                blocks_c.append(3 * obs + j)
                blocks_v.append(Mp[obs, i, j])
        Minv = sp.coo_matrix((np.concatenate(blocks_v), (np.concatenate(blocks_r), np.concatenate(blocks_c))),
                             shape=(3 * n_pix, 3 * n_pix)).tocsr()
    GtMG = (G.T @ (Minv @ G)).toarray()
    K = np.diag(Ddiag) - GtMG
    b = f_d - G.T @ (Minv @ s_d)
    a = np.linalg.lstsq(K, b, rcond=1e-13)[0]
    return K, b, a.reshape(ns, n_b)
