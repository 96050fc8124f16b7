"""Plain FP64 CPU oracle of the polarimeter destriper's hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this package; only
the test suite, the smoke check and the benchmark's CPU-baseline leg may call
it.  It shares no code with the GPU path; the two meet only through the
seeded inputs of ``synth``.

What it computes (Algorithm section of the paper):

* Data model (Eqs. 2, 7, 8): ``d = A m + F a + w`` for the streams
  k in {T, q, u} of one channel, with pointing rows
  ``A_T = (1, 0, 0)``, ``A_q = (0, cos 2psi, sin 2psi)``,
  ``A_u = (0, -sin 2psi, cos 2psi)`` (Eqs. 3-6) acting on the pixel
  ``p(t)`` (one pixel per sample), and ``F`` repeating each baseline over its
  fixed run of ``L`` samples (Eq. 7 and the Polarimeters data section).
* Hit map ``h = P^T P`` (Eq. 9) and, per pixel, ``M_p = sum_t sum_k w_k
  A_k(t)^T A_k(t)``; for a polarimeter with equal weights the QU block is
  ``w h I_2`` (the remark after Eqs. 10-11).
* Map given baselines (Eqs. 10-12): ``m = M^-1 A^T W (d - F a)``.
* Destriping equation (Eq. 13): ``F^T Z F a = F^T Z d`` with
  ``Z = W - W A M^-1 A^T W`` restricted to valid samples, solved by
  preconditioned conjugate gradient (the solver paragraph closing the
  Algorithm section).

Readings of points the paper leaves open (each is listed with its reason in
the design notes):

* Eq. 12 writes ``B = h^-1 P~^T R``; with R's rows being channels, Eqs. 10-11
  need its transpose, so ``B = M^-1 (R P~)^T W`` is used.
* ``F^T`` sums over each baseline (not averages); averaging is a diagonal
  rescale absorbed by the Jacobi preconditioner.
* Constant white-noise weight ``w_k = 1/sigma_k^2`` per stream; equal weights
  reduce exactly to the paper's unweighted form.
* The T stream is solved in the same system; the per-pixel matrix is block
  diagonal (T | QU), so this equals destriping T separately.
* Streams "IQU": one polarisation-sensitive radiometer stream with row
  ``A = (1, cos 2psi, sin 2psi)`` (the remark after Eqs. 10-11 that such a
  detector needs the full 3x3 per-pixel inverse); its block is valid when
  ``lambda_min > 0`` and ``lambda_min / lambda_max >= rcond_cut`` over all
  three eigenvalues.  A constant offset on its baselines is again a null
  vector (it equals a constant I map), handled like the T stream's.
* A block is valid when T: ``h_p > 0``; QU: ``lambda_min > 0`` and
  ``lambda_min / lambda_max >= rcond_cut``.  Samples on invalid blocks are
  dropped from that stream (both from binning and from ``F^T``).
  ``pix < 0`` masks a sample in every stream.
* Baselines start at sample 0; the last one may be shorter than ``L``.
* PCG from ``a = 0`` with Jacobi preconditioner ``1 / (w_k n_valid)``;
  stop when the recurrence residual ``||r||_2 <= tol ||b||_2``.
* A constant offset on the T baselines of one connected component of the
  baseline-pixel graph is indistinguishable from a constant sky (Eq. 8), so
  K has that null vector.  The right-hand side is orthogonal to it only up
  to rounding; the solver removes from ``b`` and from every ``K p`` their
  mean over the component's baselines, which keeps CG on the consistent
  subspace (without it, a signal-only input, whose ``b`` is pure rounding,
  makes CG diverge along the null vector).
* The T baselines are defined up to one constant per connected component of
  the baseline-pixel graph; results are canonicalised to zero mean per
  component over baselines that hold valid samples.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

ROWS = {"TQU": (0, 1, 2), "QU": (1, 2), "T": (0,), "IQU": (0,)}


def n_baselines(n_t: int, L: int) -> int:
    """Number of baselines: ceil(n_t / L) (fixed length, last may be short)."""
    return -(-int(n_t) // int(L))


def baseline_index(n_t: int, L: int) -> np.ndarray:
    """Column of F holding the 1 of row t (Eq. 7): t // L."""
    return np.arange(n_t, dtype=np.int64) // int(L)


@dataclass
class Pointing:
    """The pointing part of a problem, pre-digested for the oracle.

    ``rows[k]`` is the pointing row of stream k as three float64 arrays over
    samples (Eqs. 3-6); absent streams have weight 0.
    """

    pix: np.ndarray  # int64 [n_t], -1 masked
    n_pix: int
    L: int
    streams: str
    w: np.ndarray  # float64 [3]; 0 for absent streams
    rows: list  # rows[k] = (a0, a1, a2) float64 arrays or None
    rcond_cut: float

    @property
    def n_t(self) -> int:
        return int(self.pix.shape[0])

    @property
    def n_b(self) -> int:
        return n_baselines(self.n_t, self.L)


def make_pointing(pix, psi, n_pix: int, L: int, streams: str, weights, rcond_cut: float = 1e-3) -> Pointing:
    """Pointing rows from the angle psi (Eqs. 3-6), in FP64."""
    pix = np.asarray(pix).astype(np.int64)
    n_t = pix.shape[0]
    present = ROWS[streams]
    w = np.zeros(3)
    for k in present:
        w[k] = float(weights[k])
    rows = [None, None, None]
    if streams == "IQU":
        # one polarisation-sensitive radiometer stream: A = (1, cos 2psi, sin 2psi)
        two = 2.0 * np.asarray(psi, dtype=np.float64)
        rows[0] = (np.ones(n_t), np.cos(two), np.sin(two))
        return Pointing(pix, int(n_pix), int(L), streams, w, rows, float(rcond_cut))
    if 0 in present:
        one = np.ones(n_t)
        zero = np.zeros(n_t)
        rows[0] = (one, zero, zero)
    if 1 in present:
        two = 2.0 * np.asarray(psi, dtype=np.float64)
        c, s = np.cos(two), np.sin(two)
        zero = np.zeros(n_t)
        rows[1] = (zero, c, s)
        rows[2] = (zero, -s, c)
    return Pointing(pix, int(n_pix), int(L), streams, w, rows, float(rcond_cut))


def hit_map(pt: Pointing) -> np.ndarray:
    """Eq. 9: number of (unmasked) samples per pixel, int64."""
    good = pt.pix >= 0
    return np.bincount(pt.pix[good], minlength=pt.n_pix).astype(np.int64)


def pixel_matrices(pt: Pointing) -> np.ndarray:
    """Per-pixel ``M_p = sum_t sum_k w_k A_k(t)^T A_k(t)``, float64 [n_pix][3][3]."""
    good = pt.pix >= 0
    p = pt.pix[good]
    M = np.zeros((pt.n_pix, 3, 3))
    for k in range(3):
        if pt.rows[k] is None:
            continue
        a = [r[good] for r in pt.rows[k]]
        for i in range(3):
            for j in range(3):
                M[:, i, j] += np.bincount(p, weights=pt.w[k] * a[i] * a[j], minlength=pt.n_pix)
    return M


def block_inverse(pt: Pointing, M: np.ndarray, hits: np.ndarray):
    """Inverse of the valid T and QU blocks and the per-pixel validity flags.

    Returns ``(Minv [n_pix][3][3], valid_T [n_pix] bool, valid_QU [n_pix] bool)``.
    Invalid blocks have a zero inverse.
    """
    n = pt.n_pix
    Minv = np.zeros((n, 3, 3))
    valid_T = np.zeros(n, dtype=bool)
    valid_QU = np.zeros(n, dtype=bool)
    if pt.streams == "IQU":
        # the full 3x3 block: valid when lambda_min > 0 and lambda_min / lambda_max >= rcond_cut
        lam = np.linalg.eigvalsh(M)
        lmin, lmax = lam[:, 0], lam[:, 2]
        with np.errstate(divide="ignore", invalid="ignore"):
            rc = np.where(lmax > 0, lmin / lmax, 0.0)
        valid = (hits > 0) & (lmin > 0) & (rc >= pt.rcond_cut)
        if np.any(valid):
            Minv[valid] = np.linalg.inv(M[valid])
        return Minv, valid, valid.copy()
    if pt.rows[0] is not None:
        valid_T = hits > 0
        Minv[valid_T, 0, 0] = 1.0 / M[valid_T, 0, 0]
    if pt.rows[1] is not None:
        qu = M[:, 1:, 1:]
        lam = np.linalg.eigvalsh(qu)  # ascending per pixel
        lmin, lmax = lam[:, 0], lam[:, 1]
        with np.errstate(divide="ignore", invalid="ignore"):
            rc = np.where(lmax > 0, lmin / lmax, 0.0)
        valid_QU = (hits > 0) & (lmin > 0) & (rc >= pt.rcond_cut)
        if np.any(valid_QU):
            Minv[valid_QU, 1:, 1:] = np.linalg.inv(qu[valid_QU])
    return Minv, valid_T, valid_QU


def sample_validity(pt: Pointing, valid_T, valid_QU) -> np.ndarray:
    """v[k][t] in {0, 1}: sample t enters stream k (unmasked, on a valid block)."""
    good = pt.pix >= 0
    pp = np.where(good, pt.pix, 0)
    v = np.zeros((3, pt.n_t))
    if pt.rows[0] is not None:
        v[0] = good & valid_T[pp]
    if pt.rows[1] is not None:
        vq = good & valid_QU[pp]
        v[1] = vq
        v[2] = vq
    return v


@dataclass
class Setup:
    pt: Pointing
    hits: np.ndarray
    M: np.ndarray
    Minv: np.ndarray
    valid_T: np.ndarray
    valid_QU: np.ndarray
    v: np.ndarray  # [3][n_t] sample validity
    n_valid: np.ndarray  # [3][n_b] valid samples per baseline and stream


def setup(pt: Pointing) -> Setup:
    hits = hit_map(pt)
    M = pixel_matrices(pt)
    Minv, vT, vQU = block_inverse(pt, M, hits)
    v = sample_validity(pt, vT, vQU)
    n_valid = baseline_sums(pt, v)
    return Setup(pt, hits, M, Minv, vT, vQU, v, n_valid)


def _full(pt: Pointing, x) -> np.ndarray:
    """Stream rows [n_streams][n] -> [3][n] with zero rows for absent streams."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((3,) + x.shape[1:])
    for row, k in enumerate(ROWS[pt.streams]):
        out[k] = x[row]
    return out


def _compact(pt: Pointing, x3: np.ndarray) -> np.ndarray:
    return np.stack([x3[k] for k in ROWS[pt.streams]])


def bin_sums(st: Setup, x3: np.ndarray) -> np.ndarray:
    """``s = A^T W x`` over valid samples (the sum maps of Eqs. 10-11), [n_pix][3]."""
    pt = st.pt
    good = pt.pix >= 0
    p = pt.pix[good]
    s = np.zeros((pt.n_pix, 3))
    for k in range(3):
        if pt.rows[k] is None:
            continue
        wx = (pt.w[k] * st.v[k] * x3[k])[good]
        for i in range(3):
            s[:, i] += np.bincount(p, weights=wx * pt.rows[k][i][good], minlength=pt.n_pix)
    return s


def apply_inverse(st: Setup, s: np.ndarray) -> np.ndarray:
    """``m = M^-1 s`` per pixel (valid blocks; zero elsewhere)."""
    return np.einsum("pij,pj->pi", st.Minv, s)


def scan(st: Setup, m: np.ndarray) -> np.ndarray:
    """``(A m)_k(t) = A_k(t) . m[p(t)]``, [3][n_t]; zero on masked samples."""
    pt = st.pt
    good = pt.pix >= 0
    pp = np.where(good, pt.pix, 0)
    mp = m[pp]
    y = np.zeros((3, pt.n_t))
    for k in range(3):
        if pt.rows[k] is None:
            continue
        y[k] = good * (pt.rows[k][0] * mp[:, 0] + pt.rows[k][1] * mp[:, 1] + pt.rows[k][2] * mp[:, 2])
    return y


def baseline_sums(pt: Pointing, y3: np.ndarray) -> np.ndarray:
    """``F^T y``: sum of each stream over each baseline's samples, [3][n_b]."""
    beta = baseline_index(pt.n_t, pt.L)
    return np.stack([np.bincount(beta, weights=y3[k], minlength=pt.n_b) for k in range(3)])


def expand(pt: Pointing, a3: np.ndarray) -> np.ndarray:
    """``F a``: baseline value repeated over its samples, [3][n_t]."""
    beta = baseline_index(pt.n_t, pt.L)
    return np.stack([a3[k][beta] for k in range(3)])


def map_from(st: Setup, x3: np.ndarray) -> np.ndarray:
    """Eqs. 10-12 with the weighted reading: ``m = M^-1 A^T W x``."""
    return apply_inverse(st, bin_sums(st, x3))


def apply_Z(st: Setup, x3: np.ndarray) -> np.ndarray:
    """``Z x = W (x - A m(x))`` on valid samples (the bracket of Eq. 13)."""
    m = map_from(st, x3)
    y = scan(st, m)
    return st.pt.w[:, None] * st.v * (x3 - y)


def apply_K(st: Setup, v3: np.ndarray) -> np.ndarray:
    """Left-hand operator of Eq. 13: ``F^T Z F v``, [3][n_b]."""
    return baseline_sums(st.pt, apply_Z(st, expand(st.pt, v3)))


def rhs(st: Setup, d3: np.ndarray) -> np.ndarray:
    """Right-hand side of Eq. 13: ``F^T Z d``, [3][n_b]."""
    return baseline_sums(st.pt, apply_Z(st, d3))


def jacobi(st: Setup) -> np.ndarray:
    """Preconditioner ``1 / (w_k n_valid_k(beta))``; 0 for empty baselines."""
    d = st.pt.w[:, None] * st.n_valid
    out = np.zeros_like(d)
    nz = d > 0
    out[nz] = 1.0 / d[nz]
    return out


@dataclass
class PCGResult:
    a: np.ndarray  # [3][n_b]
    iterations: int
    converged: bool
    rel_residual: float  # recurrence residual / ||b||
    true_rel_residual: float
    history: list


def pcg(st: Setup, b3: np.ndarray, tol: float, max_iter: int, a0=None) -> PCGResult:
    """Preconditioned conjugate gradient on ``K a = b`` (Eq. 13).

    Recurrences (Shewchuk's PCG): ``alpha = (r.z)/(p.Kp)``, ``a += alpha p``,
    ``r -= alpha Kp``, stop on ``||r|| <= tol ||b||``, ``z = J r``,
    ``beta = (r'.z')/(r.z)``, ``p = z + beta p``.
    """
    J = jacobi(st)
    proj = null_projector(st)
    b3 = proj(b3)
    a = np.zeros_like(b3) if a0 is None else np.array(a0, dtype=np.float64)
    bnorm = float(np.sqrt(np.sum(b3 * b3)))
    if bnorm == 0.0:
        return PCGResult(np.zeros_like(b3), 0, True, 0.0, 0.0, [])
    r = b3 - proj(apply_K(st, a)) if a0 is not None else b3.copy()
    z = J * r
    p = z.copy()
    rz = float(np.sum(r * z))
    it = 0
    hist = []
    rel = float(np.sqrt(np.sum(r * r))) / bnorm
    converged = rel <= tol
    while not converged and it < max_iter:
        q = proj(apply_K(st, p))
        pq = float(np.sum(p * q))
        if pq <= 0.0:
            break
        alpha = rz / pq
        a += alpha * p
        r -= alpha * q
        it += 1
        rel = float(np.sqrt(np.sum(r * r))) / bnorm
        hist.append(rel)
        if rel <= tol:
            converged = True
            break
        z = J * r
        rz_new = float(np.sum(r * z))
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    true = float(np.sqrt(np.sum((b3 - apply_K(st, a)) ** 2))) / bnorm
    return PCGResult(a, it, converged, rel, true, hist)


@dataclass
class GMRESResult:
    a: np.ndarray
    iterations: int
    converged: bool
    rel_residual: float  # the least-squares residual estimate at exit
    true_rel_residual: float
    history: list


def gmres_core(op, b, M, tol: float, restart: int, max_iter: int, x0=None):
    """Restarted GMRES(m) (Saad & Schultz 1986) for ``op(x) = b`` with right preconditioner ``diag(M)``.

    Each cycle: Arnoldi with modified Gram-Schmidt on ``op(M v)`` builds an
    orthonormal basis ``V`` and the Hessenberg matrix ``H``; Givens rotations
    triangularise ``H`` column by column, so ``|g[j+1]|`` is the residual norm of
    the minimiser of ``||beta e1 - H y||`` over the current Krylov space; after
    ``restart`` steps, convergence, or ``max_iter``, ``x += M (V y)`` and the
    next cycle starts from the new residual.  Returns
    ``(x, iterations, converged, estimate, history)`` with the estimate and
    history relative to ``||b||``.
    """
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    if bnorm == 0.0:
        return x, 0, True, 0.0, []
    r = b - op(x) if x0 is not None else b.copy()
    beta = float(np.linalg.norm(r))
    rel = beta / bnorm
    it, hist = 0, []
    while rel > tol and it < max_iter and beta > 0.0:
        m = int(restart)
        V = [r / beta]
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        for j in range(m):
            w = op(M * V[j])
            for i in range(j + 1):
                H[i, j] = float(np.sum(w * V[i]))
                w = w - H[i, j] * V[i]
            hn = float(np.linalg.norm(w))
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = float(np.hypot(H[j, j], H[j + 1, j]))
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j], H[j + 1, j] = den, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            rel = abs(g[j + 1]) / bnorm
            hist.append(rel)
            if rel <= tol or it >= max_iter or hn == 0.0:
                break
            V.append(w / hn)
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):  # back substitution on the triangularised H
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        x = x + M * sum(y[i] * V[i] for i in range(k))
        r = b - op(x)
        beta = float(np.linalg.norm(r))
    return x, it, rel <= tol, rel, hist


def gmres(st: Setup, b3: np.ndarray, tol: float, max_iter: int, restart: int = 50, a0=None) -> GMRESResult:
    """Eq. 13 by restarted GMRES with the Jacobi diagonal as right preconditioner.

    Works on the same projected operator as ``pcg`` (the T null vectors
    removed from ``b`` and from every ``K v``).
    """
    J = jacobi(st)
    proj = null_projector(st)
    b3 = proj(b3)
    bnorm = float(np.sqrt(np.sum(b3 * b3)))
    if bnorm == 0.0:
        return GMRESResult(np.zeros_like(b3), 0, True, 0.0, 0.0, [])
    a, it, conv, rel, hist = gmres_core(lambda x: proj(apply_K(st, x)), b3, J, tol, restart, max_iter, a0)
    true = float(np.sqrt(np.sum((b3 - apply_K(st, a)) ** 2))) / bnorm
    return GMRESResult(a, it, conv, rel, true, hist)


def null_projector(st: Setup):
    """Orthogonal projector removing the T null vectors (one per component)."""
    if st.pt.rows[0] is None:
        return lambda x3: x3
    n_comp, lab = t_components(st)
    has = lab >= 0
    cnt = np.bincount(lab[has], minlength=n_comp).astype(float)

    def proj(x3):
        y = np.array(x3, dtype=np.float64)
        if np.any(has):
            mean = np.bincount(lab[has], weights=y[0, has], minlength=n_comp)
            nz = cnt > 0
            mean[nz] /= cnt[nz]
            y[0, has] -= mean[lab[has]]
        return y

    return proj


def t_components(st: Setup) -> tuple[int, np.ndarray]:
    """Connected components of baselines linked through shared T-valid pixels.

    Returns ``(n_comp, label[n_b])``; baselines with no valid T sample get -1.
    """
    pt = st.pt
    n_b = pt.n_b
    if pt.rows[0] is None:
        return 0, -np.ones(n_b, dtype=np.int64)
    sel = st.v[0] > 0
    beta = baseline_index(pt.n_t, pt.L)[sel]
    pix = pt.pix[sel]
    # bipartite graph: nodes 0..n_b-1 are baselines, n_b.. are pixels
    g = sp.coo_matrix((np.ones(beta.size), (beta, n_b + pix)), shape=(n_b + pt.n_pix, n_b + pt.n_pix)).tocsr()
    n_comp, lab = connected_components(g, directed=False)
    lab_b = lab[:n_b].astype(np.int64)
    lab_b[st.n_valid[0] == 0] = -1
    return n_comp, lab_b


def canonicalise(st: Setup, a3: np.ndarray) -> np.ndarray:
    """Remove the T-stream null space: zero mean of a_T over each component."""
    a = np.array(a3, dtype=np.float64)
    if st.pt.rows[0] is None:
        return a
    _, lab = t_components(st)
    has = lab >= 0
    a[0, ~has] = 0.0
    if np.any(has):
        sums = np.bincount(lab[has], weights=a[0, has])
        cnt = np.bincount(lab[has])
        mean = np.zeros_like(sums)
        mean[cnt > 0] = sums[cnt > 0] / cnt[cnt > 0]
        a[0, has] -= mean[lab[has]]
    return a


@dataclass
class Solution:
    hits: np.ndarray  # int64 [n_pix]
    binned_map: np.ndarray  # [n_pix][3]
    destriped_map: np.ndarray  # [n_pix][3]
    baselines: np.ndarray  # [n_streams][n_b], canonical
    iterations: int
    converged: bool
    rel_residual: float
    true_rel_residual: float
    valid_T: np.ndarray
    valid_QU: np.ndarray
    raw_baselines: np.ndarray  # [n_streams][n_b], as returned by PCG


def solve(pix, psi, tod, n_pix: int, L: int, streams: str, weights, tol: float = 1e-10,
          max_iter: int = 1000, rcond_cut: float = 1e-3, solver: str = "pcg", restart: int = 50) -> Solution:
    """Full destriping of one channel: hits, binned map, baselines, destriped map.

    ``solver``: "pcg" (default) or "gmres" (restarted every ``restart`` steps).
    """
    pt = make_pointing(pix, psi, n_pix, L, streams, weights, rcond_cut)
    st = setup(pt)
    d3 = _full(pt, tod)
    b = rhs(st, d3)
    res = pcg(st, b, tol, max_iter) if solver == "pcg" else gmres(st, b, tol, max_iter, restart)
    a = canonicalise(st, res.a)
    binned = map_from(st, d3)
    destriped = map_from(st, d3 - expand(pt, a))
    return Solution(st.hits, binned, destriped, _compact(pt, a), res.iterations, res.converged,
                    res.rel_residual, res.true_rel_residual, st.valid_T, st.valid_QU, _compact(pt, res.a))


# Convenience wrappers on stream-compact arrays ([n_streams][...]) -------------

def prepare(pix, psi, n_pix, L, streams, weights, rcond_cut=1e-3) -> Setup:
    return setup(make_pointing(pix, psi, n_pix, L, streams, weights, rcond_cut))


def K_compact(st: Setup, v) -> np.ndarray:
    return _compact(st.pt, apply_K(st, _full(st.pt, v)))


def rhs_compact(st: Setup, tod) -> np.ndarray:
    return _compact(st.pt, rhs(st, _full(st.pt, tod)))


def bin_compact(st: Setup, tod, baselines=None) -> np.ndarray:
    """Sum maps ``A^T W (d - F a)`` over valid samples, [n_pix][3]."""
    x = _full(st.pt, tod)
    if baselines is not None:
        x = x - expand(st.pt, _full(st.pt, baselines))
    return bin_sums(st, x)


def map_compact(st: Setup, tod, baselines=None) -> np.ndarray:
    return apply_inverse(st, bin_compact(st, tod, baselines))


def scan_compact(st: Setup, m) -> np.ndarray:
    return _compact(st.pt, scan(st, m))


def reduce_compact(st: Setup, tod) -> np.ndarray:
    """``F^T W x`` over valid samples: ``sum_{t in beta} v_k(t) w_k x_k(t)``."""
    x = _full(st.pt, tod)
    return _compact(st.pt, baseline_sums(st.pt, st.pt.w[:, None] * st.v * x))


def canonical_compact(st: Setup, a) -> np.ndarray:
    return _compact(st.pt, canonicalise(st, _full(st.pt, a)))
