"""Oracle parity on the code paths the benchmark runs, element by element.

* One day of the 30-day workload (N_side 256, L 3000): 313,004 observed
  pixels, so the run keys pack 19 bits of compact pixel with 12 of length,
  as in the headline solve.
* One day of an N_side 512 polarimeter channel (L 1500) of the uneven survey
  batch: 22 bits of pixel leave 10 for the length, so runs are split at 1024
  samples; FP64 inputs, and FP32 inputs as the batch runs them.
* One day of an N_side 512 intensity-only stream (L 6000): 16-byte run
  records, split runs.
* A 32-realization batch (32 right-hand sides) on a 6-hour N_side 256 slice.
* The 30-day workload at full size, in the benchmark's launch configuration:
  hits in full, and the maps and the operator at sampled pixels and
  baselines, each computed by the oracle from the samples it depends on.

Bars (FP64, CG tolerance 1e-13 on both sides; the oracle is FP64 NumPy):
per stream and per I/Q/U component, ||d||/||ref|| <= 1e-9 and
max|d| / RMS(ref) <= 1e-8 for baselines and destriped maps, binned maps
<= 1e-12, hits bit-exact.  One operator application differs from the
oracle only by summation order (a few ulp per term, <= 1e-12 relative at
these sizes); the solve amplifies that by the condition number PCG sees,
which the 1e-9 norm bar covers at tolerance 1e-13; the maximum of the
elementwise error stays within ten times the norm bar because the errors
spread over all baselines.  FP32 inputs: the arithmetic-only error statement
of the mixed-precision form (RMS error <= 1e-4 sigma / sqrt(L) per stream and
<= 1e-4 of the white-noise map RMS per component, against the oracle on the
same FP32 values promoted to FP64).
"""
import numpy as np
import pytest

from oracle import destripe as O
from synth import ScanSpec, make_problem, pointing, workload

pytestmark = pytest.mark.gpu

DAY = 4_320_000
SIGMA = 1e-3


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def maxrel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.max(np.abs(a - b)) / max(np.sqrt(np.mean(b * b)), 1e-300)


def rms(x):
    return float(np.sqrt(np.mean(np.square(x))))


def args(p):
    return p.pix, p.psi, p.tod, p.n_pix, p.baseline_length, p.streams, p.weights


@pytest.fixture(scope="module")
def ctx():
    from paper_1309_5609_amd import dst
    c = dst.Context(0)
    yield c
    c.close()


def host(out):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


def check_tight(p, out, ref, label):
    """Element-wise bars per stream and per map component (FP64 inputs)."""
    assert out["converged"] == 1, label
    assert np.array_equal(out["hits"], ref.hits), label
    for k in range(ref.baselines.shape[0]):
        a, r = out["baselines"][k], ref.baselines[k]
        assert rel(a, r) <= 1e-9, (label, "baselines", k, rel(a, r))
        assert maxrel(a, r) <= 1e-8, (label, "baselines max", k, maxrel(a, r))
    comps = (0,) if p.streams == "T" else ((1, 2) if p.streams == "QU" else (0, 1, 2))
    for c in comps:
        ok = ref.valid_T if c == 0 else ref.valid_QU
        m, r = out["destriped_map"][ok, c], ref.destriped_map[ok, c]
        assert rel(m, r) <= 1e-9, (label, "map", c, rel(m, r))
        assert maxrel(m, r) <= 1e-8, (label, "map max", c, maxrel(m, r))
        mb, rb = out["binned_map"][ok, c], ref.binned_map[ok, c]
        assert rel(mb, rb) <= 1e-12, (label, "binned", c, rel(mb, rb))
    assert out["true_rel_residual"] < 1e-11, label


def check_arithmetic(p, out, ref, label):
    """Mixed precision: GPU on FP32 inputs vs the oracle on the same values in FP64."""
    assert np.array_equal(out["hits"], ref.hits), label
    L = p.baseline_length
    for k in range(ref.baselines.shape[0]):
        e = rms(out["baselines"][k] - ref.baselines[k]) / (SIGMA / np.sqrt(L))
        assert e <= 1e-4, (label, "baselines", k, e)
    obs = ref.hits > 0
    noise = rms(SIGMA / np.sqrt(ref.hits[obs]))
    comps = (0,) if p.streams == "T" else (0, 1, 2)
    for c in comps:
        e = rms(out["destriped_map"][obs, c] - ref.destriped_map[obs, c]) / noise
        assert e <= 1e-4, (label, "map", c, e)


def rounded32(p):
    """The problem with FP32-rounded timelines and angles, promoted back to FP64."""
    q = p.astype(np.float32, np.float32)
    q.tod = q.tod.astype(np.float64)
    if q.psi is not None:
        q.psi = q.psi.astype(np.float64)
    return q


# ------------------------------------------------------------- one day, N_side 256

@pytest.fixture(scope="module")
def day256():
    p = workload(1, n_samples=DAY)
    ref = O.solve(*args(p), tol=1e-13, max_iter=3000)
    return p, ref


def test_day_nside256_fp64(ctx, day256):
    from paper_1309_5609_amd import dst
    p, ref = day256
    assert int((ref.hits > 0).sum()) == 313_004  # 19 bits of compact pixel + 12 of length per run key
    out = host(dst.dst_solve(ctx, dst.to_device(p), tol=1e-13, max_iter=3000))
    check_tight(p, out, ref, "day256")
    # the benchmark's tolerance: the same number of CG steps as the oracle
    ref10 = O.solve(*args(p), tol=1e-10, max_iter=3000)
    out10 = dst.dst_solve(ctx, dst.to_device(p), tol=1e-10, max_iter=3000)
    assert abs(out10["iterations"] - ref10.iterations) <= 1


# ------------------------------------------------------------- one day, N_side 512

def channel5_scan():
    # channel 5 of the uneven survey batch: az0 = 45 deg x 5, psi0 = 22.5 deg x 5
    return ScanSpec(az0_deg=225.0, psi0_deg=112.5)


@pytest.fixture(scope="module")
def day512():
    p = make_problem(nside=512, n_samples=DAY, baseline_length=1500, streams="TQU", cfg=4, channel=5,
                     fknee_hz=0.1, alpha=1.8, scan=channel5_scan())
    q = rounded32(p)
    ref = O.solve(*args(q), tol=1e-13, max_iter=3000)
    return q, ref


def test_day_nside512_channel_split_runs(ctx, day512):
    from paper_1309_5609_amd import dst
    q, ref = day512
    out = host(dst.dst_solve(ctx, dst.to_device(q), tol=1e-13, max_iter=3000))
    check_tight(q, out, ref, "day512 fp64")
    # FP32 inputs (the same values), FP32 run sums, FP64 accumulation and CG: as the survey batch runs it
    out32 = host(dst.dst_solve(ctx, dst.to_device(q, tod_dtype=np.float32, psi_dtype=np.float32), tol=1e-12,
                               max_iter=3000, flags=dst.DST_SOLVE_AUTOTUNE))
    check_arithmetic(q, out32, ref, "day512 fp32")


@pytest.fixture(scope="module")
def day512_t():
    p = make_problem(nside=512, n_samples=DAY, baseline_length=6000, streams="T", cfg=4, channel=8,
                     fknee_hz=0.05, alpha=1.7, scan=ScanSpec(az0_deg=360.0))
    q = rounded32(p)
    ref = O.solve(*args(q), tol=1e-13, max_iter=3000)
    return q, ref


def test_day_nside512_intensity_stream(ctx, day512_t):
    from paper_1309_5609_amd import dst
    q, ref = day512_t
    out = host(dst.dst_solve(ctx, dst.to_device(q), tol=1e-13, max_iter=3000))
    check_tight(q, out, ref, "T512 fp64")
    out32 = host(dst.dst_solve(ctx, dst.to_device(q, tod_dtype=np.float32), tol=1e-12, max_iter=3000,
                               flags=dst.DST_SOLVE_AUTOTUNE))
    check_arithmetic(q, out32, ref, "T512 fp32")


# ------------------------------------------------------------- 32 right-hand sides

@pytest.fixture(scope="module")
def batch32():
    n = 1_080_000
    base = workload(1, n_samples=n)
    probs = [base] + [make_problem(nside=256, n_samples=n, baseline_length=3000, cfg=1, realization=r,
                                   fknee_hz=0.05, alpha=1.7, pointing_arrays=(base.pix, base.psi), sky=base.sky)
                      for r in range(1, 32)]
    return probs


def test_batch_of_32(ctx, batch32):
    from paper_1309_5609_amd import dst
    probs = batch32
    d0 = dst.to_device(probs[0])
    dps = [d0] + [dst.Problem(d0.pix, d0.psi, dst.to_device(p).tod, d0.n_pix, d0.baseline_length, "TQU",
                              d0.weights) for p in probs[1:]]
    rc, res = dst.dst_solve_batched(ctx, dps, tol=1e-13, max_iter=3000)
    assert rc == 0
    res = [host(r) for r in res]
    for r in (0, 9, 22, 31):  # sampled realizations against the oracle
        ref = O.solve(*args(probs[r]), tol=1e-13, max_iter=3000)
        check_tight(probs[r], res[r], ref, f"batch r={r}")
    for r in range(32):  # every realization against the library's single solve (checked above)
        one = host(dst.dst_solve(ctx, dps[r], tol=1e-13, max_iter=3000))
        assert rel(res[r]["baselines"], one["baselines"]) <= 1e-9, r
        assert rel(res[r]["destriped_map"], one["destriped_map"]) <= 1e-9, r
    # FP32 inputs, as the benchmark's batch runs: arithmetic-only error on two realizations
    d32 = dst.to_device(probs[0], tod_dtype=np.float32, psi_dtype=np.float32)
    dps32 = [d32] + [dst.Problem(d32.pix, d32.psi, dst.to_device(p, tod_dtype=np.float32).tod, d32.n_pix,
                                 d32.baseline_length, "TQU", d32.weights) for p in probs[1:]]
    _, res32 = dst.dst_solve_batched(ctx, dps32, tol=1e-12, max_iter=3000)
    for r in (0, 31):
        q = rounded32(probs[r])
        ref = O.solve(*args(q), tol=1e-12, max_iter=3000)
        check_arithmetic(q, host(res32[r]), ref, f"batch32 fp32 r={r}")


# ------------------------------------------------------------- the 30-day workload at full size

def sub_setup(p, idx):
    """The oracle's setup on the samples idx alone (their pixels' blocks and validity are complete when idx holds
    every sample of those pixels)."""
    psi = None if p.psi is None else p.psi[idx]
    return O.prepare(p.pix[idx], psi, p.n_pix, p.baseline_length, p.streams, p.weights)


def samples_of(p, pixels):
    sel = np.zeros(p.n_pix, dtype=bool)
    sel[pixels] = True
    good = p.pix >= 0
    return np.flatnonzero(good & sel[np.where(good, p.pix, 0)])


@pytest.mark.timeout(1200)
def test_workload1_full_size(ctx):
    from paper_1309_5609_amd import dst
    import torch
    p = workload(1)
    dp = dst.to_device(p)
    out = host(dst.dst_solve(ctx, dp, tol=1e-10, max_iter=2000))  # the benchmark's call
    hits = np.bincount(p.pix[p.pix >= 0], minlength=p.n_pix)
    assert np.array_equal(out["hits"], hits)
    rng = np.random.default_rng(1309)
    obs = np.flatnonzero(hits > 0)
    assert obs.size == 313_004
    # binned and destriped maps at 3000 sampled pixels from those pixels' samples alone
    S = np.sort(rng.choice(obs, 3000, replace=False))
    idx = samples_of(p, S)
    st = sub_setup(p, idx)
    L = p.baseline_length
    d = O._full(st.pt, p.tod[:, idx])
    mb = O.map_from(st, d)[S]
    a = out["baselines"]
    a3 = O._full(st.pt, a)
    md = O.map_from(st, d - a3[:, idx // L])[S]
    for c in range(3):
        ok = (st.valid_T if c == 0 else st.valid_QU)[S]
        assert rel(out["binned_map"][S][ok, c], mb[ok, c]) <= 1e-12, c
        assert maxrel(out["binned_map"][S][ok, c], mb[ok, c]) <= 1e-11, c
        assert rel(out["destriped_map"][S][ok, c], md[ok, c]) <= 1e-12, c
    # b and K a at 12 sampled baselines, from the samples of every pixel those baselines visit
    B = np.sort(rng.choice(p.n_baselines, 12, replace=False))
    inB = np.concatenate([np.arange(b * L, min((b + 1) * L, p.n_samples)) for b in B])
    P = np.unique(p.pix[inB][p.pix[inB] >= 0])
    idx = samples_of(p, P)
    st = sub_setup(p, idx)
    beta = idx // L
    onB = np.isin(beta, B)

    def f_t_z(x3):  # F^T Z x on the sampled baselines: W v (x - A m(x)) summed per baseline
        z = O.apply_Z(st, x3)
        return np.stack([np.bincount(beta[onB], weights=z[k][onB], minlength=p.n_baselines)[B] for k in range(3)])

    b_or = f_t_z(O._full(st.pt, p.tod[:, idx]))
    ka_or = f_t_z(a3[:, beta])
    a_d = torch.from_numpy(a).cuda()
    b_gpu = dst.dst_residual(ctx, dp).cpu().numpy()
    ka_gpu = dst.dst_apply_operator(ctx, dp, a_d).cpu().numpy()
    assert rel(b_gpu[:, B], b_or) <= 1e-12
    assert rel(ka_gpu[:, B], ka_or) <= 1e-12
    # the solution: ||P (b - K a)|| / ||P b|| at the tolerance (T null-space mean removed over T-valid baselines)
    r = b_gpu - ka_gpu
    bp = b_gpu.copy()
    tv = out["baselines"][0] != 0.0
    r[0, tv] -= r[0, tv].mean()
    bp[0, tv] -= bp[0, tv].mean()
    assert np.linalg.norm(r) / np.linalg.norm(bp) <= 1.5e-10
    assert out["true_rel_residual"] <= 1.5e-10
    # the operator is symmetric and annihilates the T offset at full size
    u, v = (torch.from_numpy(rng.standard_normal((3, p.n_baselines))).cuda() for _ in range(2))
    ku, kv = dst.dst_apply_operator(ctx, dp, u), dst.dst_apply_operator(ctx, dp, v)
    s1, s2 = float((u * kv).sum()), float((v * ku).sum())
    assert abs(s1 - s2) <= 1e-12 * float(torch.linalg.norm(u) * torch.linalg.norm(kv))
    e = torch.zeros((3, p.n_baselines), dtype=torch.float64, device="cuda")
    e[0] = 1.0
    assert float(torch.linalg.norm(dst.dst_apply_operator(ctx, dp, e))) <= 1e-12 * float(torch.linalg.norm(ku))
