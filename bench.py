#!/usr/bin/env python3
"""Destriping throughput on one MI355X: samples x CG-iterations per second.

One step is one complete destriping solve of the workload through the C ABI
(``dst_solve``): pointing setup (runs, hits, per-pixel blocks and their
inverse, baseline counts, connected parts), right-hand side, preconditioned
CG to the tolerance, and the binned and destriped maps.  ``value`` is
n_samples x CG iterations summed over the timed steps divided by their wall
time, with the inputs already in HBM.  Kernel durations come from HIP events
the library records on its stream during a second, profiled pass.

Workloads (seeded synthetic inputs, see ``synth``):
  1 (default, the headline): 30 days at 50 Hz = 129,600,000 samples, HEALPix
     N_side 256, 3000-sample baselines (43,200 per stream), T/q/u, white 1 mK
     + 1/f noise (f_k = 50 mHz, alpha = 1.7), FP64, CG to 1e-10.
  0: 6 h = 1,080,000 samples at N_side 64, same scan and noise, FP64.
  2: workload 1 with FP32 timelines and angles (FP64 accumulation and CG).

With workload 1 the line also carries the other benchmark configurations
(6-hour workload; the 30-day workload at f_k 20 and 200 mHz; FP32 mixed
precision with its error statement; the 32-realization Monte Carlo batch;
the uneven survey batch), GMRES against PCG, the per-sample form, measured
copy / read ceilings, and two CPU baselines: the NumPy oracle on one thread
(``cpu_baseline``) and an all-core C++/OpenMP destriper (``cpu_parallel``).

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "samples x CG-iters/s per GPU (FP64 plain vs FP32-mixed batched); HBM GB/s % of peak"
HBM_PEAK_GBS = 8000.0
SIGMA = 1e-3
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "runs_30day_nside256_hbm_traffic.md")
RUN_KERNELS_SRC = os.path.join(ROOT, "paper_1309_5609_amd", "csrc", "dst_runs.hip")

# Uneven survey batch: 8 polarimeter channels (days, baseline length, f_k in Hz,
# alpha) with spin-axis phase az0 = 45 deg x c and angle offset psi0 = 22.5 deg x c,
# plus a 12-month intensity-only stream; N_side 512, FP32 timelines and angles.
UNEVEN_CHANNELS = [(3, 1500, 0.010, 1.0), (5, 2000, 0.020, 1.2), (7, 3000, 0.030, 1.4), (10, 4000, 0.050, 1.5),
                   (14, 6000, 0.075, 1.7), (20, 1500, 0.100, 1.8), (25, 3000, 0.150, 1.9), (30, 4500, 0.200, 2.0)]
UNEVEN_T_STREAM = (365, 6000, 0.050, 1.7)


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def measured_traffic(kernel: str):
    """HBM bytes per dispatch of ``kernel`` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary.

    None when the summary is missing, has no row for the kernel, or was taken
    on a different kernel source than the one built now.
    """
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        sha = hashlib.sha256(open(RUN_KERNELS_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    if f"sha256 {sha}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith(f"| `{kernel}` |"):
            return float(line.split("|")[5])
    return None


def scalars(out: dict) -> dict:
    """A solve's info without its output tensors (K solves in a row do not hold K sets of maps)."""
    return {k: v for k, v in out.items() if not hasattr(v, "data_ptr")}


def workload_name(w: int, fk: float) -> str:
    if w == 0:
        return (f"6-hour single-channel destripe: 1,080,000 samples at 50 Hz, HEALPix N_side 64, "
                f"3000-sample baselines, T/q/u, f_k {fk * 1e3:g} mHz, alpha 1.7, FP64")
    prec = "FP64" if w == 1 else "FP32 timelines and angles, FP64 accumulation and CG"
    return (f"30-day single-channel destripe: 129,600,000 samples at 50 Hz, HEALPix N_side 256, "
            f"3000-sample baselines (43,200 per stream), T/q/u, f_k {fk * 1e3:g} mHz, alpha 1.7, {prec}")


def key_bits(n: int) -> int:
    bits = 1
    while bits < 32 and (1 << bits) < n:
        bits += 1
    return bits


def model_bytes(n_t: int, n_obs: int, n_b: int, s_psi: int, n_streams: int = 3) -> dict:
    """Algorithmic bytes of one CG iteration in the per-sample form of the method (the per-sample byte model).

    bin:   per sample the pixel (4 B) and angle (s_psi); per observed pixel the
           block inverse read (4 x 8 B; 8 B intensity only) and the map written
           (3 x 8 B; 8 B intensity only); per baseline p read (8 B per stream);
    unbin: per sample the pixel and angle again; per observed pixel the map read
           (3 x 8 B); per baseline p read and q written (2 x 8 B per stream).
    The timelines are not read in the iterations.
    """
    inv_b, map_b = (8, 8) if n_streams == 1 else (32, 24)  # intensity only: one inverse entry, one map value
    bin_b = n_t * (4 + s_psi) + n_obs * (inv_b + map_b) + n_b * 8 * n_streams
    unbin_b = n_t * (4 + s_psi) + n_obs * map_b + n_b * 16 * n_streams
    return {"bin": bin_b, "unbin": unbin_b, "iteration": bin_b + unbin_b + 7 * 8 * n_streams * n_b}


def run_form_bytes(n_runs: int, n_obs: int, n_b: int, s_psi: int, L: int) -> dict:
    """Bytes the run-compressed kernels must move: per run a 32-bit key (index and length packed) and the
    pair of angle sums (2 x s_psi), with the same per-pixel and per-baseline terms as the model."""
    rec = 4 + 2 * s_psi
    return {"bin": n_runs * rec + n_obs * (32 + 24) + n_b * 24, "unbin": n_runs * rec + n_obs * 24 + n_b * 48,
            "record_bytes": rec}


def ceilings() -> dict:
    """Measured copy and read bandwidth of plain torch kernels on 2 GiB (the practical HBM ceilings)."""
    import torch
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst_ = torch.empty_like(src)
    for _ in range(2):
        dst_.copy_(src)
        src.sum()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst_.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy = 2 * 8 * n * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    e0.record()
    for _ in range(5):
        src.sum()
    e1.record()
    torch.cuda.synchronize()
    read = 8 * n * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst_
    torch.cuda.empty_cache()
    return {"copy_GBs": copy, "read_GBs": read, "note": "torch copy_ (read + write counted) and sum of 2 GiB FP64"}


def timed_solves(ctx, dp, tol, steps, warmup, **kw):
    import torch

    from paper_1309_5609_amd import dst
    for _ in range(warmup):
        dst.dst_solve(ctx, dp, tol=tol, max_iter=3000, maps=False, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [scalars(dst.dst_solve(ctx, dp, tol=tol, max_iter=3000, maps=False, **kw)) for _ in range(steps)]
    torch.cuda.synchronize()
    return res, time.perf_counter() - t0


def gpu_noise_problem(ctx, dp, sky_d, seed, fknee, alpha=1.7, tod_dtype=None):
    """The workload's sky scanned through dp's pointing plus GPU-drawn white + 1/f noise (FP64 timelines)."""
    from paper_1309_5609_amd import dst
    head = dst.Problem(dp.pix, dp.psi, None, dp.n_pix, dp.baseline_length, dp.streams, dp.weights)
    tod = dst.dst_unbin(ctx, head, sky_d)
    for k in range(tod.shape[0]):
        dst.dst_noise_generate(ctx, seed, k, dp.n_samples, 1 << 24, 50.0, SIGMA, fknee, alpha, out=tod[k],
                               accumulate=True)
    if tod_dtype is not None:
        tod = tod.to(tod_dtype)
    return tod


def error_statement(dp, out, ref, L):
    """RMS error of baselines (per stream, in sigma / sqrt(L)) and destriped maps (per component, in units of
    the white-noise map RMS sigma / sqrt(h))."""
    import numpy as np
    a, ra = out["baselines"].double().cpu().numpy(), ref["baselines"].cpu().numpy()
    base = [float(np.sqrt(np.mean((a[k] - ra[k]) ** 2)) / (SIGMA / np.sqrt(L))) for k in range(a.shape[0])]
    hits = ref["hits"].cpu().numpy()
    obs = hits > 0
    noise = float(np.sqrt(np.mean(SIGMA ** 2 / hits[obs])))
    m, rm = out["destriped_map"].cpu().numpy()[obs], ref["destriped_map"].cpu().numpy()[obs]
    maps = [float(np.sqrt(np.mean((m[:, c] - rm[:, c]) ** 2)) / noise) for c in range(3)]
    return base, maps


def cpu_baseline(p, seconds_target: float = 15.0) -> dict:
    """The NumPy oracle's operator on the first day of the workload, FP64 on one host thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import destripe as O

    n = min(p.n_samples, 4_320_000)
    sl = slice(0, n)
    psi = None if p.psi is None else np.asarray(p.psi[sl], dtype=np.float64)
    with threadpool_limits(limits=1):
        st = O.prepare(p.pix[sl], psi, p.n_pix, p.baseline_length, p.streams, p.weights)
        v = np.random.default_rng(0).standard_normal((3, st.pt.n_b))
        iters = 0
        t0 = time.perf_counter()
        while True:
            O.apply_K(st, v)
            iters += 1
            el = time.perf_counter() - t0
            if el > seconds_target or iters >= 400:
                break
    return {"value": n * iters / el, "unit": "samples*CG-iters/s", "cores": 1, "kind": "oracle",
            "sample": (f"first {n:,} samples (1 day) of the same workload; {iters} applications of the oracle's "
                       f"K = F^T Z F (one CG iteration each), NumPy FP64 on one thread, after its setup; "
                       f"{el:.1f} s")}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_parallel(p, iters_gpu: dict, uneven: dict | None) -> dict:
    """The all-core C++/OpenMP FP64 destriper: the full 30-day solve, and per-iteration rates for the batched and
    uneven configurations (extrapolated, labelled)."""
    import numpy as np

    from oracle import cpu_baseline as C
    from synth import ScanSpec, make_problem
    out = C.solve(p.pix, p.psi, p.tod, p.n_pix, p.baseline_length, p.streams, p.weights, tol=1e-10, max_iter=3000,
                  maps=True)
    it = max(out["iterations"], 1)
    res = {"kind": "C++17 + OpenMP FP64 destriper (oracle/cpu_baseline.cpp), thread-private maps",
           "nproc": os.cpu_count(), "threads": out["threads"], "cpu_model": cpu_model(),
           "workload_1": {"iterations": out["iterations"], "setup_s": out["setup_s"], "loop_s": out["loop_s"],
                          "total_s": out["total_s"], "iter_ms": out["loop_s"] / it * 1e3,
                          "value": p.n_samples * out["iterations"] / out["total_s"],
                          "loop_value": p.n_samples * out["iterations"] / out["loop_s"],
                          "unit": "samples*CG-iters/s"}}
    # batched Monte Carlo form: 32 independent solves of the same size, extrapolated from the one measured
    n_real = iters_gpu.get("n_realizations", 32)
    res["batched_extrapolated"] = {"value": p.n_samples * out["iterations"] / out["total_s"],
                                   "unit": "realizations*samples*CG-iters/s",
                                   "note": (f"{n_real} realizations solved one after another on the host: the same "
                                            "rate as one 30-day solve (measured), extrapolated linearly")}
    if uneven:
        # per-sample-iteration rates of one day at N_side 512 (polarimeter and intensity-only), times the
        # batch's samples and the GPU's iteration counts
        rates = {}
        for streams, L in (("TQU", 1500), ("T", 6000)):
            q = make_problem(nside=512, n_samples=4_320_000, baseline_length=L, streams=streams, cfg=4,
                             fknee_hz=0.05, alpha=1.7, scan=ScanSpec(az0_deg=45.0))
            v = np.random.default_rng(1).standard_normal((q.tod.shape[0], q.n_baselines))
            _, sec, setup, _ = C.apply_K(q.pix, q.psi, q.n_pix, q.baseline_length, q.streams, q.weights, v, reps=3)
            rates[streams] = (q.n_samples / sec, q.n_samples / setup)
        t_total = 0.0
        for d in uneven["problems"]:
            it_rate, setup_rate = rates["T" if d["streams"] == "T" else "TQU"]
            t_total += d["n_samples"] * d["iterations"] / it_rate + d["n_samples"] / setup_rate
        work = sum(d["n_samples"] * d["iterations"] for d in uneven["problems"])
        res["uneven_extrapolated"] = {"value": work / t_total, "unit": "samples*CG-iters/s", "seconds": t_total,
                                      "note": ("measured per-sample rates of the operator and the setup on one day "
                                               "at N_side 512 (T/q/u L 1500; T-only L 6000), extrapolated to the "
                                               "batch's samples and the GPU's iteration counts")}
    return res


def noise_form(ctx, n: int, segment: int = 1 << 24, reps: int = 3) -> dict:
    """dst_noise_generate on the workload's three FP64 timelines (white 1 mK + 1/f, f_k 50 mHz, alpha 1.7)."""
    import torch

    from paper_1309_5609_amd import dst
    out = torch.empty((3, n), dtype=torch.float64, device="cuda")
    for k in range(3):
        dst.dst_noise_generate(ctx, 1, k, n, segment, 50.0, SIGMA, 0.05, 1.7, out=out[k])
    torch.cuda.synchronize()
    t = time.perf_counter()
    for r in range(reps):
        for k in range(3):
            dst.dst_noise_generate(ctx, 2 + r, k, n, segment, 50.0, SIGMA, 0.05, 1.7, out=out[k])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    m = segment.bit_length() - 1
    passes = -(-m // 8)
    # per complex value (two samples): white write 16 B; each FFT pass reads and
    # writes 16 B, forward and inverse; the unpack reads 16 B and writes 2 x 8 B
    per_sample = (16 + 2 * passes * 32 + 16 + 16) / 2
    gbs = 3 * n * per_sample / dt / 1e9
    del out
    torch.cuda.empty_cache()
    return {"value": 3 * n / dt, "unit": "samples/s", "ms": dt * 1e3, "n_samples": 3 * n, "segment": segment,
            "fft_passes_per_transform": passes, "model_bytes_per_sample": per_sample, "achieved_GBs": gbs,
            "frac": gbs / HBM_PEAK_GBS,
            "method": "Philox4x64-10 + Box-Muller white noise, filtered per segment pair by one complex FFT: "
                      f"{passes} Stockham passes of radix <= 256 each way, computed in LDS; gain applied as the "
                      "inverse transform reads the spectrum"}


def batched_form(ctx, p, dp, n_real: int, tol: float, steps: int, warmup: int, plain_value: float) -> dict:
    """Monte Carlo batch: n_real realizations sharing dp's pointing, FP32 timelines, one batched solve."""
    import numpy as np
    import torch

    from paper_1309_5609_amd import dst

    t = time.perf_counter()
    sky_d = torch.from_numpy(p.sky).to("cuda")
    tods, tod0 = [], None
    for r in range(n_real):
        x = gpu_noise_problem(ctx, dp, sky_d, 1309_5609_000 + r, 0.05)
        if r == 0:
            tod0 = x  # the unrounded FP64 timelines of realization 0: the equal-accuracy reference
            tods.append(x.float())
        else:
            tods.append(x.float())
            del x
    torch.cuda.synchronize()
    log(f"batched form: {n_real} realizations drawn on the GPU in {time.perf_counter() - t:.1f} s")
    psi32 = dp.psi.float()
    probs = [dst.Problem(dp.pix, psi32, x, dp.n_pix, dp.baseline_length, dp.streams, dp.weights) for x in tods]
    for _ in range(max(warmup, 1)):
        dst.dst_solve_batched(ctx, probs, tol=tol, max_iter=3000, maps=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    its = 0
    for _ in range(steps):
        _, res = dst.dst_solve_batched(ctx, probs, tol=tol, max_iter=3000)
        its += sum(r["iterations"] for r in res)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = p.n_samples * its / wall
    _, prof = dst.dst_solve_batched(ctx, probs, tol=tol, max_iter=3000, flags=dst.DST_SOLVE_PROFILE, maps=False)
    ref = dst.dst_solve(ctx, dst.Problem(dp.pix, dp.psi, tod0, dp.n_pix, dp.baseline_length, dp.streams,
                                         dp.weights), tol=tol, max_iter=3000)
    obs = ref["hits"].cpu().numpy() > 0
    m64 = ref["destriped_map"].cpu().numpy()[obs]
    m32 = res[0]["destriped_map"].cpu().numpy()[obs]
    sky = p.sky[obs]
    ratio = [float(np.sqrt(np.mean((m32[:, c] - sky[:, c]) ** 2)) / np.sqrt(np.mean((m64[:, c] - sky[:, c]) ** 2)))
             for c in range(3)]
    it_ms = res[0]["t_iter_ms"]
    n_obs = int(res[0]["n_valid_pix"][0])
    b_iter = 2 * p.n_samples * (4 + 4) + n_real * (n_obs * 80 + 7 * 8 * 3 * p.n_baselines)
    out = {"value": value, "unit": "realizations*samples*CG-iters/s", "n_realizations": n_real,
           "ms_per_solve": wall * 1e3 / steps, "setup_ms": res[0]["t_setup_ms"], "iter_ms": it_ms,
           "iterations": [r["iterations"] for r in res],
           "kernel_ms": {k: prof[0][f"t_{k}_ms"] for k in ("bin", "unbin", "update")},
           "model_bytes_per_iteration": b_iter, "iteration_hbm_frac": b_iter / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "vs_plain_fp64": value / plain_value,
           "map_rms_error_ratio_vs_fp64": ratio,
           "true_rel_residual_max": max(float(r["true_rel_residual"]) for r in res),
           "equal_accuracy_reference": "realization 0's unrounded FP64 timelines solved by the plain FP64 path",
           "dtype": "f32 timelines and angles; f32 copies of p and m for the iterations' gathers; f64 sums, "
                    "inverse, CG and outputs",
           "inputs": ("sky signal of the 30-day workload scanned by dst_unbin + per-realization white 1 mK and 1/f "
                      "noise (f_k 50 mHz, alpha 1.7) drawn by dst_noise_generate (Eq. 1, seeds 1309_5609_000 + r)")}
    del probs, tods, tod0, res, prof, ref, sky_d
    torch.cuda.empty_cache()
    log(f"batched form: {value:.3e} realizations*samples*iters/s ({out['vs_plain_fp64']:.2f}x plain FP64)")
    return out


def uneven_form(ctx, tol: float, steps: int, warmup: int) -> dict:
    """The uneven survey batch, generated on the GPU by the library (pointing expansion, sky scan, noise) and solved
    by dst_solve_batched: the problems share no pointing and advance together, one launch per CG phase."""
    import torch

    from paper_1309_5609_amd import dst
    from synth import ScanSpec, gaussian_sky

    nside, rate = 512, 50.0
    n_pix = 12 * nside * nside
    t = time.perf_counter()
    sky = torch.from_numpy(gaussian_sky(n_pix, 4)).to("cuda")
    w = 1.0 / (SIGMA * SIGMA)
    probs, desc = [], []
    specs = [(c, days, L, fk, al, "TQU") for c, (days, L, fk, al) in enumerate(UNEVEN_CHANNELS)]
    specs.append((len(UNEVEN_CHANNELS),) + UNEVEN_T_STREAM + ("T",))
    for c, days, L, fk, al, streams in specs:
        n = int(days * 86400 * rate)
        scan = ScanSpec(sample_rate_hz=rate, az0_deg=45.0 * c, psi0_deg=22.5 * c)
        pix, psi = dst.dst_pointing_expand(ctx, scan, nside, n, psi_dtype=torch.float32)
        head = dst.Problem(pix, psi if streams != "T" else None, None, n_pix, L, streams, (w, w, w))
        tod = dst.dst_unbin(ctx, head, sky).float()
        for k in range(tod.shape[0]):
            dst.dst_noise_generate(ctx, 4000 + c, k, n, 1 << 22, rate, SIGMA, fk, al, out=tod[k], accumulate=True)
        probs.append(dst.Problem(pix, psi if streams != "T" else None, tod, n_pix, L, streams, (w, w, w)))
        desc.append({"days": days, "n_samples": n, "baseline_length": L, "fknee_hz": fk, "alpha": al,
                     "streams": streams, "az0_deg": 45.0 * c, "psi0_deg": 22.5 * c if streams != "T" else None})
        if streams == "T":
            del psi
    torch.cuda.synchronize()
    log(f"uneven batch: {len(probs)} problems, {sum(d['n_samples'] for d in desc):,} samples drawn on the GPU "
        f"in {time.perf_counter() - t:.1f} s")
    for _ in range(max(warmup, 1)):
        dst.dst_solve_batched(ctx, probs, tol=tol, max_iter=3000, maps=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    work = 0
    for _ in range(steps):
        _, res = dst.dst_solve_batched(ctx, probs, tol=tol, max_iter=3000, maps=False)
        work += sum(d["n_samples"] * r["iterations"] for d, r in zip(desc, res))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for d, r in zip(desc, res):
        d.update(iterations=r["iterations"], converged=r["converged"], n_runs=r["n_runs"],
                 observed_pixels=int(max(r["n_valid_pix"])))
    # every problem active: the iterations before the first problem stops
    k_all = min(d["iterations"] for d in desc)
    _, act = dst.dst_solve_batched(ctx, probs, tol=tol, max_iter=k_all, maps=False)
    _, prof = dst.dst_solve_batched(ctx, probs, tol=tol, max_iter=k_all, maps=False, flags=dst.DST_SOLVE_PROFILE)
    model = 0
    for d in desc:
        s_psi = 0 if d["streams"] == "T" else 4
        ns = 1 if d["streams"] == "T" else 3
        n_b = -(-d["n_samples"] // d["baseline_length"])
        model += model_bytes(d["n_samples"], d["observed_pixels"], n_b, s_psi, ns)["iteration"]
    all_ms = act[0]["t_iter_ms"]
    out = {"value": work / wall, "unit": "samples*CG-iters/s", "ms_per_step": wall * 1e3 / steps,
           "setup_ms": res[0]["t_setup_ms"], "iter_ms": res[0]["t_iter_ms"],
           "all_active": {"iterations": k_all, "iter_ms": all_ms, "model_bytes_per_iteration": model,
                          "hbm_frac": model / (all_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "phase_ms": {k: prof[0][f"t_{k}_ms"] for k in ("bin", "unbin", "update")}},
           "n_problems": len(probs), "total_samples": sum(d["n_samples"] for d in desc), "nside": nside,
           "dtype": "f32 timelines and angles, f64 accumulation / inverse / CG", "problems": desc,
           "solver": ("one group: per problem its own setup and CG state; every iteration one binning and one "
                      "rescan launch per stream set present and one launch per CG vector step, over all problems, "
                      "replayed from one captured graph; each problem stops on its own"),
           "inputs": ("pointing expanded on the GPU (dst_pointing_expand), Gaussian sky (I 1 mK, Q/U 0.1 mK) scanned "
                      "by dst_unbin, white 1 mK + 1/f noise by dst_noise_generate (segments of 2^22 samples)")}
    del probs, res, sky, act, prof
    torch.cuda.empty_cache()
    log(f"uneven batch: {out['value']:.3e} samples*iters/s, {out['ms_per_step']:.0f} ms per batch, "
        f"all-active iteration {all_ms:.2f} ms")
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=1, choices=(0, 1, 2))
    ap.add_argument("--fknee", type=float, default=0.05)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--realizations", type=int, default=32, help="batch size of the Monte Carlo form (0: skip)")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven survey batch (N_side 512)")
    ap.add_argument("--no-extra", action="store_true", help="only the headline solve and its roofline")
    ap.add_argument("--no-single-extras", action="store_true",
                    help="skip the single-problem rows (workload 0, other knee frequencies, FP32, GMRES, noise, "
                         "per-sample form); the batched rows still run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="copy 1 GiB device to device once (the reference kernel that scales HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the destriping path of this library is "
              f"single-GPU; independent channels and realizations shard across GPUs with no exchange.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1309_5609_amd import dst
    from synth import workload

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    log(f"generating workload {args.workload} (f_k {args.fknee} Hz)")
    t = time.perf_counter()
    p = workload(args.workload, fknee_hz=args.fknee)
    log(f"generated {p.n_samples:,} samples in {time.perf_counter() - t:.1f} s")
    dp = dst.to_device(p)
    torch.cuda.synchronize()
    log("inputs resident in HBM")
    ctx = dst.Context(0)
    ceil = ceilings()
    log(f"ceilings: copy {ceil['copy_GBs']:.0f} GB/s, read {ceil['read_GBs']:.0f} GB/s")
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst_t = torch.empty_like(src)
        torch.cuda.synchronize()
        dst_t.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB device to device")
        del src, dst_t

    # timed: K solves as a caller runs them (CG iterations replayed from a captured graph)
    for i in range(args.warmup):
        out = dst.dst_solve(ctx, dp, tol=args.tol, max_iter=3000)
        log(f"warmup {i}: {out['iterations']} iterations, {out['t_total_ms']:.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [scalars(dst.dst_solve(ctx, dp, tol=args.tol, max_iter=3000)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    iters = sum(r["iterations"] for r in plain)
    value = p.n_samples * iters / wall
    log(f"timed {args.steps} solves: {wall * 1e3:.1f} ms, {iters} iterations, {value:.3e} samples*iters/s")
    # the same K solves again with HIP events around every kernel of every iteration on the solve's stream
    # (DST_SOLVE_PROFILE: kernels launched one by one): kernel durations for the roofline
    torch.cuda.synchronize()
    tp = time.perf_counter()
    runs = [scalars(dst.dst_solve(ctx, dp, tol=args.tol, max_iter=3000, flags=dst.DST_SOLVE_PROFILE))
            for _ in range(args.steps)]
    torch.cuda.synchronize()
    prof_wall = time.perf_counter() - tp
    r0 = runs[-1]

    n_obs = int(r0["n_valid_pix"][0])
    n_runs = int(r0["n_runs"])
    s_psi = 4 if args.workload == 2 else 8
    mb = model_bytes(p.n_samples, n_obs, p.n_baselines, s_psi)
    rb = run_form_bytes(n_runs, n_obs, p.n_baselines, s_psi, p.baseline_length)
    k_ms = {k: float(np.mean([r[f"t_{k}_ms"] for r in runs])) for k in ("bin", "apply", "unbin", "update")}
    dom = max(("bin", "unbin"), key=lambda k: k_ms[k])
    rt = "float" if args.workload == 2 else "double"
    dom_kernel = {"bin": f"k_bin_runs<{rt}, true, true, false, 32, true>",
                  "unbin": f"k_unbin_runs<{rt}, true, true, false, true, 4, true>"}[dom]
    traffic = measured_traffic(dom_kernel)
    launch_s = k_ms[dom] * 1e-3
    achieved = mb[dom] / launch_s / 1e9
    iter_ms = float(np.mean([r["t_iter_ms"] for r in plain]))
    setup_ms = float(np.mean([r["t_setup_ms"] for r in plain]))

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "samples*CG-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.workload != 2 else "f32-in/f64",
        "data": "synthetic",
        "config": {"workload": workload_name(args.workload, args.fknee), "n_samples": p.n_samples,
                   "n_pix": p.n_pix, "baseline_length": p.baseline_length, "n_baselines": p.n_baselines,
                   "streams": p.streams, "tol": args.tol, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "kernel": dom_kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": mb[dom], "avg_launch_ms": k_ms[dom],
                     "bytes_model": ("per-sample algorithmic bytes of the method (pixel + angle per sample, block "
                                     "inverse and map per observed pixel, p / q per baseline); the kernel reads "
                                     "run-compressed pointing instead, so it moves fewer bytes than this"),
                     "frac_run_form": rb[dom] / launch_s / 1e9 / HBM_PEAK_GBS,
                     "run_form_bytes_per_launch": rb[dom],
                     "frac_counter": (traffic / launch_s / 1e9 / HBM_PEAK_GBS) if traffic else None,
                     "frac_of_measured_copy": achieved / ceil["copy_GBs"],
                     "frac_of_measured_read": achieved / ceil["read_GBs"],
                     "timing": ("HIP events around each kernel launch on the solve's stream, over a second "
                                f"timed pass of the same {args.steps} solves ({prof_wall * 1e3 / args.steps:.2f} ms "
                                "per solve with the events)")},
        "ceilings": ceil,
        "iterations_per_solve": r0["iterations"],
        "iter_ms": iter_ms,
        "setup_ms": setup_ms,
        "iteration_throughput": p.n_samples / (iter_ms * 1e-3),
        "iteration_model_bytes": mb["iteration"],
        "iteration_hbm_frac": mb["iteration"] / (iter_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "kernel_ms": k_ms,
        "n_runs": n_runs,
        "observed_pixels": n_obs,
        "n_components": r0["n_components"],
        "rel_residual": r0["rel_residual"],
        "true_rel_residual": r0["true_rel_residual"],
    }

    if args.workload == 1 and not args.no_extra and not args.no_single_extras:
        # workload 0: six hours at N_side 64 (cache-resident; microseconds per iteration)
        p0 = workload(0)
        d0 = dst.to_device(p0)
        res0, w0 = timed_solves(ctx, d0, args.tol, 10, 2)
        it0 = sum(r["iterations"] for r in res0)
        line["workload_0"] = {"value": p0.n_samples * it0 / w0, "unit": "samples*CG-iters/s",
                              "ms_per_solve": w0 * 1e3 / 10, "iterations": res0[0]["iterations"],
                              "us_per_iteration": float(np.mean([r["t_iter_ms"] for r in res0])) * 1e3,
                              "setup_ms": float(np.mean([r["t_setup_ms"] for r in res0]))}
        del d0, p0
        log(f"workload 0: {line['workload_0']['us_per_iteration']:.1f} us per iteration")

        # the other knee frequencies of the 30-day workload (noise drawn on the GPU over the same pointing and sky)
        sky_d = torch.from_numpy(p.sky).to("cuda")
        fk_rows = {}
        for fk in (0.02, 0.2):
            tod = gpu_noise_problem(ctx, dp, sky_d, 77 + int(fk * 1000), fk)
            dpk = dst.Problem(dp.pix, dp.psi, tod, dp.n_pix, dp.baseline_length, dp.streams, dp.weights)
            resk, wk = timed_solves(ctx, dpk, args.tol, 3, 1)
            itk = sum(r["iterations"] for r in resk)
            fk_rows[f"{fk * 1e3:g} mHz"] = {"value": p.n_samples * itk / wk, "ms_per_solve": wk * 1e3 / 3,
                                            "iterations": resk[0]["iterations"],
                                            "iter_ms": float(np.mean([r["t_iter_ms"] for r in resk]))}
            del tod, dpk
        line["workload_1_fknee"] = dict(fk_rows, inputs="same pointing and sky; white 1 mK + 1/f noise (alpha 1.7) "
                                                        "drawn by dst_noise_generate")
        log(f"f_k rows: {json.dumps({k: v['iterations'] for k, v in fk_rows.items()})}")

        # mixed precision on the same data: FP32 timelines and angles (FP64 accumulation, inverse and CG)
        dp32 = dst.Problem(dp.pix, dp.psi.float(), dp.tod.float(), dp.n_pix, dp.baseline_length, dp.streams,
                           dp.weights)
        mruns, mwall = timed_solves(ctx, dp32, args.tol, args.steps, 1)
        mit = sum(r["iterations"] for r in mruns)
        mprof = dst.dst_solve(ctx, dp32, tol=args.tol, max_iter=3000, flags=dst.DST_SOLVE_PROFILE, maps=False)
        ref64 = dst.dst_solve(ctx, dp, tol=1e-12, max_iter=3000)
        out32 = dst.dst_solve(ctx, dp32, tol=1e-12, max_iter=3000)
        base_err, map_err = error_statement(dp, out32, ref64, p.baseline_length)
        mb32 = model_bytes(p.n_samples, n_obs, p.n_baselines, 4)
        m_it = float(np.mean([r["t_iter_ms"] for r in mruns]))
        line["mixed_form"] = {
            "value": p.n_samples * mit / mwall, "ms_per_step": mwall * 1e3 / args.steps, "iter_ms": m_it,
            "setup_ms": float(np.mean([r["t_setup_ms"] for r in mruns])), "iterations_per_solve": mit // args.steps,
            "kernel_ms": {k: mprof[f"t_{k}_ms"] for k in ("bin", "unbin")},
            "iteration_hbm_frac": mb32["iteration"] / (m_it * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "error_statement": {"baseline_rms_error_in_sigma_over_sqrtL": base_err,
                                "map_rms_error_in_white_noise_map_rms": map_err,
                                "reference": ("the library's FP64 solve of the FP64 inputs at tolerance 1e-12 (oracle-"
                                              "pinned at one day and at sampled outputs of the full size); both at "
                                              "tolerance 1e-12"),
                                "bound": 1e-3},
            "dtype": "f32 timelines and angles, f32 run records, f64 accumulation / inverse / CG"}
        del dp32, ref64, out32
        log(f"mixed form: {line['mixed_form']['value']:.3e} samples*iters/s, errors {base_err} {map_err}")

        # the paper's solver: restarted GMRES against PCG at a 1e-12 reduction, same data
        dst.dst_solve(ctx, dp, tol=1e-12, max_iter=3000, flags=dst.DST_SOLVE_GMRES, maps=False)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        gm = dst.dst_solve(ctx, dp, tol=1e-12, max_iter=3000, flags=dst.DST_SOLVE_GMRES)
        torch.cuda.synchronize()
        tg = time.perf_counter() - tg
        tc = time.perf_counter()
        cg = dst.dst_solve(ctx, dp, tol=1e-12, max_iter=3000)
        torch.cuda.synchronize()
        tc = time.perf_counter() - tc
        line["gmres_vs_pcg"] = {
            "tol": 1e-12, "restart": 50,
            "gmres": {"iterations": gm["iterations"], "ms_per_solve": tg * 1e3, "iter_ms": gm["t_iter_ms"],
                      "true_rel_residual": gm["true_rel_residual"]},
            "pcg": {"iterations": cg["iterations"], "ms_per_solve": tc * 1e3, "iter_ms": cg["t_iter_ms"],
                    "true_rel_residual": cg["true_rel_residual"]},
            "baseline_rel_diff": float(torch.linalg.norm(gm["baselines"] - cg["baselines"]) /
                                       torch.linalg.norm(cg["baselines"]))}
        del gm, cg
        log(f"GMRES {line['gmres_vs_pcg']['gmres']['iterations']} / PCG {line['gmres_vs_pcg']['pcg']['iterations']}")

        # the Monte Carlo noise generator (Eq. 1) on the workload's three timelines
        line["noise_form"] = noise_form(ctx, p.n_samples)

        # the per-sample form of the same solve, for comparison with the per-sample byte model
        ps = dst.dst_solve(ctx, dp, tol=args.tol, max_iter=3000, maps=False,
                           flags=dst.DST_SOLVE_PROFILE | dst.DST_SOLVE_PER_SAMPLE)
        ps_ms = {k: ps[f"t_{k}_ms"] for k in ("bin", "unbin", "update")}
        ps_dom = max(("bin", "unbin"), key=lambda k: ps_ms[k])
        ps_ach = mb[ps_dom] / (ps_ms[ps_dom] * 1e-3) / 1e9
        line["per_sample_form"] = {"iter_ms": ps["t_iter_ms"], "kernel_ms": ps_ms, "iterations": ps["iterations"],
                                   "dominant": ps_dom, "achieved_GBs": ps_ach, "frac": ps_ach / HBM_PEAK_GBS}
        del sky_d

    if args.workload == 1 and args.realizations > 0 and not args.no_extra:
        line["batched_form"] = batched_form(ctx, p, dp, args.realizations, args.tol, args.steps, args.warmup, value)
    if args.workload == 1 and not args.no_uneven and not args.no_extra:
        line["uneven_form"] = uneven_form(ctx, args.tol, max(1, args.steps // 3), args.warmup)

    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        line["cpu_baseline"] = cpu_baseline(p)
        if args.workload == 1:
            log("timing the all-core C++ destriper on the host")
            try:
                line["cpu_parallel"] = cpu_parallel(p, line.get("batched_form") or {}, line.get("uneven_form"))
                log(f"C++: {line['cpu_parallel']['workload_1']['total_s']:.1f} s per 30-day solve on "
                    f"{line['cpu_parallel']['threads']} threads")
            except RuntimeError as e:
                line["cpu_parallel"] = {"error": str(e)}
    else:
        line["cpu_baseline"] = None
    ctx.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
