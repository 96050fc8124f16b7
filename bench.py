#!/usr/bin/env python3
"""Destriping throughput on one MI355X: samples x CG-iterations per second.

One step is one complete destriping solve of the workload through the C ABI
(``dst_solve``): pointing setup (hits, per-pixel blocks and their inverse,
baseline counts), right-hand side, preconditioned CG to the tolerance, and
the binned and destriped maps.  ``value`` is n_samples x CG iterations summed
over the timed steps divided by their wall time, with the inputs already in
HBM.  The per-kernel device times come from HIP events the library records
on its stream during the timed steps.

Workloads (seeded synthetic inputs, see ``synth``):
  1 (default): 30 days at 50 Hz = 129,600,000 samples, HEALPix N_side 256,
     3000-sample baselines (43,200 per stream), T/q/u streams, white 1 mK +
     1/f noise (f_k = 50 mHz, alpha = 1.7), FP64, CG to 1e-10.
  0: 6 h = 1,080,000 samples at N_side 64, same scan and noise, FP64.
  2: workload 1 with FP32 timelines and angles (FP64 accumulation and CG).

With workload 1 the line also carries the FP32 mixed-precision form and the
batched Monte Carlo form (``dst_solve_batched``): 32 noise realizations
(white 1 mK + 1/f, f_k 50 mHz, alpha 1.7, drawn on the GPU) of the same sky
over the shared 30-day pointing, FP32 timelines and angles, solved together;
its throughput is realizations x samples x CG-iterations per second.

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
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "runs_30day_nside256_hbm_traffic.md")
RUN_KERNELS_SRC = os.path.join(ROOT, "paper_1309_5609_amd", "csrc", "dst_runs.hip")


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


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def scalars(out: dict) -> dict:
    """A solve's info without its output tensors, so that K solves in a row do not hold K sets of maps
    (a caller that kept them all would make every solve allocate new device memory)."""
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


def algorithmic_bytes(n_t: int, n_obs: int, n_b: int, s_psi: int, n_runs: int = 0, L: int = 3000) -> dict:
    """Bytes each kernel of one CG iteration must move (per launch).

    Per-sample form (the method as written, samples streamed every iteration):
      bin:    pointing (4 B pixel or baseline index + s_psi angle) per sample,
              p (3 x 8 B per baseline) in, the 3 values of each observed
              pixel out (24 B);
      unbin:  pointing per sample, the 3 map values of each observed pixel
              in, p in and q out (2 x 3 x 8 B per baseline).
    Run form (default): one record per run replaces the per-sample pointing:
    a 32-bit key (index and length packed when both fit 32 bits, as the
    library does; else 8 B) and the sums of cos 2psi and sin 2psi (2 x 8 B,
    2 x 4 B with FP32 angles); per-pixel and per-baseline terms as above.
    """
    out = {
        "bin_samples": n_t * (4 + s_psi) + n_obs * 24 + 3 * n_b * 8,
        "unbin_samples": n_t * (4 + s_psi) + n_obs * 24 + 2 * 3 * n_b * 8,
    }
    if n_runs:
        nb = key_bits(L)
        packed = key_bits(max(n_obs, 1)) + nb <= 32 and key_bits(n_b) + nb <= 32
        rec = (4 if packed else 8) + 2 * s_psi
        out["run_record_bytes"] = rec
        out["bin_runs"] = n_runs * rec + n_obs * 24 + 3 * n_b * 8
        out["unbin_runs"] = n_runs * rec + n_obs * 24 + 2 * 3 * n_b * 8
    return out


def cpu_baseline(p, seconds_target: float = 15.0) -> dict:
    """The oracle's operator on the first day of the workload, NumPy FP64 on one host thread."""
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


def batched_form(ctx, p, dp, n_real: int, tol: float, steps: int, warmup: int, plain_value: float) -> dict:
    """Monte Carlo batch: n_real realizations sharing dp's pointing, FP32 timelines, one batched solve."""
    import numpy as np
    import torch

    from paper_1309_5609_amd import dst
    from synth import signal_timelines
    from synth.noise import one_over_f_torch

    n = p.n_samples
    sigma, fk, alpha = 1e-3, 0.05, 1.7
    t = time.perf_counter()
    sig = np.zeros((3, n))
    signal_timelines(p.sky, p.pix, p.psi, "TQU", sig)
    sig_d = torch.from_numpy(sig).to("cuda")
    del sig
    tods, tod0 = [], torch.empty((3, n), dtype=torch.float64, device="cuda")
    for r in range(n_real):
        x32 = torch.empty((3, n), dtype=torch.float32, device="cuda")
        for k in range(3):
            g = torch.Generator(device="cuda")
            g.manual_seed(1309_5609_000 + 3 * r + k)
            x = sig_d[k] + one_over_f_torch(g, n, 50.0, sigma, fk, alpha)
            x32[k] = x.float()
            if r == 0:
                tod0[k] = x32[k].double()
            del x
        tods.append(x32)
    del sig_d
    torch.cuda.synchronize()
    log(f"batched form: {n_real} realizations drawn in {time.perf_counter() - t:.1f} s")
    psi32 = dp.psi.float()
    probs = [dst.Problem(dp.pix, psi32, x, dp.n_pix, dp.baseline_length, dp.streams, dp.weights) for x in tods]
    for _ in range(max(warmup, 1)):
        dst.dst_solve_batched(ctx, probs, tol=tol, max_iter=2000, maps=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    its = 0
    for _ in range(steps):
        _, res = dst.dst_solve_batched(ctx, probs, tol=tol, max_iter=2000)
        its += sum(r["iterations"] for r in res)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = n * its / wall
    _, prof = dst.dst_solve_batched(ctx, probs, tol=tol, max_iter=2000, flags=dst.DST_SOLVE_PROFILE, maps=False)
    # equal map accuracy: realization 0 in FP64 (the FP32 timelines promoted) by the plain FP64 solve
    ref = dst.dst_solve(ctx, dst.Problem(dp.pix, dp.psi, tod0, dp.n_pix, dp.baseline_length, dp.streams,
                                         dp.weights), tol=tol, max_iter=2000)
    obs = ref["hits"].cpu().numpy() > 0
    m64 = ref["destriped_map"].cpu().numpy()[obs]
    m32 = res[0]["destriped_map"].cpu().numpy()[obs]
    sky = p.sky[obs]
    ratio = [float(np.sqrt(np.mean((m32[:, c] - sky[:, c]) ** 2)) / np.sqrt(np.mean((m64[:, c] - sky[:, c]) ** 2)))
             for c in range(3)]
    out = {"value": value, "unit": "realizations*samples*CG-iters/s", "n_realizations": n_real,
           "ms_per_solve": wall * 1e3 / steps, "setup_ms": res[0]["t_setup_ms"],
           "iter_ms": res[0]["t_iter_ms"], "iterations": [r["iterations"] for r in res],
           "kernel_ms": {k: prof[0][f"t_{k}_ms"] for k in ("bin", "unbin", "update")},
           "vs_plain_fp64": value / plain_value,
           "map_rms_error_ratio_vs_fp64": ratio,
           "dtype": "f32 timelines and angles, f64 accumulation / inverse / CG",
           "inputs": ("sky signal of the 30-day workload + per-realization white 1 mK and 1/f noise "
                      "(f_k 50 mHz, alpha 1.7) drawn on the GPU by FFT filtering")}
    del probs, tods, tod0, res, prof, ref
    torch.cuda.empty_cache()
    log(f"batched form: {value:.3e} realizations*samples*iters/s ({out['vs_plain_fp64']:.2f}x plain FP64)")
    return out


# Uneven batch of channels: 8 polarimeter channels of 3 .. 30 days plus a
# 12-month intensity-only stream at N_side 512, FP32 timelines and angles.
# Per channel: days, baseline length, f_k (Hz), alpha, spin-axis phase.
UNEVEN_CHANNELS = [(3, 1500, 0.010, 1.0), (5, 2000, 0.015, 1.15), (7, 2500, 0.022, 1.3), (10, 3000, 0.033, 1.45),
                   (14, 3500, 0.050, 1.6), (20, 4000, 0.075, 1.75), (25, 5000, 0.110, 1.9), (30, 6000, 0.200, 2.0)]
UNEVEN_T_STREAM = (365, 6000, 0.010, 1.0)


def uneven_form(ctx, tol: float, steps: int, warmup: int) -> dict:
    """The uneven channel batch, generated on the GPU by the library (pointing expansion, sky scan, noise) and solved by
    dst_solve_batched (channels share no pointing, so they are solved one after another, autotuned)."""
    import numpy as np
    import torch

    from paper_1309_5609_amd import dst
    from synth import ScanSpec, gaussian_sky

    nside, rate, sigma = 512, 50.0, 1e-3
    n_pix = 12 * nside * nside
    t = time.perf_counter()
    sky = torch.from_numpy(gaussian_sky(n_pix, 4)).to("cuda")
    w = 1.0 / (sigma * sigma)
    probs, desc = [], []
    specs = [(c, days, L, fk, al, "TQU") for c, (days, L, fk, al) in enumerate(UNEVEN_CHANNELS)]
    specs.append((len(UNEVEN_CHANNELS),) + UNEVEN_T_STREAM + ("T",))
    for c, days, L, fk, al, streams in specs:
        n = int(days * 86400 * rate)
        scan = ScanSpec(sample_rate_hz=rate, az0_deg=37.0 * c, psi0_deg=22.5 * c)
        pix, psi = dst.dst_pointing_expand(ctx, scan, nside, n, psi_dtype=torch.float32)
        rows = 1 if streams == "T" else 3
        head = dst.Problem(pix, psi if streams != "T" else None, None, n_pix, L, streams, (w, w, w))
        sig = dst.dst_unbin(ctx, head, sky)              # A m_sky per stream, FP64
        tod = sig.float()
        del sig
        for k in range(rows):
            dst.dst_noise_generate(ctx, 4000 + c, k, n, 1 << 22, rate, sigma, fk, al, out=tod[k], accumulate=True)
        probs.append(dst.Problem(pix, psi if streams != "T" else None, tod, n_pix, L, streams, (w, w, w)))
        desc.append({"days": days, "n_samples": n, "baseline_length": L, "fknee_hz": fk, "alpha": al,
                     "streams": streams})
        if streams == "T":
            del psi
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    log(f"uneven batch: {len(probs)} problems, {sum(d['n_samples'] for d in desc):,} samples drawn on the GPU "
        f"in {gen_s:.1f} s")
    flags = dst.DST_SOLVE_AUTOTUNE
    for _ in range(max(warmup, 1)):
        dst.dst_solve_batched(ctx, probs, tol=tol, max_iter=3000, flags=flags, maps=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    work = 0
    for _ in range(steps):
        _, res = dst.dst_solve_batched(ctx, probs, tol=tol, max_iter=3000, flags=flags, maps=False)
        work += sum(d["n_samples"] * r["iterations"] for d, r in zip(desc, res))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for d, r in zip(desc, res):
        d.update(iterations=r["iterations"], converged=r["converged"], setup_ms=r["t_setup_ms"],
                 iter_ms=r["t_iter_ms"], total_ms=r["t_total_ms"], n_runs=r["n_runs"])
    out = {"value": work / wall, "unit": "samples*CG-iters/s", "ms_per_step": wall * 1e3 / steps,
           "n_problems": len(probs), "total_samples": sum(d["n_samples"] for d in desc), "nside": nside,
           "dtype": "f32 timelines and angles, f64 accumulation / inverse / CG", "problems": desc,
           "inputs": ("pointing expanded on the GPU (dst_pointing_expand), Gaussian sky (I 1 mK, Q/U 0.1 mK) scanned "
                      "by dst_unbin, white 1 mK + 1/f noise by dst_noise_generate (segments of 2^22 samples)")}
    del probs, res, sky
    torch.cuda.empty_cache()
    log(f"uneven batch: {out['value']:.3e} samples*iters/s, {out['ms_per_step']:.0f} ms per batch")
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
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven channel batch (N_side 512)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference kernel for HBM counters)")
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

    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        dstb = torch.empty_like(src)
        src.fill_(1.0)
        dstb.copy_(src)
        torch.cuda.synchronize()
        del src, dstb

    for i in range(args.warmup):
        out = dst.dst_solve(ctx, dp, tol=args.tol, max_iter=2000)
        log(f"warmup {i}: {out['iterations']} iterations, {out['t_total_ms']:.1f} ms")

    # timed: K solves as a caller runs them (CG iterations replayed from a captured graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = []
    for i in range(args.steps):
        plain.append(scalars(dst.dst_solve(ctx, dp, tol=args.tol, max_iter=2000)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    iters = sum(r["iterations"] for r in plain)
    value = p.n_samples * iters / wall
    log(f"timed {args.steps} solves: {wall * 1e3:.1f} ms, {iters} iterations, {value:.3e} samples*iters/s")
    # the same K solves again with HIP events around every kernel of every iteration on the solve's stream
    # (DST_SOLVE_PROFILE: kernels launched one by one, so this pass is slower): kernel durations for the roofline
    torch.cuda.synchronize()
    tp = time.perf_counter()
    runs = [scalars(dst.dst_solve(ctx, dp, tol=args.tol, max_iter=2000, flags=dst.DST_SOLVE_PROFILE))
            for _ in range(args.steps - 1)]
    runs.append(dst.dst_solve(ctx, dp, tol=args.tol, max_iter=2000, flags=dst.DST_SOLVE_PROFILE))
    torch.cuda.synchronize()
    prof_wall = time.perf_counter() - tp
    r0 = runs[-1]

    n_obs = int(r0["n_valid_pix"][0])
    n_runs = int(r0["n_runs"])
    s_psi = 4 if args.workload == 2 else 8
    algo = algorithmic_bytes(p.n_samples, n_obs, p.n_baselines, s_psi, n_runs, p.baseline_length)
    k_ms = {k: float(np.mean([r[f"t_{k}_ms"] for r in runs])) for k in ("bin", "apply", "unbin", "update")}
    dom = max(("bin", "unbin"), key=lambda k: k_ms[k])
    dom_bytes = algo[f"{dom}_runs"]
    rt = "float" if args.workload == 2 else "double"
    # the default launch shapes: 32 lanes per pixel in the binning, 4 baselines per wavefront in the rescan,
    # packed 32-bit run keys
    dom_kernel = {"bin": f"k_bin_runs<{rt}, true, true, false, 32, true>",
                  "unbin": f"k_unbin_runs<{rt}, true, true, false, true, 4, true>"}[dom]
    traffic = measured_traffic(dom_kernel)
    achieved = dom_bytes / (k_ms[dom] * 1e-3) / 1e9
    iter_ms = float(np.mean([r["t_iter_ms"] for r in plain]))
    b_iter = algo["bin_samples"] + algo["unbin_samples"]

    # mixed precision on the same data: FP32 timelines and angles (FP64 accumulation, inverse and CG)
    mixed = None
    if args.workload == 1:
        dp32 = dst.Problem(dp.pix, dp.psi.float(), dp.tod.float(), dp.n_pix, dp.baseline_length, dp.streams,
                           dp.weights)
        dst.dst_solve(ctx, dp32, tol=args.tol, max_iter=2000)
        torch.cuda.synchronize()
        tm = time.perf_counter()
        mruns = [scalars(dst.dst_solve(ctx, dp32, tol=args.tol, max_iter=2000)) for _ in range(args.steps)]
        torch.cuda.synchronize()
        mwall = time.perf_counter() - tm
        mit = sum(r["iterations"] for r in mruns)
        mprof = dst.dst_solve(ctx, dp32, tol=args.tol, max_iter=2000, flags=dst.DST_SOLVE_PROFILE)
        mixed = {"value": p.n_samples * mit / mwall, "ms_per_step": mwall * 1e3 / args.steps,
                 "iter_ms": float(np.mean([r["t_iter_ms"] for r in mruns])),
                 "setup_ms": float(np.mean([r["t_setup_ms"] for r in mruns])),
                 "iterations_per_solve": mruns[-1]["iterations"],
                 "kernel_ms": {k: mprof[f"t_{k}_ms"] for k in ("bin", "unbin")},
                 "dtype": "f32 timelines and angles, f32 run records, f64 accumulation / inverse / CG"}
        del dp32
        log(f"mixed form: {mixed['value']:.3e} samples*iters/s")

    # the paper's solver: restarted GMRES against PCG at a 1e-12 reduction, same data
    log("GMRES vs PCG at 1e-12")
    gm = dst.dst_solve(ctx, dp, tol=1e-12, max_iter=2000, flags=dst.DST_SOLVE_GMRES)
    torch.cuda.synchronize()
    tg = time.perf_counter()
    gm = dst.dst_solve(ctx, dp, tol=1e-12, max_iter=2000, flags=dst.DST_SOLVE_GMRES)
    torch.cuda.synchronize()
    tg = time.perf_counter() - tg
    tc = time.perf_counter()
    cg = dst.dst_solve(ctx, dp, tol=1e-12, max_iter=2000)
    torch.cuda.synchronize()
    tc = time.perf_counter() - tc
    gmres = {"tol": 1e-12, "restart": 50,
             "gmres": {"iterations": gm["iterations"], "ms_per_solve": tg * 1e3, "iter_ms": gm["t_iter_ms"],
                       "true_rel_residual": gm["true_rel_residual"]},
             "pcg": {"iterations": cg["iterations"], "ms_per_solve": tc * 1e3, "iter_ms": cg["t_iter_ms"],
                     "true_rel_residual": cg["true_rel_residual"]},
             "baseline_rel_diff": float(torch.linalg.norm(gm["baselines"] - cg["baselines"]) /
                                        torch.linalg.norm(cg["baselines"]))}
    log(f"GMRES {gm['iterations']} iterations {tg * 1e3:.1f} ms; PCG {cg['iterations']} iterations {tc * 1e3:.1f} ms")

    batched = None
    if args.workload == 1 and args.realizations > 0:
        batched = batched_form(ctx, p, dp, args.realizations, args.tol, args.steps, args.warmup, value)
    uneven = None
    if args.workload == 1 and not args.no_uneven:
        uneven = uneven_form(ctx, args.tol, max(1, args.steps // 3), args.warmup)

    # the per-sample form of the same solve, for comparison with the per-sample byte model
    log("per-sample form: one profiled solve")
    ps = dst.dst_solve(ctx, dp, tol=args.tol, max_iter=2000,
                       flags=dst.DST_SOLVE_PROFILE | dst.DST_SOLVE_PER_SAMPLE)
    ps_ms = {k: ps[f"t_{k}_ms"] for k in ("bin", "unbin", "update")}
    ps_dom = max(("bin", "unbin"), key=lambda k: ps_ms[k])
    ps_ach = algo[f"{ps_dom}_samples"] / (ps_ms[ps_dom] * 1e-3) / 1e9

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
                     "algorithmic_bytes_per_launch": dom_bytes, "avg_launch_ms": k_ms[dom],
                     "timing": ("HIP events around each kernel launch on the solve's stream, over a second "
                                f"timed pass of the same {args.steps} solves ({prof_wall * 1e3 / args.steps:.2f} ms "
                                "per solve with the events)")},
        "per_sample_model": {"bytes_per_iteration": b_iter,
                             "equivalent_GBs": b_iter / (iter_ms * 1e-3) / 1e9,
                             "note": "per-sample algorithmic bytes of one CG iteration / measured iteration time"},
        "per_sample_form": {"iter_ms": ps["t_iter_ms"], "kernel_ms": ps_ms, "iterations": ps["iterations"],
                            "dominant": ps_dom, "achieved_GBs": ps_ach, "frac": ps_ach / HBM_PEAK_GBS},
        "n_runs": n_runs,
        "mixed_form": mixed,
        "batched_form": batched,
        "gmres_vs_pcg": gmres,
        "uneven_form": uneven,
        "iterations_per_solve": r0["iterations"],
        "iter_ms": iter_ms,
        "iteration_throughput": p.n_samples / (iter_ms * 1e-3),
        "iteration_hbm_frac": b_iter / (iter_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "setup_ms": float(np.mean([r["t_setup_ms"] for r in plain])),
        "kernel_ms": k_ms,
        "rel_residual": r0["rel_residual"],
        "true_rel_residual": r0["true_rel_residual"],
        "observed_pixels": n_obs,
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        line["cpu_baseline"] = cpu_baseline(p)
    else:
        line["cpu_baseline"] = None
    ctx.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
