#!/usr/bin/env python3
"""Benchmark of the Chebyshev-moment hot path on one MI355X.

Workload (one "step" = one pass of the whole path over one batch of input):
spin-1/2 Heisenberg ring, N = 24, J = 1, S^z = 0 sector (2,704,156 states),
10 complex Gaussian random vectors (20 real columns; column-block width, step
kernel and tile shape autotuned in the warm-up), M = 2000 moments (1000
recursion launches), eps = 0.025, bounds from 50-step Lanczos with
a 1% margin, float32 vector storage with float64 arithmetic and dots, then the
Jackson-kernel thermodynamics at 200 log-spaced temperatures in [0.01, 10].

`value` is state-column-steps per second of the whole pass (dim x real columns
x recursion steps / wall time of the pass, inputs resident on the GPU).  The
JSON line also carries:
  roofline      (also `measured_GBs` = counter bytes / launch time, and
                `copy_GBs` = a 1 GiB device copy's rate, the achievable line)
                the step kernel's algorithmic HBM bytes (3 x 4 B per state and
                column, + 4 B per state when the kernel streams the state
                words) over its average launch time, measured with hipEvents on
                the launch stream during the timed passes; `traffic` is the
                rocprofv3-measured bytes per launch from the committed counter
                summary, or null
  fp64_plain    the same recursion in float64, one column per block (the
                reference form), and fp64_batched (float64, tuned blocks)
  fp32r         the same recursion with float32 + 16-bit residual storage
                (6 bytes per element, relative storage error <= 2^-38): rate,
                speedups over both float64 comparators, and its accuracy
  speedup_at_error_1e-6  float32 form (and the fp32r form) over fp64_plain,
                with the temperature band in which C(T) and chi(T) stay
                within 1e-6 of float64
  accuracy      float32-storage (and fp32r) error against float64 on the same
                seeds, all 13 S^z >= 0 sectors of the ring: C(T), chi(T),
                ln Z, E, moments
  cpu_baseline  the CPU oracle on a bounded sample of the same workload (32
                recursion steps of the same sector and columns): on the host's
                cores (up to the 16 of a one-GPU share, columns split over
                forked processes, run before this process touches the GPU) and
                on one core; the host's core count and CPU model are recorded

`--workload` measures one of the other workloads instead (one JSON line of
the same form, no CPU leg): batched_rr3 (64 random 3-regular clusters,
N = 16..22, all sectors, 32 Rademacher vectors, float32, M = 1024),
j1j2_grad (the adjoint: dL/dJ of L = sum_T C(T) for the J1-J2 chain N = 20,
S^z = 0, 16 vectors, float64, M = 1000, checkpoints every 64 steps), rr4_30
(random 4-regular graph, N = 30, S^z = 0 = 155,117,520 states, 4 Rademacher
vectors, M = 500, float32 and float64), ftlm_ring24 (finite-temperature
Lanczos on the headline sector, 20 real columns, 200 Lanczos steps), fe10
(the spin-5/2 ferric wheel, all 26 sectors, 100 vectors, M = 200) and
ed_batched (exact spectra of the batched clusters' sectors of D <= 1024).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Chebyshev steps·dim/s + HBM GB/s at N=24 S^z=0; speedup vs FP64 at C(T) err"
HBM_PEAK_GBS = 8000.0
# step kernel families as reported by kpm_last_run_stats()["kernel"]
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X, dense float64 vector arithmetic
KERNEL_FAMILY = {0: "step_kernel", 1: "row_kernel", 2: "block_kernel", 3: "tab_kernel", 4: "spin_kernel",
                 5: "slice_kernel"}
PROFILES = os.path.join(ROOT, "profiles")


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--M", type=int, default=2000)
    ap.add_argument("--skip-extras", action="store_true",
                    help="only the timed workload (for profiler runs)")
    ap.add_argument("--cpu-steps", type=int, default=32,
                    help="recursion steps of the CPU-oracle sample")
    ap.add_argument("--workload", default="ring24_sz0",
                    choices=["ring24_sz0", "batched_rr3", "j1j2_grad", "rr4_30", "ftlm_ring24", "fe10",
                             "ed_batched"])
    ap.add_argument("--accuracy-curve", default=None, metavar="PATH",
                    help="also write the per-T float32-vs-float64 error curves of C and chi (JSON)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device-to-device (reference for HBM byte counters)")
    return ap.parse_args()


def _traffic(family, tag="ring24_sz0_fp32", st=None):
    """Measured HBM-side bytes per step launch from the committed rocprofv3
    counter summary of this kernel on this workload (`tag`), when it was taken
    on the current kernel source and, where the record names the launch shape
    (column block, mean rows per tile, waves per tile), on the shape of the
    run `st`."""
    path = os.path.join(PROFILES, f"{family}_{tag}_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_text_sha256") != kernel_text_sha256(family):
        return None
    # one record, or one per launch shape the tuner may pick
    for rec in d.get("records", [d]):
        shape = rec.get("shape")
        if shape and st is not None and any(st.get(k) != v for k, v in shape.items()):
            continue
        return rec.get("hbm_bytes_per_launch")
    return None


def _shape(st):
    """The launch shape a counter record must share with a run."""
    return {k: st[k] for k in ("col_block", "rows_per_tile", "waves")}


def kernel_text_sha256(family):
    """sha256 of the kernel function's source text (its template line to the
    closing brace in column 0) in the library's sources: a counter record
    stays valid while that text is unchanged."""
    import glob
    import hashlib
    import re
    from paper_2104_13218_amd import build as _b
    for path in sorted(glob.glob(os.path.join(_b.CSRC, "*.hip"))):
        src = open(path).read()
        m = re.search(r"template <[^\n]*>\n__global__[^\n]*void %s\(" % re.escape(family), src)
        if m is not None:
            end = src.index("\n}\n", m.start())
            return hashlib.sha256(src[m.start():end + 3].encode()).hexdigest()
    return None


def _copy_rate(torch):
    """Achievable line: read + write bytes of a 1 GiB device-to-device copy
    over its hipEvent time (best of 5)."""
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * (1 << 30) / best / 1e9


def main():
    args = _parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(the work would shard over independent sectors and column blocks).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W

    # the CPU oracle runs first: its worker processes are forked before
    # anything in this process touches the GPU
    cpu = None
    if args.workload == "ring24_sz0" and not args.skip_extras:
        cpu = cpu_baseline(args, W, np, W.sectors(W.ring(24), only_sz0=True))

    from paper_2104_13218_amd import kpm

    kpm.load()
    torch.cuda.init()
    dev = torch.cuda.get_device_name(0)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.workload != "ring24_sz0":
        print(json.dumps(other_workload(args, kpm, W, np, torch, dev)), flush=True)
        return

    ring = W.ring(24)
    sec = W.sectors(ring, only_sz0=True)
    M = args.M
    T = torch.tensor(W.log_temperatures(200, 0.01, 10.0), device="cuda")
    ps = kpm.ProblemSet(sec)
    # block width, step kernel and tile shape measured by the library's tuner
    q32 = kpm.make_params(M, 10, "complex_gaussian", "fp32", 0.025, 0, col_block=0, autotune=True)
    ws = torch.empty(kpm.moments_workspace_size(ps, q32), dtype=torch.uint8, device="cuda")

    def one_pass():
        mu, ab = kpm.chebyshev_moments(None, M, 10, "complex_gaussian", "fp32", 0.025, 0, col_block=0,
                                       workspace=ws, problems=ps, autotune=True)
        kpm.thermo(mu, ab, ps, T, "jackson")
        return kpm.last_run_stats()

    # measure and cache the launch shape once (a few steps per candidate)
    kpm.chebyshev_moments(None, 8, 10, "complex_gaussian", "fp32", 0.025, 0, col_block=0,
                          workspace=ws, problems=ps, autotune=True)
    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(one_pass())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    st = stats[-1]
    value = st["state_col_steps"] / dt
    avg_launch_s = sum(s["recursion_ms"] for s in stats) / len(stats) / 1e3 / st["step_launches"]
    achieved = st["bytes_per_launch"] / avg_launch_s / 1e9
    family = KERNEL_FAMILY.get(st["kernel"], "step_kernel")
    traffic = _traffic(family, st=st)
    copy_gbs = _copy_rate(torch)
    line = {
        "metric": METRIC, "value": value, "unit": "state-column-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-storage/f64-arithmetic", "data": "synthetic",
        "config": {"workload": "heisenberg_ring_N24_Sz0", "dim": sec[0].dim, "vectors": "10 complex Gaussian",
                   "real_columns": 20, "M": M, "recursion_launches": st["step_launches"], "eps": 0.025,
                   "bounds": "lanczos50+1%", "storage": "f32", "col_block": st["col_block"],
                   "rows_per_tile": st["rows_per_tile"], "waves_per_tile": st["waves"], "graph_segment": st["graph_segment"],
                   "device": dev},
        "roofline": {"bound": "hbm", "kernel": family, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_launch": st["bytes_per_launch"],
                     "avg_launch_us": avg_launch_s * 1e6,
                     "shape": _shape(st), "traffic": traffic,
                     "measured_GBs": None if traffic is None else traffic / avg_launch_s / 1e9,
                     "measured_frac": None if traffic is None else traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS,
                     "copy_GBs": copy_gbs},
    }

    if not args.skip_extras:
        line.update(extras(args, kpm, W, np, torch, sec, ps, T, M, value, ws))
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def _line(args, workload, value, unit, dt, config, roofline=None, extra=None):
    line = {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": dict({"workload": workload}, **config)}
    if roofline is not None:
        line["roofline"] = roofline
    if extra:
        line.update(extra)
    return line


def _roofline(st, tag=None):
    t = st["recursion_ms"] / 1e3 / st["step_launches"]
    ach = st["bytes_per_launch"] / t / 1e9
    family = KERNEL_FAMILY.get(st["kernel"], "step_kernel")
    traffic = _traffic(family, tag, st) if tag else None
    return {"bound": "hbm", "kernel": family, "achieved": ach,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "algorithmic_bytes_per_launch": st["bytes_per_launch"], "avg_launch_us": t * 1e6,
            "shape": _shape(st), "traffic": traffic,
            "measured_GBs": None if traffic is None else traffic / t / 1e9,
            "measured_frac": None if traffic is None else traffic / t / 1e9 / HBM_PEAK_GBS}


def _timed(args, torch, fn):
    """fn() warmup + timed; returns (seconds per call, last result)."""
    out = None
    for _ in range(max(1, args.warmup)):
        out = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / args.steps, out


def other_workload(args, kpm, W, np, torch, dev):
    name = args.workload
    if name in ("batched_rr3", "rr4_30"):
        wl = W.batched_workload() if name == "batched_rr3" else W.rr4_30_workload("fp32")
        ab = kpm.spectral_bounds(wl.problems)              # fixed bounds: Lanczos outside the timing
        ps = kpm.ProblemSet(wl.problems, [tuple(x) for x in ab])
        T = torch.tensor(wl.temperatures, device="cuda")

        def run(prec):
            mu, abd = kpm.chebyshev_moments(None, wl.M, wl.R, wl.vec_kind, prec, wl.eps, wl.seed,
                                            problems=ps, autotune=True)
            kpm.thermo(mu, abd, ps, T, wl.kernel)
            return kpm.last_run_stats()

        dt, st = _timed(args, torch, lambda: run("fp32"))
        dims = [s.dim for s in wl.problems]
        cfg = {"problems": len(dims), "states": int(sum(dims)), "max_dim": int(max(dims)), "M": wl.M,
               "vectors": f"{wl.R} {wl.vec_kind}", "storage": "f32", "col_block": st["col_block"],
               "bounds": "lanczos50+1% (outside the timing)", "device": dev}
        extra = None
        if name == "rr4_30":
            dt64, st64 = _timed(args, torch, lambda: run("fp64"))
            extra = {"fp64": {"value": st64["state_col_steps"] / dt64, "ms": dt64 * 1e3,
                              "roofline": _roofline(st64, "rr4_30_sz0_fp64")},
                     "speedup_vs_fp64": (st["state_col_steps"] / dt) / (st64["state_col_steps"] / dt64)}
        tag = "rr4_30_sz0_fp32" if name == "rr4_30" else "batched_rr3_fp32"
        return _line(args, name, st["state_col_steps"] / dt, "state-column-steps/s", dt, cfg,
                     _roofline(st, tag), extra)
    if name == "fe10":
        wl = W.fe10_workload("fp32")
        ab = kpm.spectral_bounds(wl.problems)              # fixed bounds: Lanczos outside the timing
        ps = kpm.ProblemSet(wl.problems, [tuple(x) for x in ab])
        T = torch.tensor(wl.temperatures, device="cuda")

        def run(prec):
            mu, abd = kpm.chebyshev_moments(None, wl.M, wl.R, wl.vec_kind, prec, wl.eps, wl.seed,
                                            problems=ps)
            kpm.thermo(mu, abd, ps, T, wl.kernel)
            return kpm.last_run_stats()

        dt, st = _timed(args, torch, lambda: run("fp32"))
        dt64, st64 = _timed(args, torch, lambda: run("fp64"))
        dims = [s.dim for s in wl.problems]
        cfg = {"sites": 10, "spin": "5/2", "problems": len(dims), "states": int(sum(dims)),
               "max_dim": int(max(dims)), "M": wl.M, "vectors": f"{wl.R} {wl.vec_kind}", "storage": "f32",
               "col_block": st["col_block"], "bounds": "lanczos50+1% (outside the timing)", "device": dev}
        extra = {"fp64": {"value": st64["state_col_steps"] / dt64, "ms": dt64 * 1e3,
                          "roofline": _roofline(st64, "fe10_fp64")}}
        return _line(args, name, st["state_col_steps"] / dt, "state-column-steps/s", dt, cfg,
                     _roofline(st, "fe10_fp32"), extra)
    if name == "ed_batched":
        # exact spectra of the small sectors of the 64 random clusters (the
        # hybrid form: sectors of dimension <= 1024 diagonalised completely)
        secs = []
        for cid, cl in enumerate(W.batched_clusters(64)):
            secs += W.sectors(cl, cluster_id=cid)
        small = [s for s in secs if s.dim <= 1024]
        ps = kpm.ProblemSet(small)
        dt, _ = _timed(args, torch, lambda: kpm.sector_eigenvalues(ps, 1024))
        # Householder tridiagonalisation: 2 n^2 (A v) + 4 n^2 (rank-2 update) per column
        flops = float(sum(2.0 * s.dim ** 3 for s in small))
        # ... at about half a flop per byte it is bound by memory: each step reads
        # and writes the n x n trailing block once (16 n^2 bytes), n = D-1 .. 2
        nbytes = float(sum(16.0 * ((s.dim - 1) * s.dim * (2 * s.dim - 1) // 6 - 1)
                           for s in small if s.dim > 2))
        ach = nbytes / dt / 1e9
        cfg = {"sectors": len(small), "max_dim": int(max(s.dim for s in small)),
               "states": int(sum(s.dim for s in small)), "storage": "f64", "device": dev}
        # the whole call (build, ~3 launches per Householder step, bisection) against its bytes
        roof = {"bound": "hbm", "kernel": "ed_* (one kpm_sector_eigenvalues call)", "achieved": ach,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "algorithmic_bytes_per_launch": nbytes, "traffic": None,
                "flops": {"algorithmic_flops_per_launch": flops, "achieved_TFLOPs": flops / dt / 1e12,
                          "frac_of_fp64_vector_peak": flops / dt / 1e12 / FP64_VECTOR_PEAK_TFLOPS}}
        return _line(args, name, len(small) / dt, "sectors/s", dt, cfg, roof)
    if name == "j1j2_grad":
        wl = W.j1j2_grad_workload()
        ab = kpm.spectral_bounds(wl.problems)
        bl = [tuple(x) for x in ab]
        T = wl.temperatures
        wC = np.ones((1, T.size))
        wX = np.zeros((1, T.size))

        # every v_n of the forward pass kept (M/2 + 2 vectors of dim x R float64,
        # 12 GB here): the reverse sweep recomputes nothing
        ckpt = wl.M // 2

        def run():
            return kpm.thermo_grad(wl.problems, wl.M, wl.R, T, wC, wX, wl.vec_kind, "fp64", wl.eps, wl.seed,
                                   kernel=wl.kernel, ckpt_every=ckpt, bounds=bl)

        dt, _ = _timed(args, torch, run)

        def forward():
            kpm.chebyshev_moments(wl.problems, wl.M, wl.R, wl.vec_kind, "fp64", wl.eps, wl.seed, bounds=bl)
            return kpm.last_run_stats()

        dtf, stf = _timed(args, torch, forward)
        dim = wl.problems[0].dim
        work = dim * wl.R * (wl.M // 2)
        cfg = {"dim": dim, "bonds": wl.problems[0].cluster.n_bonds, "M": wl.M, "vectors": f"{wl.R} rademacher",
               "storage": "f64", "checkpoint_every": ckpt,
               "trajectory_bytes": (wl.M // 2 + 2) * dim * wl.R * 8, "loss": "sum_T C(T), 64 T in [0.05, 5]",
               "device": dev}
        # the reverse step reads w_{n+1} (gathers), w_{n+2}, v_{n-1}, v_n, v_{n+1}
        # and writes w_n: 6 x 8 bytes per state and column; its launch time is
        # in the committed kernel trace (profiles/j1j2_grad_kernels.md)
        adj = {"kernel": "adjoint_kernel", "launches_per_gradient": wl.M // 2,
               "algorithmic_bytes_per_launch": 6.0 * 8 * wl.R * dim,
               "traffic": _traffic("adjoint_kernel", "j1j2_n20_sz0_fp64")}
        return _line(args, name, work / dt, "forward-equivalent state-column-steps/s", dt, cfg,
                     _roofline(stf, "j1j2_n20_sz0_fp64"),
                     {"forward_ms": dtf * 1e3, "gradient_over_forward_time": dt / dtf, "adjoint": adj})
    if name == "ftlm_ring24":
        sec = W.sectors(W.ring(24), only_sz0=True)
        T = W.log_temperatures(200, 0.01, 10.0)
        ML = 200
        dt, _ = _timed(args, torch, lambda: kpm.ftlm(sec, ML, 10, "complex_gaussian", T=T))
        work = sec[0].dim * 20 * ML
        cfg = {"dim": sec[0].dim, "vectors": "10 complex Gaussian (20 real columns)", "lanczos_steps": ML,
               "storage": "f64", "device": dev}
        return _line(args, name, work / dt, "state-column-steps/s", dt, cfg)
    raise ValueError(name)


def _time_moments(kpm, torch, sec, M, R, kind, precision, col_block, reps=1):
    """One timed call after a warm-up (which also tunes the launch shape for
    this block width)."""
    kpm.chebyshev_moments(sec, M, R, kind, precision, 0.025, 0, col_block=col_block, autotune=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        mu, ab = kpm.chebyshev_moments(sec, M, R, kind, precision, 0.025, 0, col_block=col_block,
                                       autotune=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    st = kpm.last_run_stats()
    return mu, ab, dt, st


def _accuracy(kpm, np, allsec, T, Th, mu64, ab64, mu_f, ab_f, curves=None):
    """Error of a reduced-storage run against float64 on the same vectors:
    moments, and per kernel g_n C(T), chi(T) (peak-normalised on T >= T_phys,
    the lowest grid T from which the float64 estimate has Z > 0 and C >= 0)
    with the lowest T above which the error stays <= 1e-6, ln Z and E."""
    acc = {"moments_max_abs_err_over_mu0": float((mu_f - mu64).abs().max(dim=1).values.div(mu64[:, 0]).max())}
    for kern in ("jackson", "none"):
        t64 = kpm.thermo(mu64, ab64, allsec, T, kern)
        tf = kpm.thermo(mu_f, ab_f, allsec, T, kern)
        C64 = t64["C"].cpu().numpy()[0]
        bad = np.nonzero((C64 < 0) | t64["z_nonpos"].cpu().numpy()[0].astype(bool))[0]
        i_phys = bad.max() + 1 if bad.size else 0
        band = np.arange(Th.size) >= i_phys
        rec = {"T_phys": float(Th[min(i_phys, Th.size - 1)])}
        for qn in ("C", "chi"):
            a = t64[qn].cpu().numpy()[0]
            b = tf[qn].cpu().numpy()[0]
            err = np.abs(a - b) / np.abs(a[band]).max()
            if curves is not None:
                curves[f"{kern}_{qn}_err_over_peak"] = err.tolist()
                curves[f"{kern}_{qn}_fp64"] = a.tolist()
            rec[f"{qn}_max_err_T>=T_phys"] = float(err[band].max())
            lowest = None
            for i in range(Th.size - 1, -1, -1):
                if err[i] > 1e-6:
                    break
                lowest = float(Th[i])
            rec[f"{qn}_lowest_T_with_err<=1e-6"] = lowest
        for qn in ("lnZ", "E"):
            a = t64[qn].cpu().numpy()[0][band]
            b = tf[qn].cpu().numpy()[0][band]
            rec[f"{qn}_max_rel_err_T>=T_phys"] = float(np.nanmax(np.abs(a - b) / np.abs(a)))
        acc[kern] = rec
    return acc


def extras(args, kpm, W, np, torch, sec, ps, T, M, value, ws):
    out = {}
    # float64 comparators on the same workload.  The single-column form needs
    # real vectors (a complex vector's Re and Im share one block): 20 real
    # Gaussian vectors give the same dim x columns x steps.
    _, _, dt, st = _time_moments(kpm, torch, sec, M, 20, "gaussian", "fp64", 1)
    plain = st["state_col_steps"] / dt
    _, _, dtb, stb = _time_moments(kpm, torch, sec, M, 10, "complex_gaussian", "fp64", 0)
    batched = stb["state_col_steps"] / dtb
    out["fp64_plain"] = {"value": plain, "ms": dt * 1e3, "col_block": 1,
                         "avg_launch_us": st["recursion_ms"] * 1e3 / st["step_launches"]}
    out["fp64_batched"] = {"value": batched, "ms": dtb * 1e3, "col_block": stb["col_block"],
                           "avg_launch_us": stb["recursion_ms"] * 1e3 / stb["step_launches"]}
    # recursion-only rate of the float32 form, for a like-for-like speedup
    _, _, dtf, stf = _time_moments(kpm, torch, sec, M, 10, "complex_gaussian", "fp32", 0)
    out["speedup_vs_fp64_plain"] = (stf["state_col_steps"] / dtf) / plain
    out["speedup_vs_fp64_batched"] = (stf["state_col_steps"] / dtf) / batched

    # the float32 + 16-bit residual storage form (6 bytes per element)
    _, _, dtr, str_ = _time_moments(kpm, torch, sec, M, 10, "complex_gaussian", "fp32r", 0)
    out["fp32r"] = {"value": str_["state_col_steps"] / dtr, "ms": dtr * 1e3, "col_block": str_["col_block"],
                    "kernel": KERNEL_FAMILY.get(str_["kernel"]),
                    "avg_launch_us": str_["recursion_ms"] * 1e3 / str_["step_launches"],
                    "dtype": "f32+i16-residual-storage/f64-arithmetic",
                    "speedup_vs_fp64_plain": (str_["state_col_steps"] / dtr) / plain,
                    "speedup_vs_fp64_batched": (str_["state_col_steps"] / dtr) / batched}

    # accuracy of both reduced-storage forms against float64, all S^z >= 0 sectors
    allsec = W.sectors(W.ring(24))
    mu64, ab64 = kpm.chebyshev_moments(allsec, M, 10, "complex_gaussian", "fp64", 0.025, 0, col_block=20)
    Th = T.cpu().numpy()
    curves = {"T": Th.tolist()}
    for form in ("fp32", "fp32r"):
        mu_f, ab_f = kpm.chebyshev_moments(allsec, M, 10, "complex_gaussian", form, 0.025, 0, col_block=20)
        acc = _accuracy(kpm, np, allsec, T, Th, mu64, ab64, mu_f, ab_f, curves if form == "fp32" else None)
        if form == "fp32":
            out["accuracy_fp32_vs_fp64_all_sectors"] = acc
        else:
            out["fp32r"]["accuracy_vs_fp64_all_sectors"] = acc
    acc = out["accuracy_fp32_vs_fp64_all_sectors"]
    accr = out["fp32r"]["accuracy_vs_fp64_all_sectors"]
    # the speedup holds where the reduced-storage form meets C(T), chi(T) error
    # <= 1e-6 (peak-normalised) against float64: the temperature band, per kernel g_n
    out["speedup_at_error_1e-6"] = {
        "speedup_vs_fp64_plain": out["speedup_vs_fp64_plain"],
        "T_grid": [float(Th[0]), float(Th[-1])],
        **{f"{kern}_{qn}_valid_for_T>=": acc[kern][f"{qn}_lowest_T_with_err<=1e-6"]
           for kern in ("jackson", "none") for qn in ("C", "chi")},
        "fp32r": {"speedup_vs_fp64_plain": out["fp32r"]["speedup_vs_fp64_plain"],
                  **{f"{kern}_{qn}_valid_for_T>=": accr[kern][f"{qn}_lowest_T_with_err<=1e-6"]
                     for kern in ("jackson", "none") for qn in ("C", "chi")}}}
    if args.accuracy_curve:
        # conditioning of C(T) in the moments, from the thermodynamics VJP at
        # one temperature at a time: kappa(T) = sum_{p,n} |dC/dmu_pn| mu_p0 / |C|
        one, zero = np.ones((1, 1)), np.zeros((1, 1))
        for kern in ("jackson", "none"):
            C64 = kpm.thermo(mu64, ab64, allsec, T, kern)["C"].cpu().numpy()[0]
            kap = []
            for i in range(Th.size):
                lam = kpm.thermo_vjp(mu64, ab64, allsec, Th[i:i + 1], one, zero, kern)
                kap.append(float((lam.abs() * mu64[:, :1]).sum()) / abs(float(C64[i])))
            curves[f"{kern}_C_condition"] = kap
        with open(args.accuracy_curve, "w") as f:
            json.dump({"workload": "ring N=24, all S^z >= 0 sectors, 10 complex Gaussian vectors, M=%d" % M,
                       **curves, **{k: v for k, v in acc.items() if k != "moments_max_abs_err_over_mu0"},
                       "moments_max_abs_err_over_mu0": acc["moments_max_abs_err_over_mu0"]}, f)

    return out


_CPU = {}


def _cpu_worker(cols):
    """Recursion of a subset of the columns (forked worker; one BLAS thread)."""
    from threadpoolctl import threadpool_limits

    import numpy as np
    from oracle import moments
    with threadpool_limits(1):
        moments.chebyshev_dots(_CPU["Ht"], _CPU["V0"][:, cols], _CPU["K"], store=np.float32)
    return len(cols)


def cpu_baseline(args, W, np, sec):
    """The oracle's float32-storage recursion on the benchmark's sector and
    columns for a bounded number of steps: on one core, and on the host's
    cores (up to 16) with the columns split over forked processes."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from oracle import hamiltonian, moments, rng

    s = sec[0]
    H = hamiltonian.sector_hamiltonian(s.cluster, s.n_up)
    lo, hi = -11.0, 7.0          # encloses the ring's spectrum (E_0 = -10.77, E_max = 6)
    a, b = hamiltonian.scale_from_bounds(lo, hi, 0.025)
    Ht = hamiltonian.rescaled(H, a, b)
    V0, _, _ = rng.random_columns("complex_gaussian", 0, 0, s.n_up, 10, H.shape[0])
    K = args.cpu_steps
    work = H.shape[0] * V0.shape[1] * K
    with threadpool_limits(1):
        t0 = time.perf_counter()
        moments.chebyshev_dots(Ht, V0, K, store=np.float32)
        dt1 = time.perf_counter() - t0
    # one process per column group, up to the 16 host cores a one-GPU share
    # of the machine holds (whatever the host reports in total)
    nproc = os.cpu_count() or 1
    P = max(1, min(16, nproc, V0.shape[1]))
    _CPU.update(Ht=Ht, V0=V0, K=K)
    groups = [list(g) for g in np.array_split(np.arange(V0.shape[1]), P)]
    with mp.get_context("fork").Pool(P) as pool:
        t0 = time.perf_counter()
        pool.map(_cpu_worker, groups)
        dtp = time.perf_counter() - t0
    _CPU.clear()
    sample = (f"oracle float32-storage recursion, N=24 S^z=0 sector, 20 real columns, {K} steps "
              f"(matrix build excluded)")
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": work / dtp, "unit": "state-column-steps/s", "cores": P, "kind": "oracle",
            "sample": f"{sample}: columns split over {P} forked processes, {dtp:.1f} s",
            "host_nproc": nproc, "cpu_model": model,
            "threads_per_process": {"OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"),
                                    "OPENBLAS_NUM_THREADS": os.environ.get("OPENBLAS_NUM_THREADS"),
                                    "blas_limit": 1},
            "single_core": {"value": work / dt1, "cores": 1, "seconds": dt1}}

if __name__ == "__main__":
    main()
