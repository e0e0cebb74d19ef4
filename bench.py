"""Benchmark of the FLD radiation-energy update on one MI355X.

A step is one whole split step: opacity law, flux-limited diffusion solve to
a relative residual of 1e-8, and the exchange quartic, all on the GPU
through the C ABI, with inputs resident in HBM before the timed region.

The headline (`value`) is the 2D 1024^2 Kramers/log-normal workload with
plain FP64 multigrid, timed over --steps steps after --warmup.  The same
line carries the metric's comparison on that workload (FP32 V-cycles in FP64
refinement, the learned guess with either precision), the dominant kernel's
roofline (HIP events the kernel's own launches record over the timed
region), and under `configs` the 3D 256^3 stratified workload (its first
12 steps: FP64 / FP32 refinement / both inside flexible CG / learned guess,
each step's error bound against the exact solve from its FP64 residual, and
the explicit-source kernel's roofline) and the 96 batched 2D grids (20
steps).  `cpu_baseline` is the FP64 oracle on the host's cores, timed
on a bounded sample before the GPU is touched.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = ("FLD cell-updates/s at rel. residual 1e-8, learned+FP32-MG vs "
          "plain FP64 MG")


# V-cycle of the 2D workloads: V(1,1) on the finest level, V(3,3) on the
# coarse ones.  The coarse levels are latency-bound, so three sweeps there
# cost little; with them the 1024^2 workload needs 5.05 cycles per step
# whatever the finest level's counts (V(1,1) to V(3,3)), and V(1,1) makes
# the finest passes cheapest (6% less time per step than V(2,3) with the same
# coarse levels; V(2,3) everywhere needed 5.15 cycles, V(2,2) everywhere
# 5.85).  The library's default stays V(2,2) everywhere.
PRE, POST = 1, 1
COARSE_PRE, COARSE_POST = 3, 3
# V-cycles of the 3D workload: V(2,2) on the finest level (two fused
# one-launch sweeps each side) and more sweeps on the coarse levels, whose
# rediscretised operators are the weak part on the stratified 256^3 medium
# (face alpha spanning ~8 decades).  Over the first 12 steps, plain V-cycles
# (FP64, or FP32 in FP64 refinement) do best with coarse V(5,5): FP64 15.5
# ms per step against 16.0 with V(4,4), 15.7 with V(6,6), 20.6 with V(3,3);
# as flexible-CG preconditioners they do best with coarse V(4,4) and two
# FP32 V-cycles per iteration (11.6 ms against 12.1 with V(5,5), 13.1 with
# V(3,3); one V-cycle per iteration 12.6-13.5).
PRE3, POST3 = 2, 2
COARSE3, COARSE_KRYLOV3 = 5, 4
COARSE_PRE3, COARSE_POST3 = COARSE3, COARSE3

# Steps of the batched config (its own count), and of the 3D one.  Its 50
# configured steps are out of reach of plain V-cycles: from about the 18th
# step on the stratified medium's thin top mixes free-streaming and
# diffusive cells (face coefficients ~4 next to ~1e6) and the V-cycles stop
# converging; flexible CG around them runs all 50 (FP64 V-cycles, or FP32
# ones that give way to FP64 where they stall).  The comparison of every
# variant covers the first 12 steps; the configured 50-step run covers the
# flexible-CG variants.
C3_STEPS, C3_CONFIG_STEPS, C4_STEPS, AMR_STEPS = 12, 50, 20, 10


def measured_traffic(kernel, shape, nu=None):
    """HBM bytes per launch of `kernel` in tile shape `shape` (and, when the
    record states it, smoothing sweep count `nu`), or None.

    profiles/*.md carry `traffic_record:` lines, one per tile shape, written
    from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE, scaled by a
    plain-copy calibration) together with the hash of the kernel source they
    were taken on; a changed source makes the record stale and the figure
    null, and so does a shape with no record.
    """
    import glob
    import hashlib
    shape = shape.replace(" ", "_")
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic_record:"):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            if kv.get("kernel") != kernel or kv.get("shape") != shape:
                continue
            if nu is not None and "nu" in kv and int(kv["nu"]) != nu:
                continue
            src = os.path.join(ROOT, kv["source"])
            sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
            if sha != kv["sha256_16"]:
                return None
            return float(kv["bytes_per_launch"])
    return None


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle, timed before the GPU is initialised
# ---------------------------------------------------------------------------

def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_steps(workload, n, steps, rtol):
    """Worker: `steps` oracle split steps of a seeded workload; returns
    (seconds, cells).  Runs in a fresh process (no GPU), one thread: the
    math libraries are held to one thread before numpy is first imported."""
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    import media
    from oracle import fldref as F
    m = media.config_c2(n=n) if workload == "c2" else media.config_c3(n=n)
    prob = F.problem_from_medium(m)
    E, e = m.E, m.e
    t0 = time.perf_counter()
    for _ in range(steps):
        E, e, _ = F.step(E, e, m.rho, prob, m.dt, opacity=m.opacity, rtol=rtol)
    return time.perf_counter() - t0, m.cells


def cpu_baseline(steps_c2=2, n3=128):
    """The oracle (numpy/scipy FP64, exact solve by Jacobi-preconditioned CG
    to the benchmark's relative residual 1e-8, then the exchange) on the
    headline workload, single-threaded over `steps_c2` steps, and on every
    usable core at once (one independent step of the same medium per worker
    process: the aggregate rate of the host), plus one step of the 3D
    workload's statistics at n3^3.  Worker processes are started before
    this process touches the GPU."""
    import concurrent.futures as cf
    import multiprocessing as mp
    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(cores, 16))
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        secs, cells = ex.submit(_oracle_steps, "c2", 1024, steps_c2, 1e-8).result()
        t0 = time.perf_counter()
        futs = [ex.submit(_oracle_steps, "c2", 1024, 1, 1e-8)
                for _ in range(workers)]
        for f in futs:
            f.result()
        wall = time.perf_counter() - t0
        s3, c3 = ex.submit(_oracle_steps, "c3", n3, 1, 1e-8).result()
    return {
        "value": cells * steps_c2 / secs, "unit": "cell-updates/s", "cores": 1,
        "kind": "oracle",
        "sample": f"{steps_c2} split steps of the 1024x1024 workload (opacity, "
                  f"Jacobi-PCG to rel. residual 1e-8, exchange), {secs:.1f} s, "
                  f"one thread of numpy/scipy (the oracle is single-threaded); "
                  f"its 100 configured steps extrapolate linearly per step",
        "all_cores": {"value": workers * cells / wall, "workers": workers,
                      "seconds": wall,
                      "sample": f"{workers} worker processes, one independent "
                                f"split step of the same medium each"},
        "c3_sample": {"value": c3 / s3, "cells": c3, "seconds": s3,
                      "sample": f"1 split step of the 3D workload's statistics "
                                f"at {n3}^3, one thread"},
        "nproc": os.cpu_count(), "usable_cores": cores,
        "cpu_model": _cpu_model(), "threads": 1,
    }


# ---------------------------------------------------------------------------
# Byte models and rooflines
# ---------------------------------------------------------------------------

def step_model_bytes(ndim, precision, vcycles, pre, post, cpre, cpost,
                     outer=0.0, inner=2, krylov=False):
    """Per-pass byte model of one split step per fine cell, at the V-cycle
    actually run: every pass streams its operands once (w = 8 FP64, 4 FP32),
    each smoothing sweep reads b, the d face arrays and the iterate and
    writes it ((3 + d) w), the residual + restriction reads (2 + d) w and
    writes 2 w and the prolongation 2 w / 2^d, with the finest level's sweep
    counts (pre, post) and the coarse levels' (cpre, cpost), the coarse
    levels holding 1/3 (2D) or 1/7 (3D) of the cells.  Fixed per step:
    coefficients (3 + d) 8 (+ 4 d for the FP32 copies), hierarchy
    d w (2g - 1) (g = 4/3, 8/7), copy of E^n 16, exchange 48.  FP32
    refinement adds per outer iteration the FP64 residual (2 + d) 8 + 4 and
    the correction 20.  Flexible CG (krylov; `outer` its iterations,
    `vcycles` all V-cycles, FP32 widths in FP32_IR) adds its initial
    residual (2 + d) 8 + 8 (+ 4) once and per iteration (z, q) w + 8, the
    direction and q = A p w + (4 + d) 8, and the update 48 (+ 4)."""
    d = ndim
    gsum = {1: 1.0, 2: 1.0 / 3.0, 3: 1.0 / 7.0}[d]
    g = 1.0 + gsum

    def cycle(w):
        def level(nu):
            return nu * (3 + d) * w + (2 + d) * w + 2 * w + 2 * w / 2 ** d
        return level(pre + post) + gsum * level(cpre + cpost)

    if krylov:
        w = 8 if precision == "fp64" else 4
        x = 0 if precision == "fp64" else 4
        base = (3 + d) * 8 + (4 * d if x else 0) + d * w * (2 * g - 1) + 16 + 48
        base += (2 + d) * 8 + 8 + x
        per_iter = (w + 8) + (w + (4 + d) * 8) + 48 + x
        return base + outer * per_iter + vcycles * cycle(w)
    if precision == "fp64":
        base = (3 + d) * 8 + d * 8 * (2 * g - 1) + 16 + 48
        return base + vcycles * cycle(8)
    base = (3 + d) * 8 + 4 * d + d * 4 * (2 * g - 1) + 16 + 48
    return base + outer * ((2 + d) * 8 + 4 + 20 + inner * cycle(4))


def step_model_roofline(bytes_per_cell, value, cycle):
    gbs = bytes_per_cell * value / 1e9
    return {"bytes_per_cell_step": bytes_per_cell, "cycle": cycle,
            "model": "per-pass streaming byte model at the cycle run",
            "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS}


def _hbm_roofline(kt, shape):
    """Roofline entry of a kernel timed with fld_kernel_timing (algorithmic
    bytes per launch over its mean launch duration, against HBM peak)."""
    if not kt["launches"]:
        return None
    avg_ms = kt["ms"] / kt["launches"]
    per_launch = kt["bytes"] / kt["launches"]
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kt["kernel"], "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(kt["kernel"], shape),
            "avg_launch_us": avg_ms * 1e3,
            "algorithmic_bytes_per_launch": per_launch,
            "launches": kt["launches"]}


def copy_bandwidth(reps=10):
    """Achievable HBM bandwidth: a plain 1 GiB device-to-device copy (read +
    write bytes over the mean time per copy, torch events on the stream the
    copies run on)."""
    import torch
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "bytes_per_copy": 2 * n * 8}


def _bound_factor(E):
    """sqrt(N) |b| / sum(b): rel-L2 error <= rel-residual x this factor (A
    has eigenvalues >= 1 and unit column sums)."""
    b = E.reshape(-1)
    return float(b.numel() ** 0.5 * b.norm() / b.sum())


# ---------------------------------------------------------------------------
# The headline: 2D 1024^2
# ---------------------------------------------------------------------------

def run_c2(args, weights):
    import numpy as np
    import torch
    import media
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import Stepper, make_params
    m = media.config_c2(n=args.n)
    dev = torch.device("cuda:0")

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    def run(precision, steps, warmup, timed_kernel=True, weights=None,
            policy="adaptive"):
        """warmup + timed steps of one solver variant from the initial state"""
        params = make_params(m.ndim, m.n[:2], m.dx[:2], m.bc, rtol=1e-8,
                             precision=precision, pre_smooth=PRE, post_smooth=POST,
                             coarse_pre_smooth=COARSE_PRE,
                             coarse_post_smooth=COARSE_POST,
                             guess="prev" if weights is None else "learned",
                             guess_policy=policy)
        st = Stepper(params, opacity=m.opacity)
        shapes = fld.fld_autotune(st.ctx)[:6] if not args.no_autotune else None
        if weights is not None:
            fld.fld_set_model(st.ctx, weights)
        rho, E, e = d(m.rho), d(m.E), d(m.e)
        kap = torch.empty_like(rho)
        for _ in range(warmup):
            st.step(m.dt, rho, kap, E, e)
        torch.cuda.synchronize()
        fld.fld_kernel_timing_enable(st.ctx, timed_kernel)
        fld.fld_kernel_timing_read(st.ctx)  # reset
        cycles, outer, res, rej, skip = [], [], [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s = st.step(m.dt, rho, kap, E, e)
            cycles.append(s["cycles"])
            outer.append(s["outer_iters"])
            res.append(s["rel_res_final"])
            rej.append(s["guess_rejected"])
            skip.append(s["guess_skipped"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kt = fld.fld_kernel_timing_read(st.ctx)
        fld.fld_kernel_timing_enable(st.ctx, False)
        secs = t1 - t0
        return dict(value=m.cells * steps / secs, ms_per_step=secs * 1e3 / steps,
                    vcycles_per_step=float(np.mean(cycles)),
                    outer_per_step=float(np.mean(outer)),
                    rel_res_final_max=float(np.max(res)), kernel=kt,
                    rejected=int(np.sum(rej)), skipped=int(np.sum(skip)),
                    tile_shapes=shapes,
                    E=E.cpu().numpy(), bound_factor=_bound_factor(E))

    base = run("fp64", args.steps, args.warmup)
    if args.headline_only:
        kt = base["kernel"]
        print(json.dumps({"ms_per_step": base["ms_per_step"],
                          "vcycles_per_step": base["vcycles_per_step"],
                          "finest_down_us": 1e3 * kt["ms"] / max(kt["launches"], 1),
                          "tile_shapes": base["tile_shapes"]}))
        return None
    # only the headline run's kernel is priced against the roofline; the
    # variants run without per-launch timing events
    mixed = run("fp32_ir", args.steps, args.warmup, timed_kernel=False)
    lrn64 = run("fp64", args.steps, args.warmup, timed_kernel=False, weights=weights)
    lrn32 = run("fp32_ir", args.steps, args.warmup, timed_kernel=False, weights=weights)
    # the network evaluated on every step, whatever it saves
    lrn32e = run("fp32_ir", args.steps, args.warmup, timed_kernel=False,
                 weights=weights, policy="every_step")
    # network inference alone on the same grid
    net = fld.fldnn_create(1, m.n[1], m.n[0], training=False)
    fld.fldnn_set_params(net, weights)
    xin = torch.zeros(m.cells * 4, dtype=torch.float32, device=dev)
    dout = torch.empty(m.cells, dtype=torch.float32, device=dev)
    for _ in range(3):
        fld.fldnn_forward(net, xin, dout)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        fld.fldnn_forward(net, xin, dout)
    torch.cuda.synchronize()
    unet_ms = (time.perf_counter() - t0) * 100.0
    del net
    from paper_2503_02764_amd.train_guess import forward_flops
    unet_flops = forward_flops(m.n[1], m.n[0])
    kt = base["kernel"]
    if base["tile_shapes"]:
        level0_down = base["tile_shapes"][0][0]
    else:  # the library's fixed shape (0 unless FLD_TILE_VARIANT names one)
        v = int(os.environ.get("FLD_TILE_VARIANT", "0"))
        level0_down = fld.load().fld_tile_shape_name(
            v if 0 <= v < 7 else 0).decode()
    avg_ms = kt["ms"] / max(kt["launches"], 1)
    bytes_per_launch = kt["bytes"] / max(kt["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    diff = float(np.linalg.norm(mixed["E"] - base["E"]) /
                 np.linalg.norm(base["E"]))
    cyc = f"V({PRE},{POST}), coarse V({COARSE_PRE},{COARSE_POST})"

    def model(r, precision):
        return step_model_roofline(step_model_bytes(
            2, precision, r["vcycles_per_step"], PRE, POST, COARSE_PRE,
            COARSE_POST, r["outer_per_step"], 2), r["value"], cyc)

    def variant(r, precision, learned=False):
        out = {"value": r["value"], "ms_per_step": r["ms_per_step"],
               "vcycles_per_step": r["vcycles_per_step"],
               "outer_per_step": r["outer_per_step"],
               "rel_res_final_max": r["rel_res_final_max"],
               "error_bound_max": r["rel_res_final_max"] * r["bound_factor"],
               "speedup_vs_fp64": r["value"] / base["value"],
               "step_model_roofline": model(r, precision)}
        if learned:
            out["network_steps"] = args.steps - r["skipped"]
            out["guess_rejected_steps"] = r["rejected"]
        return out

    out = {
        "metric": METRIC,
        "value": base["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": base["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"2d-{m.n[0]}x{m.n[1]}-kramers-lognormal-fp64-plain-mg",
            "grid": [m.n[0], m.n[1]],
            "bc": "neumann",
            "rtol": 1e-8,
            "cycle": cyc,
            "precision": "fp64",
            "guess": "prev",
            "dt": m.dt,
        },
        "vcycles_per_step": base["vcycles_per_step"],
        "rel_res_final_max": base["rel_res_final_max"],
        "error_bound_max": base["rel_res_final_max"] * base["bound_factor"],
        "learned_fp32_vs_plain_fp64": lrn32["value"] / base["value"],
        "tile_shapes_autotuned": base["tile_shapes"],
        "variants": {
            "fp32_vcycles_fp64_refinement": dict(
                variant(mixed, "fp32_ir"), rel_l2_vs_fp64_after_steps=diff),
            "learned_guess_fp64": variant(lrn64, "fp64", True),
            "learned_guess_fp32_vcycles_fp64_refinement":
                variant(lrn32, "fp32_ir", True),
            "learned_guess_every_step_fp32_vcycles_fp64_refinement":
                variant(lrn32e, "fp32_ir", True),
            "unet_forward_ms": unet_ms,
            "unet_forward": {
                "gflop_executed": unet_flops / 1e9,
                "gflop_useful": forward_flops(m.n[1], m.n[0], False) / 1e9,
                "tflops": unet_flops / (unet_ms * 1e-3) / 1e12,
                "frac_of_bf16_peak": unet_flops / (unet_ms * 1e-3) / 2.5e15},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kt["kernel"],
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(kt["kernel"], level0_down, PRE),
            "tile_shape": level0_down,
            "avg_launch_us": avg_ms * 1e3,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "launches": kt["launches"],
        },
        "step_model_roofline": model(base, "fp64"),
    }
    return out


# ---------------------------------------------------------------------------
# 3D 256^3 stratified medium
# ---------------------------------------------------------------------------

def run_c3(steps, warmup, weights, config_run=True):
    """The 3D workload in two parts.  First every variant over `steps`
    steps after `warmup` (from the initial state): plain FP64 V-cycles, FP32
    V-cycles in FP64 refinement, both inside flexible CG, and FP32
    refinement with the learned guess applied per z-slice (adaptive policy,
    and on every step).  Then (config_run) the configured 50 steps from the
    initial state with the flexible-CG variants, the only ones that last
    them.  Every step's error against its exact solve is bounded by its
    FP64 relative residual x sqrt(N)|b|/sum(b) (the GPU tests check, on the
    same workload, that the oracle's own residual of the iterate agrees
    with the GPU's)."""
    import numpy as np
    import torch
    import media
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import Stepper, make_params
    m = media.config_c3()

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()

    def run(precision, weights=None, policy="adaptive", krylov=False,
            nsteps=steps, nwarm=warmup):
        coarse = COARSE_KRYLOV3 if krylov else COARSE3
        cyc = f"V({PRE3},{POST3}), coarse V({coarse},{coarse})"
        params = make_params(3, m.n, m.dx, m.bc, rtol=1e-8, precision=precision,
                             guess="prev" if weights is None else "learned",
                             guess_policy=policy, krylov=krylov,
                             max_cycles=400, pre_smooth=PRE3,
                             post_smooth=POST3, coarse_pre_smooth=coarse,
                             coarse_post_smooth=coarse)
        st = Stepper(params, opacity=m.opacity)
        if weights is not None:
            fld.fld_set_model(st.ctx, weights)
        rho, E, e = d(m.rho), d(m.E), d(m.e)
        kap = torch.empty_like(rho)
        for _ in range(nwarm):
            st.step(m.dt, rho, kap, E, e)
        torch.cuda.synchronize()
        f0 = _bound_factor(E)
        # the first fused finest-level sweep of every V-cycle records its own
        # duration (HIP events the launch records)
        fld.fld_kernel_timing_enable(st.ctx, True)
        fld.fld_kernel_timing_read(st.ctx)  # reset
        cyc_n, outer, res, rej, skip, pre64 = [], [], [], [], [], []
        t0 = time.perf_counter()
        for _ in range(nsteps):
            s = st.step(m.dt, rho, kap, E, e)
            cyc_n.append(s["cycles"])
            outer.append(s["outer_iters"])
            res.append(s["rel_res_final"])
            rej.append(s["guess_rejected"])
            skip.append(s["guess_skipped"])
            pre64.append(s["precond_fp64"])
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        kt = fld.fld_kernel_timing_read(st.ctx)
        fld.fld_kernel_timing_enable(st.ctx, False)
        factor = max(f0, _bound_factor(E))
        value = m.cells * nsteps / secs
        r = dict(value=value, ms_per_step=secs * 1e3 / nsteps, cycle=cyc,
                 vcycles_per_step=float(np.mean(cyc_n)),
                 outer_per_step=float(np.mean(outer)),
                 rel_res_final_max=float(np.max(res)),
                 bound_factor=factor,
                 error_bound_max=float(np.max(res)) * factor,
                 roofline=_hbm_roofline(kt, "256^3"))
        if nsteps <= 16:
            r["error_bound_per_step"] = [float(x) * factor for x in res]
        else:
            r["iterations_per_step"] = [int(x) for x in
                                        (outer if krylov or precision != "fp64"
                                         else cyc_n)]
        if krylov and precision == "fp32_ir":
            r["steps_with_fp64_vcycles"] = int(np.sum(pre64))
        r["step_model_roofline"] = step_model_roofline(step_model_bytes(
            3, precision, r["vcycles_per_step"], PRE3, POST3, coarse, coarse,
            r["outer_per_step"], 2, krylov), value, cyc)
        if weights is not None:
            r["network_steps"] = nsteps - int(np.sum(skip))
            r["guess_rejected_steps"] = int(np.sum(rej))
        E_out = E.cpu().numpy()
        del st, rho, E, e, kap
        torch.cuda.empty_cache()
        return r, E_out

    explicit = _explicit_roofline(m)
    f64, E64 = run("fp64")
    f32, E32 = run("fp32_ir")
    k64, _ = run("fp64", krylov=True)
    k32, _ = run("fp32_ir", krylov=True)
    lrn, _ = run("fp32_ir", weights)
    lrnk, _ = run("fp32_ir", weights, krylov=True)
    lrne, _ = run("fp32_ir", weights, policy="every_step")
    f32["rel_l2_vs_fp64_after_steps"] = float(
        np.linalg.norm(E32 - E64) / np.linalg.norm(E64))
    for r in (f32, k64, k32, lrn, lrnk, lrne):
        r["speedup_vs_fp64"] = r["value"] / f64["value"]
    out = {
        "workload": "3d-256cube-stratified-kramers",
        "grid": list(m.n), "bc": list(m.bc), "rtol": 1e-8,
        "cycle": f"V({PRE3},{POST3}), coarse V({COARSE3},{COARSE3}); as "
                 f"flexible-CG preconditioner coarse V({COARSE_KRYLOV3},"
                 f"{COARSE_KRYLOV3})",
        "steps": steps, "warmup": warmup, "dt": m.dt,
        "config_steps": C3_CONFIG_STEPS,
        "steps_note": f"every variant over steps {warmup + 1}-"
                      f"{warmup + steps}; plain V-cycles stop converging "
                      f"from about the 18th step on this medium, flexible CG "
                      f"runs the configured {C3_CONFIG_STEPS} (config_run)",
        "value": f32["value"], "ms_per_step": f32["ms_per_step"],
        "dtype": "f32 V-cycles, f64 refinement and exchange",
        "learned_fp32_vs_plain_fp64": lrn["value"] / f64["value"],
        "learned_fp32_krylov_vs_plain_fp64": lrnk["value"] / f64["value"],
        "roofline": f32["roofline"],
        "explicit_sources": explicit,
        "variants": {"fp64_plain_mg": f64, "fp32_vcycles_fp64_refinement": f32,
                     "fp64_vcycles_in_flexible_cg": k64,
                     "fp32_vcycles_in_fp64_flexible_cg": k32,
                     "learned_guess_fp32_vcycles_fp64_refinement": lrn,
                     "learned_guess_fp32_vcycles_in_fp64_flexible_cg": lrnk,
                     "learned_guess_every_step_fp32_vcycles_fp64_refinement":
                         lrne},
    }
    if config_run:
        n = C3_CONFIG_STEPS
        c64, _ = run("fp64", krylov=True, nsteps=n, nwarm=0)
        c32, _ = run("fp32_ir", krylov=True, nsteps=n, nwarm=0)
        cl, _ = run("fp32_ir", weights, krylov=True, nsteps=n, nwarm=0)
        for r in (c32, cl):
            r["speedup_vs_fp64_flexible_cg"] = r["value"] / c64["value"]
        out["config_run"] = {
            "steps": n, "warmup": 0,
            "note": "the configured steps from the initial state; plain "
                    "V-cycles (FP64 or FP32 refinement) diverge before the "
                    "end, so the FP64 reference here is flexible CG over "
                    "FP64 V-cycles",
            "learned_fp32_vs_fp64": cl["value"] / c64["value"],
            "variants": {"fp64_vcycles_in_flexible_cg": c64,
                         "fp32_vcycles_in_fp64_flexible_cg": c32,
                         "learned_guess_fp32_vcycles_in_fp64_flexible_cg": cl},
        }
        # the configured workload: its 50 steps, FP32 V-cycles in FP64
        # iterations
        out.update(value=c32["value"], ms_per_step=c32["ms_per_step"],
                   roofline=c32["roofline"],
                   value_from="config_run fp32_vcycles_in_fp64_flexible_cg")
    else:
        out["value_from"] = "variants fp32_vcycles_fp64_refinement"
    return out


def _explicit_roofline(m, reps=10):
    """fld_explicit_sources on the 256^3 medium with a seeded velocity field,
    all outputs: algorithmic bytes (E, rho, kappa, 3 velocity components
    read; 3 force components, work, tiring, Eddington factor written: 96 B
    per cell) over the mean time per launch (torch events on the context's
    stream, which is torch's current stream here)."""
    import numpy as np
    import torch
    import media
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import make_params
    ctx = fld.fld_setup(make_params(3, m.n, m.dx, m.bc))
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    rho, E = d(m.rho), d(m.E)
    kap = torch.full_like(rho, 1.0)
    o = m.opacity
    fld.fld_opacity_powerlaw(ctx, rho, d(m.e), o["k0"], o["a"], o["b"],
                             o["kmin"], o["kmax"], kap)
    v = [d(c) for c in media.velocity_field(m.E.shape, 3, seed=31, ell=8.0)]
    outs = [torch.empty_like(rho) for _ in range(6)]
    args = (ctx, rho, kap, E, v, outs[:3], outs[3], outs[4], outs[5])
    fld.fld_explicit_sources(*args)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fld.fld_explicit_sources(*args)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    nbytes = 96.0 * m.cells
    gbs = nbytes / (us * 1e-6) / 1e9
    del ctx, outs, v
    torch.cuda.empty_cache()
    return {"bound": "hbm", "kernel": "k_explicit_3d<true>", "achieved": gbs,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": measured_traffic("k_explicit_3d<true>", "256^3"),
            "avg_launch_us": us,
            "algorithmic_bytes_per_launch": nbytes, "launches": reps}


# ---------------------------------------------------------------------------
# 96 batched 2D grids
# ---------------------------------------------------------------------------

def run_c4(steps, warmup):
    """96 independent 2D grids (sides 128..1024) in one batched context:
    FP32 V-cycles in FP64 refinement, one launch per phase, hipGraph
    replay, autotuned tiles; against the same grids stepped one by one with
    single-grid contexts (same precision, and plain FP64).  The learned
    guess is not offered for batches."""
    import numpy as np
    import torch
    import media
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import Stepper, make_params
    ms = media.config_c4()
    o = ms[0].opacity
    cells = sum(m.cells for m in ms)
    cyc = f"V({PRE},{POST}), coarse V({COARSE_PRE},{COARSE_POST})"

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()

    def fields():
        rho = [d(m.rho) for m in ms]
        return rho, [d(m.E) for m in ms], [d(m.e) for m in ms], \
            [torch.empty_like(r) for r in rho]

    dts = [m.dt for m in ms]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        params = [make_params(2, m.n[:2], m.dx[:2], m.bc, rtol=1e-8,
                              precision="fp32_ir", pre_smooth=PRE,
                              coarse_pre_smooth=COARSE_PRE,
                              coarse_post_smooth=COARSE_POST,
                              post_smooth=POST) for m in ms]
        bctx = fld.fld_setup_batch(params, stream=stream)
        fld.fld_batch_set_graph(bctx, True)
        shapes = fld.fld_autotune(bctx)[:6]
        rho, E, e, kap = fields()
        res = []

        def step():
            fld.fld_opacity_powerlaw_batch(bctx, rho, e, o["k0"], o["a"],
                                           o["b"], o["kmin"], o["kmax"], kap)
            _, s = fld.fld_step_batch(bctx, dts, rho, kap, E, E)
            fld.fld_exchange_batch(bctx, dts, rho, kap, E, e)
            return s

        for _ in range(warmup):
            step()
        stream.synchronize()
        factor0 = max(_bound_factor(x) for x in E)
        outer = []
        t0 = time.perf_counter()
        for _ in range(steps):
            s = step()
            res.append(max(x["rel_res_final"] for x in s))
            outer.append(float(np.mean([x["outer_iters"] for x in s])))
        stream.synchronize()
        secs = time.perf_counter() - t0
        factor = max(factor0, max(_bound_factor(x) for x in E))
        E_batch = [x.cpu().numpy() for x in E]
        # the dominant kernel, the finest-level down pass over all grids:
        # its launch records its own events, which a graph replay cannot,
        # so it is timed on 3 more steps without the graph (the first down
        # pass of each step, while every grid is running)
        fld.fld_batch_set_graph(bctx, False)
        fld.fld_kernel_timing_enable(bctx, True)
        fld.fld_kernel_timing_read(bctx)
        for _ in range(3):
            step()
        stream.synchronize()
        kt = fld.fld_kernel_timing_read(bctx)
        fld.fld_kernel_timing_enable(bctx, False)
    value = cells * steps / secs
    batch = dict(value=value, ms_per_step=secs * 1e3 / steps,
                 tile_shapes_autotuned=shapes,
                 outer_per_step=float(np.mean(outer)),
                 rel_res_final_max=float(np.max(res)), bound_factor=factor,
                 error_bound_per_step=[r * factor for r in res])
    del bctx, rho, E, e, kap
    torch.cuda.empty_cache()

    def one_by_one(precision):
        sts = []
        for m in ms:
            st = Stepper(make_params(2, m.n[:2], m.dx[:2], m.bc, rtol=1e-8,
                                     precision=precision, pre_smooth=PRE,
                                     coarse_pre_smooth=COARSE_PRE,
                                     coarse_post_smooth=COARSE_POST,
                                     post_smooth=POST), opacity=m.opacity)
            fld.fld_autotune(st.ctx)
            sts.append(st)
        rho, E, e, kap = fields()
        for _ in range(warmup):
            for g, st in enumerate(sts):
                st.step(dts[g], rho[g], kap[g], E[g], e[g])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for g, st in enumerate(sts):
                st.step(dts[g], rho[g], kap[g], E[g], e[g])
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        out = [x.cpu().numpy() for x in E]
        del sts, rho, E, e, kap
        torch.cuda.empty_cache()
        return dict(value=cells * steps / secs, ms_per_step=secs * 1e3 / steps), out

    seq32, _ = one_by_one("fp32_ir")
    seq64, E64 = one_by_one("fp64")
    diff = max(float(np.linalg.norm(a - b) / np.linalg.norm(b))
               for a, b in zip(E_batch, E64))
    batch["speedup_vs_one_by_one_fp32"] = batch["value"] / seq32["value"]
    batch["speedup_vs_one_by_one_fp64"] = batch["value"] / seq64["value"]
    batch["max_rel_l2_vs_fp64_after_steps"] = diff
    # the outer count varies per grid: the model takes the mean
    batch["step_model_roofline"] = step_model_roofline(step_model_bytes(
        2, "fp32_ir", 0.0, PRE, POST, COARSE_PRE, COARSE_POST,
        batch["outer_per_step"], 2), value, cyc)
    return {
        "workload": f"2d-batched-{len(ms)}-grids-{cells}-cells",
        "grids": len(ms), "cells": cells, "rtol": 1e-8, "cycle": cyc,
        "steps": steps, "warmup": warmup,
        "value": value, "ms_per_step": batch["ms_per_step"],
        "dtype": "f32 V-cycles, f64 refinement and exchange",
        "roofline": dict(_hbm_roofline(kt, "batch96") or {},
                         timed="the first finest-level down pass of 3 steps "
                               "after the timed ones, without graph replay"),
        "variants": {"batched_fp32_vcycles_fp64_refinement_graph": batch,
                     "one_by_one_fp32": seq32, "one_by_one_fp64": seq64},
    }


def run_amr(steps, warmup, one_level_only=False):
    """The block-adaptive 2D step: the 1024^2 Kramers / log-normal medium as
    the base grid (16 x 16 blocks), the 1/8 of the blocks with the steepest
    log E refined (fine fields interpolated from the base), FP64 flexible
    CG to rel. residual 1e-8 preconditioned by fine sweeps around a base
    V-cycle; E stepped in place, rho and kappa fixed.  Throughput counts
    leaf cells.  A second variant refines half of the 2:1-eligible patches
    of level 1 again (two refined levels)."""
    import numpy as np
    import torch
    import media
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import make_params

    def leaf_cells(w):
        levels = w["blocks"] if w["blocks"] and isinstance(
            w["blocks"][0][0], (list, tuple)) else [w["blocks"]]
        n, b = w["n"], w["b"]
        cells = n * n - len(levels[0]) * b * b
        for k, bl in enumerate(levels):
            cells += len(bl) * 4 * b * b
            if k + 1 < len(levels):
                cells -= len(levels[k + 1]) * b * b
        return cells, len(levels)

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()

    def one(w, timed_kernel):
        n, b = w["n"], w["b"]
        leaf, nlev = leaf_cells(w)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            p = make_params(2, (n, n), (w["dx"], w["dx"]), w["bc"], rtol=1e-8,
                            pre_smooth=PRE, post_smooth=POST, max_cycles=200)
            ctx = fld.fld_amr_setup(p, b, w["blocks"], stream=stream)
            rb, kb, eb = d(w["rho_b"]), d(w["kappa_b"]), d(w["E_b"])
            rf, kf, ef = d(w["rho_f"]), d(w["kappa_f"]), d(w["E_f"])
            for _ in range(warmup):
                fld.fld_amr_step(ctx, w["dt"], rb, kb, eb, eb, rf, kf, ef, ef)
            stream.synchronize()
            iters, res = [], []
            t0 = time.perf_counter()
            for _ in range(steps):
                _, st = fld.fld_amr_step(ctx, w["dt"], rb, kb, eb, eb, rf, kf,
                                         ef, ef)
                iters.append(st["cycles"])
                res.append(st["rel_res_final"])
            stream.synchronize()
            secs = time.perf_counter() - t0
            kt = None
            if timed_kernel:
                # the kernel's launch time from events, in steps of their own
                # so that the events stay out of the throughput above
                fld.fld_amr_kernel_timing_enable(ctx, True)
                fld.fld_amr_kernel_timing_read(ctx)
                for _ in range(3):
                    fld.fld_amr_step(ctx, w["dt"], rb, kb, eb, eb, rf, kf,
                                     ef, ef)
                kt = fld.fld_amr_kernel_timing_read(ctx)
                fld.fld_amr_kernel_timing_enable(ctx, False)
        del ctx
        torch.cuda.empty_cache()
        return dict(workload=w["name"], refined_levels=nlev,
                    leaf_cells=int(leaf), value=leaf * steps / secs,
                    ms_per_step=secs * 1e3 / steps,
                    iterations_per_step=float(np.mean(iters)),
                    rel_res_final_max=float(np.max(res))), kt

    r1, kt = one(media.config_amr(), True)
    variants = {"one_refined_level": r1}
    if not one_level_only:
        variants["two_refined_levels"], _ = one(media.config_amr(levels=2),
                                                False)
    return {"workload": r1["workload"], "leaf_cells": r1["leaf_cells"],
            "refined_blocks": len(media.config_amr()["blocks"]), "block": 16,
            "rtol": 1e-8, "steps": steps, "warmup": warmup,
            "value": r1["value"], "ms_per_step": r1["ms_per_step"],
            "iterations_per_step": r1["iterations_per_step"],
            "rel_res_final_max": r1["rel_res_final_max"], "dtype": "f64",
            "cycle": f"FCG; a cycle through the levels, RB-GS {PRE}+{POST} on "
                     "each refined level around one base V-cycle",
            "roofline": dict(_hbm_roofline(kt, "amr-1024sq-b16") or {},
                             timed="every level-1 red-black half-sweep "
                                   "of three steps after the timed ones "
                                   "(events recorded by each launch)"),
            "variants": variants}


def _line(metric_value, ms, args, workload, dtype, extra):
    out = {
        "metric": METRIC, "value": metric_value, "unit": "cell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": workload}, "roofline": None,
        "cpu_baseline": None}
    out.update(extra)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default tile shape on every level")
    ap.add_argument("--headline-only", action="store_true",
                    help="run only the headline variant (for profiling)")
    ap.add_argument("--amr-one-level", action="store_true",
                    help="block-adaptive leg: the one-level variant only")
    ap.add_argument("--workload", choices=("all", "c2", "c3", "c4", "amr"),
                    default="all",
                    help="all: the headline line with the 3D and batched "
                         "configs under `configs`; c2 / c3 / c4: one workload "
                         "alone (for profiling)")
    ap.add_argument("--skip-config-run", action="store_true",
                    help="3D workload: leave out the configured 50-step run "
                         "(for profiling)")
    ap.add_argument("--unet-only", action="store_true",
                    help="only run the learned guess's network on a 1024^2 "
                         "image (for profiling its kernels)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if (not args.no_cpu_baseline and not args.headline_only
            and not args.copy_calibration and not args.unet_only
            and args.workload in ("all", "c2")):
        cpu = cpu_baseline()  # before this process touches the GPU

    import torch

    if args.copy_calibration:
        n = 1 << 27  # 1 GiB of float64 read, 1 GiB written
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 8, "launches": 3}))
        return

    torch.cuda.set_device(0)
    from paper_2503_02764_amd.guess import load_weights
    weights = load_weights()
    if args.unet_only:
        from paper_2503_02764_amd import fld
        from paper_2503_02764_amd.train_guess import forward_flops
        n = args.n
        net = fld.fldnn_create(1, n, n, training=False)
        fld.fldnn_set_params(net, weights)
        xin = torch.randn(n * n * 4, dtype=torch.float32, device="cuda")
        dout = torch.empty(n * n, dtype=torch.float32, device="cuda")
        for _ in range(args.warmup):
            fld.fldnn_forward(net, xin, dout)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fld.fldnn_forward(net, xin, dout)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        fl = forward_flops(n, n)
        print(json.dumps({"unet_forward_ms": ms, "n": n,
                          "tflops": fl / (ms * 1e-3) / 1e12}))
        return
    if args.workload == "c3":
        r = run_c3(min(args.steps, C3_STEPS), min(args.warmup, 1), weights,
                   config_run=not args.skip_config_run)
        if "config_run" in r:
            args.steps, args.warmup = r["config_run"]["steps"], 0
        else:
            args.steps, args.warmup = r["steps"], r["warmup"]
        _line(r["value"], r["ms_per_step"], args, r["workload"], "f32",
              {"roofline": r["roofline"], "c3": r,
               "achievable_copy": copy_bandwidth()})
        return
    if args.workload == "amr":
        r = run_amr(min(args.steps, AMR_STEPS), min(args.warmup, 2),
                    one_level_only=args.amr_one_level)
        args.steps, args.warmup = r["steps"], r["warmup"]
        _line(r["value"], r["ms_per_step"], args, r["workload"], "f64",
              {"amr": r})
        return
    if args.workload == "c4":
        r = run_c4(min(args.steps, C4_STEPS), min(args.warmup, 1))
        args.steps, args.warmup = r["steps"], r["warmup"]
        _line(r["value"], r["ms_per_step"], args, r["workload"], "f32",
              {"c4": r})
        return
    out = run_c2(args, weights)
    if out is None:
        return
    if args.workload == "all":
        out["configs"] = {}
        for name, fn in (("c3", lambda: run_c3(C3_STEPS, 1, weights)),
                         ("c4", lambda: run_c4(C4_STEPS, 1)),
                         ("amr", lambda: run_amr(AMR_STEPS, 2))):
            try:
                out["configs"][name] = fn()
            except Exception as exc:  # reported in the line, not hidden
                out["configs"][name] = {"error": f"{type(exc).__name__}: {exc}"}
                import torch
                torch.cuda.synchronize()
                torch.cuda.empty_cache()
    out["achievable_copy"] = copy_bandwidth()
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
