"""Benchmark of the FLD radiation-energy update on one MI355X.

A step is one whole split step on the 2D 1024^2 Kramers/log-normal
workload: opacity law, flux-limited diffusion solve to a relative residual
of 1e-8 (FP64 V-cycles), and the exchange quartic, all on the GPU through
the C ABI.  Inputs are resident in HBM before the timed region.

Prints one JSON line with the throughput (cell-updates/s), the dominant
kernel's roofline figures (HIP events around each of its launches, over the
timed region) and the CPU oracle's rate on a bounded sample.
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
# V-cycle of the 3D workload: V(2,2) on the finest level (two fused
# one-launch sweeps), V(3,3) on the coarse ones.  On the 256^3 stratified
# medium (face alpha spanning ~8 decades) the coarse levels need the extra
# sweeps: 7.2-7.6 V-cycles per step instead of 11.6 with V(2,2) everywhere.
# Against V(1,2) with coarse V(4,4) (one sweep of colour passes and one
# fused pair on the finest level): FP64 12.7 instead of 12.9 ms per step,
# FP32 refinement 10.6 instead of 11.3.
PRE3, POST3 = 2, 2
COARSE_PRE3, COARSE_POST3 = 3, 3


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


def cpu_baseline(m, budget_s=30.0):
    """Oracle (FP64, numpy/scipy) on one step of the same workload."""
    from oracle import fldref as F
    prob = F.problem_from_medium(m)
    t0 = time.perf_counter()
    F.step(m.E, m.e, m.rho, prob, m.dt, opacity=m.opacity)
    t = time.perf_counter() - t0
    return {"value": m.cells / t, "unit": "cell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"1 split step of the same {m.n[0]}x{m.n[1]} medium "
                      f"(opacity, exact solve by Jacobi-PCG to 1e-13, "
                      f"exchange), {t:.1f} s, single-threaded numpy/scipy"}


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
    ap.add_argument("--workload", choices=("c2", "c3", "c4"), default="c2",
                    help="c2: 2D 1024^2 (the headline); c3: 3D 256^3 "
                         "stratified; c4: 96 batched 2D grids")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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

    import media
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import Stepper, make_params

    if args.workload == "c3":
        return bench_c3(args)
    if args.workload == "c4":
        return bench_c4(args)
    m = media.config_c2(n=args.n)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    def run(precision, steps, warmup, timed_kernel=True, weights=None):
        """warmup + timed steps of one solver variant from the initial state"""
        params = make_params(m.ndim, m.n[:2], m.dx[:2], m.bc, rtol=1e-8,
                             precision=precision, pre_smooth=PRE, post_smooth=POST,
                             coarse_pre_smooth=COARSE_PRE,
                             coarse_post_smooth=COARSE_POST,
                             guess="prev" if weights is None else "learned")
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
        cycles, outer, res, rej = [], [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s = st.step(m.dt, rho, kap, E, e)
            cycles.append(s["cycles"])
            outer.append(s["outer_iters"])
            res.append(s["rel_res_final"])
            rej.append(s["guess_rejected"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kt = fld.fld_kernel_timing_read(st.ctx)
        fld.fld_kernel_timing_enable(st.ctx, False)
        secs = t1 - t0
        return dict(value=m.cells * steps / secs, ms_per_step=secs * 1e3 / steps,
                    vcycles_per_step=float(np.mean(cycles)),
                    outer_per_step=float(np.mean(outer)),
                    rel_res_final_max=float(np.max(res)), kernel=kt,
                    rejected=int(np.sum(rej)), tile_shapes=shapes,
                    E=E.cpu().numpy())

    from paper_2503_02764_amd.guess import load_weights
    weights = load_weights()
    base = run("fp64", args.steps, args.warmup)
    if args.headline_only:
        kt = base["kernel"]
        print(json.dumps({"ms_per_step": base["ms_per_step"],
                          "vcycles_per_step": base["vcycles_per_step"],
                          "finest_down_us": 1e3 * kt["ms"] / max(kt["launches"], 1),
                          "tile_shapes": base["tile_shapes"]}))
        return
    # only the headline run's kernel is priced against the roofline; the
    # variants run without per-launch timing events
    mixed = run("fp32_ir", args.steps, args.warmup, timed_kernel=False)
    lrn64 = run("fp64", args.steps, args.warmup, timed_kernel=False, weights=weights)
    lrn32 = run("fp32_ir", args.steps, args.warmup, timed_kernel=False, weights=weights)
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
            "cycle": f"V({PRE},{POST}), coarse V({COARSE_PRE},{COARSE_POST})",
            "precision": "fp64",
            "guess": "prev",
            "dt": m.dt,
        },
        "vcycles_per_step": base["vcycles_per_step"],
        "rel_res_final_max": base["rel_res_final_max"],
        "tile_shapes_autotuned": base["tile_shapes"],
        "variants": {
            "fp32_vcycles_fp64_refinement": {
                "value": mixed["value"],
                "ms_per_step": mixed["ms_per_step"],
                "vcycles_per_step": mixed["vcycles_per_step"],
                "outer_per_step": mixed["outer_per_step"],
                "rel_res_final_max": mixed["rel_res_final_max"],
                "speedup_vs_fp64": mixed["value"] / base["value"],
                "rel_l2_vs_fp64_after_steps": diff,
            },
            "learned_guess_fp64": {
                "value": lrn64["value"],
                "ms_per_step": lrn64["ms_per_step"],
                "vcycles_per_step": lrn64["vcycles_per_step"],
                "guess_rejected_steps": lrn64["rejected"],
                "speedup_vs_fp64": lrn64["value"] / base["value"],
            },
            "learned_guess_fp32_vcycles_fp64_refinement": {
                "value": lrn32["value"],
                "ms_per_step": lrn32["ms_per_step"],
                "vcycles_per_step": lrn32["vcycles_per_step"],
                "outer_per_step": lrn32["outer_per_step"],
                "guess_rejected_steps": lrn32["rejected"],
                "speedup_vs_fp64": lrn32["value"] / base["value"],
            },
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
        "step_model_roofline": step_model_roofline(
            2, "fp64", base["value"], base["vcycles_per_step"]),
        "achievable_copy": copy_bandwidth(),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


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


def step_model_roofline(ndim, precision, value, vcycles, outer=None, inner=2):
    """Step-level roofline from the byte model of the path (each pass streams
    its operands once; V(2,2); w = 8 FP64, 4 FP32): per fine cell and step,
    FP64 131 + 283 n_V bytes (2D) or 143 + 286 n_V (3D); FP32 V-cycles in FP64
    refinement with m outer iterations of k inner cycles, 125 + m(56 + 141 k)
    (2D) or 140 + m(64 + 143 k) (3D).  Model bytes x cell-updates/s against
    8 TB/s."""
    if precision == "fp64":
        base, per = (131.0, 283.0) if ndim == 2 else (143.0, 286.0)
        b = base + per * vcycles
    else:
        base, ob, ib = (125.0, 56.0, 141.0) if ndim == 2 else (140.0, 64.0, 143.0)
        b = base + outer * (ob + ib * inner)
    gbs = b * value / 1e9
    return {"bytes_per_cell_step": b, "achieved": gbs, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}


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


def bench_c3(args):
    """3D 256^3 stratified medium: FP64 V-cycles vs FP32 V-cycles in FP64
    refinement (and with the learned guess applied per z-slice)."""
    import numpy as np
    import torch
    import media
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.guess import load_weights
    from paper_2503_02764_amd.solver import Stepper, make_params
    m = media.config_c3()
    steps = min(args.steps, 5)
    warm = min(args.warmup, 1)

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()

    def run(precision, weights=None):
        # the strongly stratified medium (face alpha spans ~8 decades) takes
        # about 50-60 V-cycles per step with rediscretised coarse operators
        params = make_params(3, m.n, m.dx, m.bc, rtol=1e-8, precision=precision,
                             guess="prev" if weights is None else "learned",
                             max_cycles=300, pre_smooth=PRE3,
                             post_smooth=POST3, coarse_pre_smooth=COARSE_PRE3,
                             coarse_post_smooth=COARSE_POST3)
        st = Stepper(params, opacity=m.opacity)
        if weights is not None:
            fld.fld_set_model(st.ctx, weights)
        rho, E, e = d(m.rho), d(m.E), d(m.e)
        kap = torch.empty_like(rho)
        for _ in range(warm):
            st.step(m.dt, rho, kap, E, e)
        torch.cuda.synchronize()
        # the first finest-level colour pass of every V-cycle records its own
        # duration (HIP events the launch records)
        fld.fld_kernel_timing_enable(st.ctx, True)
        fld.fld_kernel_timing_read(st.ctx)  # reset
        cyc, outer = [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            s = st.step(m.dt, rho, kap, E, e)
            cyc.append(s["cycles"])
            outer.append(s["outer_iters"])
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        kt = fld.fld_kernel_timing_read(st.ctx)
        fld.fld_kernel_timing_enable(st.ctx, False)
        res = dict(value=m.cells * steps / secs, ms_per_step=secs * 1e3 / steps,
                   vcycles_per_step=float(np.mean(cyc)),
                   outer_per_step=float(np.mean(outer)),
                   roofline=_hbm_roofline(kt, "256^3"))
        res["step_model_roofline"] = step_model_roofline(
            3, precision, res["value"], res["vcycles_per_step"],
            res["outer_per_step"])
        E_out = E.cpu().numpy()
        del st, rho, E, e, kap
        torch.cuda.empty_cache()
        return res, E_out

    f64, E64 = run("fp64")
    f32, E32 = run("fp32_ir")
    lrn, _ = run("fp32_ir", load_weights())
    f32["rel_l2_vs_fp64_after_steps"] = float(
        np.linalg.norm(E32 - E64) / np.linalg.norm(E64))
    f32["speedup_vs_fp64"] = f32["value"] / f64["value"]
    lrn["speedup_vs_fp64"] = lrn["value"] / f64["value"]
    args.steps, args.warmup = steps, warm
    _line(f32["value"], f32["ms_per_step"], args,
          "3d-256cube-stratified-kramers-fp32-vcycles-fp64-refinement", "f32",
          {"variants": {"fp64_plain_mg": f64, "fp32_vcycles_fp64_refinement": f32,
                        "learned_guess_fp32_vcycles": lrn},
           "cycle": f"V({PRE3},{POST3}), coarse V({COARSE_PRE3},{COARSE_POST3})",
           "roofline": f32["roofline"],
           "step_model_roofline": f32["step_model_roofline"],
           "achievable_copy": copy_bandwidth()})


def bench_c4(args):
    """96 independent 2D grids (sides 128..1024) in one batched context:
    FP32 V-cycles in FP64 refinement, one launch per phase, hipGraph
    replay, autotuned tiles; against the same grids stepped one by one with
    single-grid contexts (same precision, and plain FP64)."""
    import numpy as np
    import torch
    import media
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import Stepper, make_params
    ms = media.config_c4()
    steps = min(args.steps, 5)
    warm = min(args.warmup, 1)
    o = ms[0].opacity
    cells = sum(m.cells for m in ms)

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

        def step():
            fld.fld_opacity_powerlaw_batch(bctx, rho, e, o["k0"], o["a"],
                                           o["b"], o["kmin"], o["kmax"], kap)
            fld.fld_step_batch(bctx, dts, rho, kap, E, E)
            fld.fld_exchange_batch(bctx, dts, rho, kap, E, e)

        for _ in range(warm):
            step()
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        stream.synchronize()
        secs = time.perf_counter() - t0
        E_batch = [x.cpu().numpy() for x in E]
    batch = dict(value=cells * steps / secs, ms_per_step=secs * 1e3 / steps,
                 tile_shapes_autotuned=shapes)
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
        for _ in range(warm):
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

    seq32, E32 = one_by_one("fp32_ir")
    seq64, E64 = one_by_one("fp64")
    diff = max(float(np.linalg.norm(a - b) / np.linalg.norm(b))
               for a, b in zip(E_batch, E64))
    batch["speedup_vs_one_by_one_fp32"] = batch["value"] / seq32["value"]
    batch["speedup_vs_one_by_one_fp64"] = batch["value"] / seq64["value"]
    batch["max_rel_l2_vs_fp64_after_steps"] = diff
    args.steps, args.warmup = steps, warm
    _line(batch["value"], batch["ms_per_step"], args,
          f"2d-batched-{len(ms)}-grids-{cells}-cells-fp32-vcycles-fp64-refinement-graph",
          "f32", {"variants": {"batched": batch, "one_by_one_fp32": seq32,
                               "one_by_one_fp64": seq64}})


if __name__ == "__main__":
    main()
