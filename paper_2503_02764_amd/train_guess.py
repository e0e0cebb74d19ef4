"""Train the learned initial guess on the GPU with the library's own kernels.

Training set: seeded 256^2 media with the 2D log-normal/Kramers statistics
(log-normal rho, T = 1 + 0.1 g, Kramers opacity, Neumann walls), a
diffusion number drawn log-uniformly from [10, 1000] and a cell width
between 1/1024 and 1/256 (media.config_c5_train, seeds 5,000,000 + i;
held-out media use 6,000,000 + i).  Medium i is sampled after 0, 1, 3 or 7
full split steps (i mod 4), so that the states the solver meets later in a
run are represented.  The network input is what fld_step feeds the network
(fld_features) and the target is delta = (E* - E^n) / E^n, where E* is the
backward-Euler diffusion solve of the same library in FP64 to relative
residual 1e-11 (its error against the exact solve is below 1e-10, far under
the BF16 resolution of the network).  Inputs and targets stay resident in
device memory; training runs fldnn_train_step (BF16 MFMA forward/backward,
FP32 Adam) over shuffled mini-batches, by default on the energy-norm loss
of the guess error (fldnn_set_loss), which weighs the error the way the
multigrid solve that follows sees it.

Writes the FP32 parameter array (little-endian, layer order of fldnn.h) and
a JSON record of the recipe, the loss history and the held-out evaluation.

Usage: python -m paper_2503_02764_amd.train_guess --samples 20000 --epochs 4
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_DIR = os.path.join(PKG, "weights")
DEFAULT_WEIGHTS = os.path.join(WEIGHTS_DIR, "unet_c5_256.f32")
HELDOUT_OFFSET = 1_000_000  # index offset: seeds 6,000,000 + i


PRE_STEPS = (0, 1, 3, 7)  # full steps taken before medium i is sampled


def _medium(index):
    import media
    m = media.config_c5_train(index)
    return index, m.rho, m.E, m.e, m.dt, m.dx[0], m.opacity


def _media_stream(indices, pool):
    """Seeded media, in order, from a CPU process pool (or in-process)."""
    if pool is None:
        for i in indices:
            yield _medium(i)
        return
    for item in pool.imap(_medium, indices, chunksize=8):
        yield item


class _Grid:
    """Contexts on n^2 Neumann grids of any cell width, sharing workspaces."""

    def __init__(self, n):
        import torch
        from . import fld
        self.fld = fld
        self.n = n
        self.ws = {}
        self.torch = torch

    def ctx(self, dx, rtol, precision="fp64", guess="prev", key=0):
        from .solver import make_params
        p = make_params(2, (self.n, self.n), (dx, dx), ("neumann", "neumann"),
                        rtol=rtol, precision=precision, guess=guess,
                        max_cycles=200, guess_policy="every_step")
        need = self.fld.fld_workspace_bytes(p)
        ws = self.ws.get(key)
        if ws is None or ws.numel() < need:
            ws = self.torch.empty(need, dtype=self.torch.uint8, device="cuda")
            self.ws[key] = ws
        return self.fld.fld_setup(p, workspace=ws)

    def state(self, item, ctx):
        """Device fields of a medium after its pre-steps (opacity, diffusion,
        exchange), and the opacity of the step to sample."""
        torch, fld = self.torch, self.fld
        i, rho, E, e, dt, dx, o = item
        r = torch.from_numpy(rho).cuda().reshape(-1)
        En = torch.from_numpy(E).cuda().reshape(-1)
        ei = torch.from_numpy(e).cuda().reshape(-1)
        kap = torch.empty_like(r)
        for _ in range(PRE_STEPS[i % len(PRE_STEPS)]):
            fld.fld_opacity_powerlaw(ctx, r, ei, o["k0"], o["a"], o["b"],
                                     o["kmin"], o["kmax"], kap)
            fld.fld_step(ctx, dt, r, kap, En, En)
            fld.fld_exchange(ctx, dt, r, kap, En, ei)
        fld.fld_opacity_powerlaw(ctx, r, ei, o["k0"], o["a"], o["b"],
                                 o["kmin"], o["kmax"], kap)
        return r, kap, En, dt


def build_dataset(indices, n, pool, log):
    import torch
    from . import fld
    S = len(indices)
    X = torch.empty((S, n, n, 4), dtype=torch.float32, device="cuda")
    Y = torch.empty((S, n, n), dtype=torch.float32, device="cuda")
    grid = _Grid(n)
    t0 = time.time()
    for k, item in enumerate(_media_stream(indices, pool)):
        ctx = grid.ctx(item[5], 1e-11)
        r, kap, En, dt = grid.state(item, ctx)
        fld.fld_features(ctx, dt, r, kap, En, X[k].reshape(-1))
        Es = torch.empty_like(En)
        fld.fld_step(ctx, dt, r, kap, En, Es)
        Y[k].reshape(-1).copy_(((Es - En) / En).to(torch.float32))
        if (k + 1) % 2000 == 0 or k + 1 == S:
            torch.cuda.synchronize()
            log(f"data {k + 1}/{S} samples, {time.time() - t0:.1f} s")
    return X, Y


def evaluate(weights, indices, n, pool, precision="fp64"):
    """V-cycles and initial residuals with and without the learned guess, on
    the same states (rel. residual 1e-8)."""
    import torch
    from . import fld
    grid = _Grid(n)
    rows = []
    for item in _media_stream(indices, pool):
        dx = item[5]
        prev = grid.ctx(dx, 1e-8, precision, "prev", key=0)
        learned = grid.ctx(dx, 1e-8, precision, "learned", key=1)
        fld.fld_set_model(learned, weights)
        r, kap, En, dt = grid.state(item, prev)
        x0, x1 = torch.empty_like(En), torch.empty_like(En)
        _, s0 = fld.fld_step(prev, dt, r, kap, En, x0)
        _, s1 = fld.fld_step(learned, dt, r, kap, En, x1)
        rows.append(dict(index=item[0], cycles_prev=s0["cycles"],
                         cycles_learned=s1["cycles"],
                         res0_prev=s0["rel_res_initial"],
                         res0_learned=s1["rel_res_initial"],
                         rejected=s1["guess_rejected"]))
    c0 = np.array([r["cycles_prev"] for r in rows], dtype=float)
    c1 = np.array([r["cycles_learned"] for r in rows], dtype=float)
    q = np.array([r["res0_learned"] / r["res0_prev"] for r in rows])
    return dict(media=len(rows), precision=precision,
                mean_cycles_prev=float(c0.mean()),
                mean_cycles_learned=float(c1.mean()),
                median_initial_residual_ratio=float(np.median(q)),
                rejected=int(sum(r["rejected"] for r in rows)))


# the network of fldnn.h: (input channels, output channels, kernel size,
# resolution level) per layer, in parameter order
LAYERS = [(4, 16, 3, 0), (16, 16, 3, 0), (16, 32, 3, 1), (32, 32, 3, 1),
          (32, 64, 3, 2), (64, 64, 3, 2), (64, 128, 3, 3), (128, 128, 3, 3),
          (192, 64, 3, 2), (64, 64, 3, 2), (96, 32, 3, 1), (32, 32, 3, 1),
          (48, 16, 3, 0), (16, 16, 3, 0), (16, 1, 1, 0)]


def forward_flops(H, W, padded=True):
    """Multiply-add flops of one forward pass on an H x W image (the kernels
    pad channel counts to multiples of 16)."""
    pad = (lambda c: (c + 15) // 16 * 16) if padded else (lambda c: c)
    total = 0
    for ci, co, k, lev in LAYERS:
        pixels = (H >> lev) * (W >> lev)
        total += 2 * k * k * pad(ci) * (pad(co) if k > 1 else co) * pixels
    return total


def he_init(seed):
    """He-normal weights, zero biases, head scaled down (FP32, fldnn.h order)."""
    rng = np.random.default_rng(seed)
    layers = [(ci, co, k) for ci, co, k, _ in LAYERS]
    parts = []
    for li, (ci, co, k) in enumerate(layers):
        std = math.sqrt(2.0 / (ci * k * k))
        if li == len(layers) - 1:
            std = 0.1 / math.sqrt(ci)
        parts.append(std * rng.standard_normal(k * k * ci * co))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def run(args, log=print):
    # the media workers start before this process touches the GPU
    pool = (mp.get_context("spawn").Pool(args.workers)
            if args.workers > 1 else None)
    try:
        return _run(args, pool, log)
    finally:
        if pool is not None:
            pool.close()
            pool.join()


def _run(args, pool, log):
    import torch
    from . import fld
    n = args.size
    train_idx = list(range(args.samples))
    log(f"building {args.samples} training media of {n}^2")
    X, Y = build_dataset(train_idx, n, pool, log)
    B = args.batch
    net = fld.fldnn_create(B, n, n, training=True)
    fld.fldnn_set_params(net, he_init(args.seed))
    fld.fldnn_set_loss(net, args.loss)
    steps_per_epoch = args.samples // B
    total = steps_per_epoch * args.epochs
    g = torch.Generator(device="cpu").manual_seed(args.seed)
    xb = torch.empty((B, n, n, 4), dtype=torch.float32, device="cuda")
    yb = torch.empty((B, n, n), dtype=torch.float32, device="cuda")
    history = []
    step = 0
    t0 = time.time()
    for ep in range(args.epochs):
        perm = torch.randperm(args.samples, generator=g).cuda()
        losses = []
        for s in range(steps_per_epoch):
            idx = perm[s * B:(s + 1) * B]
            torch.index_select(X, 0, idx, out=xb)
            torch.index_select(Y, 0, idx, out=yb)
            step += 1
            lr = args.lr * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / total))
            want = (s % 50 == 0) or s == steps_per_epoch - 1
            loss = fld.fldnn_train_step(net, xb, yb, lr, step, want_loss=want)
            if want:
                losses.append(loss)
            if s % 250 == 0:
                log(f"epoch {ep + 1} step {s}/{steps_per_epoch}: loss {loss:.5f} "
                    f"lr {lr:.2e}, {time.time() - t0:.1f} s")
        torch.cuda.synchronize()
        history.append(float(np.mean(losses)))
        log(f"epoch {ep + 1}/{args.epochs}: mean sampled loss "
            f"{history[-1]:.5f}, {time.time() - t0:.1f} s")
    train_s = time.time() - t0
    w = fld.fldnn_get_params(net)
    del X, Y
    torch.cuda.empty_cache()
    held = list(range(HELDOUT_OFFSET, HELDOUT_OFFSET + args.heldout))
    ev = evaluate(w, held, n, pool)
    log(f"held-out FP64: {ev}")
    ev32 = evaluate(w, held, n, pool, precision="fp32_ir")
    log(f"held-out FP32_IR: {ev32}")
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    w.astype("<f4").tofile(args.out)
    meta = dict(
        file=os.path.basename(args.out), params=int(w.size), dtype="float32 LE",
        layout="fldnn.h parameter order", size=n, samples=args.samples,
        epochs=args.epochs, batch=B, lr=args.lr, schedule="cosine",
        loss=args.loss, pre_steps=list(PRE_STEPS),
        optimizer="Adam(0.9, 0.999, 1e-8)", init_seed=args.seed,
        train_media="media.config_c5_train(i), i < samples (seed 5e6 + i), "
                    "sampled after PRE_STEPS[i % 4] full steps",
        heldout_media=f"media.config_c5_train(1e6 + i), i < {args.heldout}",
        target="delta = (E* - E^n) / E^n, E* = FP64 solve to rel. residual 1e-11",
        loss_history=history, train_seconds=train_s,
        heldout_fp64=ev, heldout_fp32_ir=ev32)
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log(f"wrote {args.out}")
    return meta


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--samples", type=int, default=20000)
    ap.add_argument("--heldout", type=int, default=200)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--loss", choices=("mse", "energy"), default="energy")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--eval-only", metavar="WEIGHTS",
                    help="only evaluate these weights on the held-out media")
    args = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)  # noqa: E731
    if args.eval_only:
        w = np.fromfile(args.eval_only, dtype="<f4")
        held = list(range(HELDOUT_OFFSET, HELDOUT_OFFSET + args.heldout))
        for prec in ("fp64", "fp32_ir"):
            log(f"held-out {prec}: {evaluate(w, held, args.size, None, prec)}")
        return 0
    run(args, log=log)
    return 0


if __name__ == "__main__":
    sys.exit(main())
