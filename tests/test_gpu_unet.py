"""The learned initial guess on the GPU, through the C ABI.

Network arithmetic against the FP64 CPU U-Net (oracle/unet_ref.py, itself
pinned by finite differences): forward pass, loss, every parameter gradient
and the Adam update.  The GPU computes in BF16 with FP32 accumulation; the
reference gets the same BF16-rounded weights and inputs, so the remaining
difference is the BF16 rounding of activations (unit roundoff 2^-8 per
stored value, accumulated over 15 layers): forward rel-L2 <= 1e-2, loss
<= 1e-2 relative.  Gradients: the backward pass rounds the incoming gradient
of every layer to BF16 before its two GEMMs, so the error grows with the
number of layers crossed (measured: 0.8% at the last decoder level, 2.5% at
the bottleneck); it is largest on the first layer's weights (3.5%), whose
sums over zero-mean inputs cancel.  The stored activations that feed every
weight gradient are BF16 as well (the forward pass differs from the FP64
reference by about 1e-2), so no tensor can be held much below that.
Bar: rel-L2 <= 2e-2 averaged over the parameter tensors, <= 4e-2 for every
tensor.

The solver side: the features fld_step feeds the network match the
oracle's coefficients to FP32 rounding, and a step with the learned guess
returns the oracle's solution whatever the network proposes (the guess only
changes where the iteration starts; a worse guess is rejected).
"""
import numpy as np
import pytest

import media
from oracle import fldref as F
from oracle import unet_ref as U
from gpu_common import announce, dev, host, params_for, rel_l2

pytestmark = pytest.mark.gpu


def _bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _flat(p):
    return np.concatenate([np.concatenate([p[n + ".w"].ravel(),
                                           p[n + ".b"].ravel()])
                           for n, _, _, _ in U.LAYERS]).astype(np.float32)


def _slices():
    out, o = {}, 0
    for n, ci, co, k in U.LAYERS:
        out[n + ".w"] = (o, o + k * k * ci * co, (k, k, ci, co))
        o += k * k * ci * co
        out[n + ".b"] = (o, o + co, (co,))
        o += co
    return out


def _params(seed):
    rng = np.random.default_rng(100 + seed)
    p = U.init_params(seed)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    return {k: _bf16(v) for k, v in p.items()}


def _f32dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("N,H,W", [(2, 16, 16), (1, 24, 80), (1, 64, 136)])
def test_forward_vs_oracle(N, H, W):
    import torch
    from paper_2503_02764_amd import fld
    rng = np.random.default_rng(N * H + W)
    p = _params(1)
    x = _bf16(rng.standard_normal((N, H, W, 4)))
    ref, _ = U.forward(p, x)
    announce(f"unet forward N={N} H={H} W={W}")
    net = fld.fldnn_create(N, H, W, training=False)
    fld.fldnn_set_params(net, _flat(p))
    delta = torch.empty(N * H * W, dtype=torch.float32, device="cuda")
    fld.fldnn_forward(net, _f32dev(x), delta)
    torch.cuda.synchronize()
    got = host(delta).reshape(ref.shape)
    assert rel_l2(got, ref) <= 1e-2, rel_l2(got, ref)
    # parameters round-trip unchanged
    np.testing.assert_array_equal(fld.fldnn_get_params(net), _flat(p))


@pytest.mark.parametrize("N,H,W", [(2, 16, 16), (1, 24, 80), (3, 64, 136)])
def test_fused_inference_forward_is_bit_identical(N, H, W):
    """Without training the decoders read their upsampled input straight
    from the coarser level and the encoders write the pooled tensor from
    their convolution's epilogue; a training-mode network (upsampled copy
    materialised) must give the same bits."""
    import torch
    from paper_2503_02764_amd import fld
    rng = np.random.default_rng(7 * N + H + W)
    p = _params(2)
    x = _f32dev(_bf16(rng.standard_normal((N, H, W, 4))))
    announce(f"unet fused inference vs training forward N={N} H={H} W={W}")
    out = []
    for training in (False, True):
        net = fld.fldnn_create(N, H, W, training=training)
        fld.fldnn_set_params(net, _flat(p))
        delta = torch.empty(N * H * W, dtype=torch.float32, device="cuda")
        fld.fldnn_forward(net, x, delta)
        torch.cuda.synchronize()
        out.append(host(delta))
    np.testing.assert_array_equal(out[0], out[1])


def test_gradients_vs_oracle():
    from paper_2503_02764_amd import fld
    N, H, W = 2, 16, 16
    rng = np.random.default_rng(7)
    p = _params(2)
    x = _bf16(rng.standard_normal((N, H, W, 4)))
    t = 0.1 * rng.standard_normal((N, H, W, 1)).astype(np.float32)
    d, cache = U.forward(p, x)
    loss_ref, dd = U.mse_loss(d, t.astype(np.float64))
    g_ref, _ = U.backward(p, cache, dd)
    announce("unet gradients N=2 16x16")
    net = fld.fldnn_create(N, H, W, training=True)
    fld.fldnn_set_params(net, _flat(p))
    loss, g = fld.fldnn_gradients(net, _f32dev(x), _f32dev(t))
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref, (loss, loss_ref)
    errs = {name: rel_l2(g[a:b].reshape(shape), g_ref[name])
            for name, (a, b, shape) in _slices().items()}
    print("gradient rel-L2 per parameter:", errs)
    assert max(errs.values()) <= 4e-2, errs
    assert np.mean(list(errs.values())) <= 2e-2, errs


def test_energy_loss_kernel_vs_oracle():
    """The loss kernel alone: with all weights zero the network predicts the
    constant delta = b (the head's bias), every activation is zero, and the
    bias gradient is the sum over pixels of d loss / d delta.  Rough targets
    and face coefficients up to ~400 exercise every face term."""
    from paper_2503_02764_amd import fld
    N, H, W = 3, 16, 24
    rng = np.random.default_rng(18)
    f = np.empty((N, H, W, 4))
    f[..., 0] = 0.3 * rng.standard_normal((N, H, W))
    f[..., 1] = rng.standard_normal((N, H, W))
    f[..., 2:] = 0.25 * np.log1p(np.exp(3 * rng.standard_normal((N, H, W, 2))))
    f32 = f.astype(np.float32).astype(np.float64)
    t = (0.2 * rng.standard_normal((N, H, W, 1))).astype(np.float32)
    announce("unet energy-norm loss kernel")
    net = fld.fldnn_create(N, H, W, training=True)
    fld.fldnn_set_loss(net, "energy")
    for b in (0.0, 0.05, -0.3):
        fld.fldnn_set_params(net, _zero_model(b))
        loss, g = fld.fldnn_gradients(net, _f32dev(f32), _f32dev(t))
        ref, gref = U.energy_loss(np.full((N, H, W, 1), b), t.astype(np.float64),
                                  f32)
        assert abs(loss - ref) <= 1e-5 * ref, (b, loss, ref)
        assert abs(g[-1] - gref.sum()) <= 1e-4 * np.abs(gref).sum(), \
            (b, g[-1], gref.sum())
        assert np.all(g[:-1] == 0.0)


def _smooth(a, passes=8):
    """Unit-variance low-pass noise: repeated 5-point averaging (periodic)."""
    for _ in range(passes):
        a = (a + np.roll(a, 1, 1) + np.roll(a, -1, 1) + np.roll(a, 1, 2) +
             np.roll(a, -1, 2)) / 5.0
    return a / a.std()


def test_energy_loss_gradients_vs_oracle():
    """The energy-norm loss's gradient in delta is 2 E (A e).  Where e is
    rough (the output of an untrained network is) it is a high-pass field
    whose 2x2 sums cancel, so the coarse levels of the network receive
    gradients made of cancellation and a BF16-vs-FP64 comparison loses its
    meaning there (measured: 10% at levels 1-3).  This case keeps e smooth,
    as it is near a trained network: smooth E and targets (like the solve's
    delta*), a head scaled down so that delta is small, alpha of order
    one.  The loss itself is checked too, and that a network predicting
    delta = 0 (the plain guess) scores exactly 1.  The kernel itself is
    pinned tightly by test_energy_loss_kernel_vs_oracle; here the bar is the
    chain's: rel-L2 <= 1.5e-1 per tensor (measured at most 10%, at level 2)
    and <= 6e-2 on average."""
    import torch
    from paper_2503_02764_amd import fld
    N, H, W = 2, 16, 24
    rng = np.random.default_rng(17)
    p = _params(4)
    p["head.w"] = _bf16(0.01 * p["head.w"])
    p["head.b"] = _bf16(0.01 * p["head.b"])
    f = np.empty((N, H, W, 4))
    f[..., 0] = 0.3 * _smooth(rng.standard_normal((N, H, W)))
    f[..., 1] = rng.standard_normal((N, H, W))
    f[..., 2:] = 0.25 * np.log1p(np.exp(0.5 * rng.standard_normal((N, H, W, 2))))
    x = _bf16(f)  # the network sees BF16; the loss reads the FP32 copy
    f32 = x.astype(np.float32).astype(np.float64)
    t = (0.2 * _smooth(rng.standard_normal((N, H, W))))[..., None]
    t = t.astype(np.float32)
    d, cache = U.forward(p, x)
    loss_ref, dd = U.energy_loss(d, t.astype(np.float64), f32)
    g_ref, _ = U.backward(p, cache, dd)
    announce("unet energy-norm loss gradients N=2 16x24")
    net = fld.fldnn_create(N, H, W, training=True)
    fld.fldnn_set_params(net, _flat(p))
    fld.fldnn_set_loss(net, "energy")
    loss, g = fld.fldnn_gradients(net, _f32dev(x), _f32dev(t))
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref, (loss, loss_ref)
    errs = {name: rel_l2(g[a:b].reshape(shape), g_ref[name])
            for name, (a, b, shape) in _slices().items()}
    print("energy-loss gradient rel-L2 per parameter:", errs)
    assert max(errs.values()) <= 1.5e-1, errs
    assert np.mean(list(errs.values())) <= 6e-2, errs
    fld.fldnn_set_params(net, _zero_model(0.0))
    loss0, _ = fld.fldnn_gradients(net, _f32dev(x), _f32dev(t))
    torch.cuda.synchronize()
    assert abs(loss0 - 1.0) <= 1e-5, loss0


def test_adam_update_matches_oracle_formula():
    from paper_2503_02764_amd import fld
    N, H, W = 1, 16, 24
    rng = np.random.default_rng(8)
    p = _params(3)
    x = _bf16(rng.standard_normal((N, H, W, 4)))
    t = 0.1 * rng.standard_normal((N, H, W, 1)).astype(np.float32)
    announce("unet adam step")
    net = fld.fldnn_create(N, H, W, training=True)
    flat = _flat(p)
    fld.fldnn_set_params(net, flat)
    xd, td = _f32dev(x), _f32dev(t)
    _, g = fld.fldnn_gradients(net, xd, td)
    lr = 1e-3
    fld.fldnn_train_step(net, xd, td, lr, 1)
    got = fld.fldnn_get_params(net).astype(np.float64)
    # the oracle's Adam on the GPU gradient (step 1: m/(1-b1) = g,
    # v/(1-b2) = g^2)
    pd = {"w": flat.astype(np.float64)}
    gd = {"w": g.astype(np.float64)}
    m = {"w": np.zeros_like(pd["w"])}
    v = {"w": np.zeros_like(pd["w"])}
    U.adam_step(pd, gd, m, v, 1, lr=lr)
    err = np.abs(got - pd["w"])
    # the recomputed gradient may differ in its last bits (atomic sums):
    # a relative change eps of g moves the step by about lr * eps
    tol = 1e-3 * lr + 4 * np.spacing(np.abs(flat)).astype(np.float64)
    assert np.mean(err <= tol) >= 0.999, np.sort(err - tol)[-5:]
    assert err.max() <= 2 * lr


def test_training_reduces_loss():
    import torch
    from paper_2503_02764_amd import fld
    N, H, W = 4, 32, 32
    rng = np.random.default_rng(11)
    x = _bf16(rng.standard_normal((N, H, W, 4)))
    t = (0.1 * np.tanh(x[..., :1]) - 0.05 * x[..., 1:2]).astype(np.float32)
    p = U.init_params(4)
    announce("unet training 150 steps")
    net = fld.fldnn_create(N, H, W, training=True)
    fld.fldnn_set_params(net, _flat(p))
    xd, td = _f32dev(x), _f32dev(t)
    l0 = fld.fldnn_train_step(net, xd, td, 2e-3, 1, want_loss=True)
    for step in range(2, 150):
        fld.fldnn_train_step(net, xd, td, 2e-3, step)
    l1 = fld.fldnn_train_step(net, xd, td, 2e-3, 150, want_loss=True)
    torch.cuda.synchronize()
    assert np.isfinite(l1) and l1 < 0.2 * l0, (l0, l1)


def _kappa(m, prob):
    return m.kappa if m.kappa is not None else \
        F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)


@pytest.mark.parametrize("case", ["c2-64", "3d-16x8x4"])
def test_features_vs_oracle(case):
    import torch
    from paper_2503_02764_amd import fld
    if case == "c2-64":
        m = media.config_c2(n=64)
    else:
        m = media.random_small_medium(5, (16, 8, 4),
                                      ("periodic", "neumann", "neumann"))
    prob = F.problem_from_medium(m)
    kap = _kappa(m, prob)
    al = F.face_coefficients(m.E, m.rho, kap, m.dt, prob)
    E3 = m.E.reshape(-1, m.n[1], m.n[0])
    ref = np.concatenate([
        U.features(E3[k], (m.rho * kap).reshape(E3.shape)[k] * m.dx[0],
                   al[0].reshape(E3.shape)[k], al[1].reshape(E3.shape)[k])
        for k in range(E3.shape[0])])
    announce(f"features {case}")
    ctx = fld.fld_setup(params_for(m))
    out = torch.empty(m.cells * 4, dtype=torch.float32, device="cuda")
    fld.fld_features(ctx, m.dt, dev(m.rho), dev(kap), dev(m.E), out)
    got = host(out).reshape(ref.shape)
    np.testing.assert_allclose(got, ref, rtol=2e-7, atol=1e-7)


def _zero_model(head_bias):
    """All weights zero; the head's bias (the last parameter) = head_bias."""
    z = np.zeros(sum(k * k * ci * co + co for _, ci, co, k in U.LAYERS),
                 dtype=np.float32)
    z[-1] = head_bias
    return z


def _learned_step(m, kap, model, **kw):
    """One step with the network evaluated (FLD_GUESS_EVERY_STEP)."""
    from paper_2503_02764_amd import fld
    kw.setdefault("guess_policy", "every_step")
    ctx = fld.fld_setup(params_for(m, guess="learned", **kw))
    fld.fld_set_model(ctx, model)
    out = dev(np.zeros_like(m.E))
    _, stats = fld.fld_step(ctx, m.dt, dev(m.rho), dev(kap), dev(m.E), out)
    return host(out), stats


def test_learned_guess_step_matches_oracle():
    m = media.config_c2(n=128)
    prob = F.problem_from_medium(m)
    kap = _kappa(m, prob)
    ref = F.diffusion_step(m.E, m.rho, kap, m.dt, prob)
    announce("learned guess c2 128: random network, FP64 and FP32_IR")
    x, stats = _learned_step(m, kap, _flat(U.init_params(5)), rtol=1e-12)
    assert stats["guess_rejected"] in (0, 1)
    assert rel_l2(x, ref) <= 1e-10, stats
    x, stats = _learned_step(m, kap, _flat(U.init_params(5)), rtol=1e-9,
                             precision="fp32_ir")
    assert rel_l2(x, ref) <= 1e-8, stats


def test_learned_guess_fallback():
    m = media.config_c2(n=128)
    prob = F.problem_from_medium(m)
    kap = _kappa(m, prob)
    ref = F.diffusion_step(m.E, m.rho, kap, m.dt, prob)
    announce("learned guess fallback c2 128")
    # delta = 0: the candidate equals E^n and stays equal to it through the
    # same smoothing, so it is not strictly better: rejected
    x0, s0 = _learned_step(m, kap, _zero_model(0.0), rtol=1e-12)
    assert s0["guess_rejected"] == 1
    assert rel_l2(x0, ref) <= 1e-10, s0
    # delta = 0.5: far worse than E^n, rejected, the same iterate follows
    x1, s1 = _learned_step(m, kap, _zero_model(0.5), rtol=1e-12)
    assert s1["guess_rejected"] == 1
    np.testing.assert_array_equal(x1, x0)
    assert s1["cycles"] == s0["cycles"]


def test_learned_guess_3d_slices_match_oracle():
    m = media.random_small_medium(9, (16, 16, 6),
                                  ("periodic", "periodic", "neumann"))
    prob = F.problem_from_medium(m)
    ref = F.diffusion_step(m.E, m.rho, m.kappa, m.dt, prob)
    announce("learned guess 3d 16x16x6")
    x, stats = _learned_step(m, m.kappa, _flat(U.init_params(6)), rtol=1e-12)
    assert rel_l2(x, ref) <= 1e-10, stats


def test_learned_guess_requires_model():
    from paper_2503_02764_amd import fld
    m = media.config_c2(n=64)
    announce("learned guess without model")
    ctx = fld.fld_setup(params_for(m, guess="learned"))
    kap = _kappa(m, F.problem_from_medium(m))
    st, _ = fld.fld_step(ctx, m.dt, dev(m.rho), dev(kap), dev(m.E),
                         dev(np.zeros_like(m.E)), check=False)
    assert st == fld.FLD_ERR_MODEL
    bad = np.zeros(fld.fldnn_param_count(), dtype=np.float32)
    bad[3] = np.nan
    with pytest.raises(fld.FldError):
        fld.fld_set_model(ctx, bad)
    with pytest.raises(ValueError):
        fld.fld_set_model(ctx, bad[:-1])


def test_training_targets_match_oracle_solve():
    """The training pipeline's targets (library FP64 solve after the
    medium's pre-steps) equal the oracle's exact solve of the same state."""
    import torch
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd import train_guess as TG
    idx = 2  # sampled after 3 full steps
    item = TG._medium(idx)
    _, rho, E, e, dt, dx, o = item
    announce("training target vs oracle, medium 2 (3 pre-steps)")
    grid = TG._Grid(rho.shape[0])
    ctx = grid.ctx(dx, 1e-11)
    r, kap, En, dt = grid.state(item, ctx)
    feats = torch.empty(En.numel() * 4, dtype=torch.float32, device="cuda")
    fld.fld_features(ctx, dt, r, kap, En, feats)
    Es = torch.empty_like(En)
    fld.fld_step(ctx, dt, r, kap, En, Es)
    n = rho.shape[0]
    prob = F.Problem(ndim=2, n=(n, n, 1), dx=(dx, dx, 1.0),
                     bc=("neumann", "neumann"))
    En_h = host(En).reshape(n, n)
    kap_h = host(kap).reshape(n, n)
    ref = F.diffusion_step(En_h, rho, kap_h, dt, prob)
    assert rel_l2(host(Es).reshape(n, n), ref) <= 1e-10
    al = F.face_coefficients(En_h, rho, kap_h, dt, prob)
    fref = U.features(En_h, rho * kap_h * dx, al[0], al[1])[0]
    np.testing.assert_allclose(host(feats).reshape(n, n, 4), fref, rtol=2e-7,
                               atol=1e-7)


def test_trained_network_gains_over_plain_guess():
    """What the committed network gains on held-out media (seeds never seen
    in training): its guess, after the finest pre-smoothing, has a smaller
    residual than E^n on most media and the solve needs fewer V-cycles on
    average, with the same answer."""
    from paper_2503_02764_amd import train_guess as TG
    from paper_2503_02764_amd.guess import load_weights
    w = load_weights()
    held = list(range(TG.HELDOUT_OFFSET + 500, TG.HELDOUT_OFFSET + 532))
    announce("trained network on 32 held-out 256^2 media")
    ev = TG.evaluate(w, held, 256, None, "fp64")
    print("held-out evaluation:", ev)
    assert ev["media"] == 32
    assert ev["median_initial_residual_ratio"] < 0.5, ev
    assert ev["rejected"] <= 4, ev
    assert ev["mean_cycles_learned"] < ev["mean_cycles_prev"], ev


def test_adam_three_steps_match_oracle():
    """Three Adam steps on three different batches: from the second step on
    the bias corrections 1 - beta^t no longer cancel (at t = 1 the update is
    about lr sign(g) whatever they are), so this pins them on the GPU.  The
    oracle's Adam (pinned by hand-worked values) replays the same three
    gradients, read from the GPU before each step."""
    from paper_2503_02764_amd import fld
    N, H, W = 1, 16, 24
    rng = np.random.default_rng(28)
    p = _params(5)
    announce("unet adam three steps")
    net = fld.fldnn_create(N, H, W, training=True)
    flat = _flat(p)
    fld.fldnn_set_params(net, flat)
    lr = 1e-3
    pd = {"w": flat.astype(np.float64)}
    m = {"w": np.zeros_like(pd["w"])}
    v = {"w": np.zeros_like(pd["w"])}
    for step in (1, 2, 3):
        x = _bf16(rng.standard_normal((N, H, W, 4)))
        t = (0.1 * step * rng.standard_normal((N, H, W, 1))).astype(np.float32)
        xd, td = _f32dev(x), _f32dev(t)
        _, g = fld.fldnn_gradients(net, xd, td)
        fld.fldnn_train_step(net, xd, td, lr, step)
        # the oracle steps from the GPU's current parameters (FP32) with the
        # same gradient
        U.adam_step(pd, {"w": g.astype(np.float64)}, m, v, step, lr=lr)
        got = fld.fldnn_get_params(net).astype(np.float64)
        err = np.abs(got - pd["w"])
        tol = 3e-3 * lr * step + 4 * np.spacing(np.abs(got).astype(np.float32)
                                                ).astype(np.float64) * step
        assert np.mean(err <= tol) >= 0.999, (step, np.sort(err - tol)[-5:])
        assert err.max() <= 2 * lr * step
        pd["w"] = got  # carry the GPU's FP32 parameters forward


def test_adaptive_policy_on_heldout_1024():
    """The default network policy (FLD_GUESS_ADAPTIVE) on the 1024^2
    workload, a medium the network never saw (it was trained on 256^2 media
    of other seeds), over 12 steps that each start both solvers from the
    same E^n: a step that ran without the network is bit for bit a plain
    step; a step whose guess the judge accepted needed no more V-cycles than
    the plain step (the judge asks the guess's smoothed residual to be a
    cycle's contraction below that of E^n); the first step runs without
    the network, and tries whose saved V-cycles took less time than the
    network pause it (at 1024^2 the network costs about a whole solve, so
    it runs on a few steps only)."""
    import torch
    import bench
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.guess import load_weights
    from paper_2503_02764_amd.solver import Stepper
    m = media.config_c2(n=1024)
    kw = dict(rtol=1e-8, pre_smooth=bench.PRE, post_smooth=bench.POST,
              coarse_pre_smooth=bench.COARSE_PRE,
              coarse_post_smooth=bench.COARSE_POST)
    plain = Stepper(params_for(m, **kw), opacity=m.opacity)
    lrn = fld.fld_setup(params_for(m, guess="learned", **kw))
    fld.fld_set_model(lrn, load_weights())
    rho, E, e = dev(m.rho), dev(m.E), dev(m.e)
    kap = torch.empty_like(rho)
    o = m.opacity
    announce("adaptive learned-guess policy, 12 steps of 1024^2")
    net_steps, accepted, cyc_p, cyc_l = 0, 0, 0, 0
    for step in range(12):
        fld.fld_opacity_powerlaw(plain.ctx, rho, e, o["k0"], o["a"], o["b"],
                                 o["kmin"], o["kmax"], kap)
        xp, xl = torch.empty_like(E), torch.empty_like(E)
        _, sp = fld.fld_step(plain.ctx, m.dt, rho, kap, E, xp)
        _, sl = fld.fld_step(lrn, m.dt, rho, kap, E, xl)
        cyc_p += sp["cycles"]
        cyc_l += sl["cycles"]
        if sl["guess_skipped"]:
            assert torch.equal(xl, xp), step
            assert sl["cycles"] == sp["cycles"]
        else:
            net_steps += 1
            if not sl["guess_rejected"]:
                accepted += 1
                assert sl["cycles"] <= sp["cycles"], (step, sp, sl)
        assert sl["rel_res_final"] <= 1e-8
        if step == 0:
            assert sl["guess_skipped"] == 1
        fld.fld_exchange(plain.ctx, m.dt, rho, kap, xp, e)
        E = xp
    print(f"network on {net_steps} of 12 steps, accepted {accepted}; "
          f"V-cycles {cyc_l} (plain {cyc_p})")
    assert 1 <= net_steps <= 4
    assert cyc_l <= cyc_p
