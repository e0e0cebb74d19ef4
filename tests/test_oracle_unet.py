"""Pins of the CPU FP64 U-Net reference (the learned guess's arithmetic).

- convolution against scipy.signal.correlate (an independent routine);
- every parameter gradient and the input gradient against central finite
  differences of the loss (FP64, relative error <= 1e-6 on sampled entries);
- pooling/upsampling adjointness.
"""
import numpy as np
import pytest
from scipy.signal import correlate

from oracle import unet_ref as U


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 9, 7, 3))
    w = rng.standard_normal((3, 3, 3, 5))
    b = rng.standard_normal(5)
    y = U.conv(x, w, b)
    for n in range(2):
        for co in range(5):
            ref = b[co] + sum(
                correlate(x[n, :, :, ci], w[:, :, ci, co], mode="same")
                for ci in range(3))
            np.testing.assert_allclose(y[n, :, :, co], ref, rtol=1e-12,
                                       atol=1e-12)


def test_pool_up_adjoint():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 8, 6, 3))
    y = rng.standard_normal((1, 4, 3, 3))
    # <pool x, y> = <x, pool^T y>; <up y, x> = <y, up^T x>
    assert np.isclose(np.sum(U.pool(x) * y), np.sum(x * U.pool_backward(y)))
    assert np.isclose(np.sum(U.up(y) * x), np.sum(y * U.up_backward(x)))


def _loss(p, x, t):
    d, _ = U.forward(p, x)
    return U.mse_loss(d, t)[0]


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_vs_finite_differences(seed):
    rng = np.random.default_rng(10 + seed)
    p = U.init_params(seed)
    for k in p:  # non-zero biases so every term is exercised
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((2, 8, 8, 4))
    t = 0.1 * rng.standard_normal((2, 8, 8, 1))
    d, cache = U.forward(p, x)
    _, dd = U.mse_loss(d, t)
    g, dx = U.backward(p, cache, dd)
    h = 1e-6
    for name in sorted(p):
        flat = p[name].reshape(-1)
        idx = rng.choice(flat.size, size=min(3, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = _loss(p, x, t)
            flat[i] = old - h
            lm = _loss(p, x, t)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10, \
                (name, i, fd, an)
    xf = x.reshape(-1)
    for i in rng.choice(xf.size, size=5, replace=False):
        old = xf[i]
        xf[i] = old + h
        lp = _loss(p, x, t)
        xf[i] = old - h
        lm = _loss(p, x, t)
        xf[i] = old
        fd = (lp - lm) / (2 * h)
        assert abs(fd - dx.reshape(-1)[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10


def test_parameter_count():
    p = U.init_params(0)
    n = sum(v.size for v in p.values())
    assert 480_000 < n < 500_000


def test_adam_descends():
    rng = np.random.default_rng(3)
    p = U.init_params(3)
    x = rng.standard_normal((1, 8, 8, 4))
    t = 0.05 * rng.standard_normal((1, 8, 8, 1))
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    l0 = _loss(p, x, t)
    for step in range(1, 30):
        d, c = U.forward(p, x)
        _, dd = U.mse_loss(d, t)
        g, _ = U.backward(p, c, dd)
        U.adam_step(p, g, m, v, step, lr=1e-3)
    assert _loss(p, x, t) < 0.5 * l0


def _feats(rng, N, H, W):
    f = np.empty((N, H, W, 4))
    f[..., 0] = 0.3 * rng.standard_normal((N, H, W))
    f[..., 1] = rng.standard_normal((N, H, W))
    f[..., 2:] = 0.25 * np.log1p(np.exp(3 * rng.standard_normal((N, H, W, 2))))
    return f


def test_energy_loss_quadratic_form_matches_fld_operator():
    """|e|_A^2 equals e . A e with the oracle's own backward-Euler operator
    (a 2D Neumann problem whose wall faces carry alpha = 0)."""
    from oracle import fldref as F
    rng = np.random.default_rng(21)
    N, H, W = 2, 8, 12
    f = _feats(rng, N, H, W)
    f[:, :, -1, 2] = 0.0  # wall faces of the Neumann problem
    f[:, -1, :, 3] = 0.0
    d = 0.1 * rng.standard_normal((N, H, W, 1))
    t = 0.1 * rng.standard_normal((N, H, W, 1))
    loss, _ = U.energy_loss(d, t, f)
    prob = F.Problem(ndim=2, n=(W, H, 1), dx=(1.0, 1.0, 1.0),
                     bc=("neumann", "neumann"))
    E = np.exp(f[..., 0])
    ratios = []
    for k in range(N):
        al = [np.expm1(4 * f[k, :, :, 2]), np.expm1(4 * f[k, :, :, 3])]
        e = E[k] * (d[k, ..., 0] - t[k, ..., 0])
        e0 = E[k] * t[k, ..., 0]
        ratios.append(np.sum(e * F.apply_operator(e, al, prob)) /
                      np.sum(e0 * F.apply_operator(e0, al, prob)))
    assert np.isclose(loss, np.mean(ratios), rtol=1e-12)
    # a perfect prediction has zero loss; delta = 0 (the plain guess) has 1
    assert U.energy_loss(t, t, f)[0] == 0.0
    assert np.isclose(U.energy_loss(0 * t, t, f)[0], 1.0, rtol=1e-14)


def test_energy_loss_gradient_vs_finite_differences():
    rng = np.random.default_rng(22)
    N, H, W = 2, 8, 8
    f = _feats(rng, N, H, W)
    d = 0.1 * rng.standard_normal((N, H, W, 1))
    t = 0.1 * rng.standard_normal((N, H, W, 1))
    _, g = U.energy_loss(d, t, f)
    h = 1e-7
    df = d.reshape(-1)
    for i in rng.choice(df.size, size=12, replace=False):
        old = df[i]
        df[i] = old + h
        lp = U.energy_loss(d, t, f)[0]
        df[i] = old - h
        lm = U.energy_loss(d, t, f)[0]
        df[i] = old
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g.reshape(-1)[i]) <= 1e-6 * max(abs(fd), 1e-3), i


def test_adam_three_steps_hand_values():
    """Adam (Kingma & Ba, Algorithm 1) on one scalar parameter, p0 = 1,
    lr = 0.1, beta1 = 0.9, beta2 = 0.999, eps = 1e-8, gradients 0.5, -0.25, 2:
      t=1: m = 0.05,  v = 2.5e-4,      m^ = 0.5,      v^ = 0.25,
           p = 1 - 0.1 * 0.5 / (0.5 + 1e-8)              = 0.90000000199999996
      t=2: m = 0.02,  v = 3.1225e-4,   m^ = 0.02/0.19, v^ = 3.1225e-4/1.999e-3,
           p                                             = 0.87336629870784616
      t=3: m = 0.218, v = 4.31193775e-3, m^ = 0.218/0.271,
           v^ = 4.31193775e-3 / 2.997001e-3,  p          = 0.80630153452915290
    (worked to 30 digits; without the bias correction the first step alone
    gives 0.6838)."""
    p = {"w": np.array([1.0])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    expect = [0.90000000199999996, 0.87336629870784616, 0.80630153452915290]
    for t, (g, want) in enumerate(zip([0.5, -0.25, 2.0], expect), start=1):
        U.adam_step(p, {"w": np.array([g])}, m, v, t, lr=0.1)
        assert p["w"][0] == pytest.approx(want, rel=1e-14), t
    assert m["w"][0] == pytest.approx(0.218, rel=1e-14)
    assert v["w"][0] == pytest.approx(4.31193775e-3, rel=1e-14)


def test_features_hand_values():
    """Network inputs on a 1 x 2 image with E = (1, e^2) (log E = 0, 2, mean
    1), rho kappa dx = (e^4, e^-8), alpha_x = (e^8 - 1, 0),
    alpha_y = (0, e^4 - 1): features (-1, 1) / (1, -2) / (2, 0) / (0, 1)."""
    E = np.exp(np.array([[0.0, 2.0]]))
    f = U.features(E, np.exp(np.array([[4.0, -8.0]])),
                   np.array([[np.expm1(8.0), 0.0]]),
                   np.array([[0.0, np.expm1(4.0)]]))
    assert f.shape == (1, 1, 2, 4)
    np.testing.assert_allclose(f[0, 0], [[-1.0, 1.0, 2.0, 0.0],
                                         [1.0, -2.0, 0.0, 1.0]],
                               rtol=1e-14, atol=1e-15)
