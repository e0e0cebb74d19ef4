"""FP64 CPU reference of the learned initial guess (a small U-Net).

TEST INFRASTRUCTURE ONLY: used by the tests (finite-difference pins, GPU
forward/backward parity) and never by the product.  It shares no code with
the HIP kernels; the architecture below is the definition both follow.

Not part of the paper: the learned guess is a growth direction of this
project.  Parity of its *predictions* with any physical truth is not a
paper result (the multigrid solve that follows decides the answer); this
module pins the network arithmetic itself.

Architecture (2D, NHWC, 'same' 3x3 convolutions with zero padding):
  level 0 (H x W):        conv 4->16, ReLU, conv 16->16, ReLU      = s0
  level 1 (H/2):  pool s0; conv 16->32, ReLU, conv 32->32, ReLU    = s1
  level 2 (H/4):  pool s1; conv 32->64, ReLU, conv 64->64, ReLU    = s2
  level 3 (H/8):  pool s2; conv 64->128, ReLU, conv 128->128, ReLU = b
  up 2:  concat(s2, up(b))   192 -> conv 64, ReLU, conv 64, ReLU  = u2
  up 1:  concat(s1, up(u2))   96 -> conv 32, ReLU, conv 32, ReLU  = u1
  up 0:  concat(s0, up(u1))   48 -> conv 16, ReLU, conv 16, ReLU  = u0
  head:  1x1 conv 16 -> 1 (no activation)                          = delta
pool = 2x2 average, up = 2x nearest.  Weights W[ky, kx, ci, co], bias b[co].
"""
from __future__ import annotations

import numpy as np

# (name, c_in, c_out, kernel size)
LAYERS = [
    ("e0a", 4, 16, 3), ("e0b", 16, 16, 3),
    ("e1a", 16, 32, 3), ("e1b", 32, 32, 3),
    ("e2a", 32, 64, 3), ("e2b", 64, 64, 3),
    ("e3a", 64, 128, 3), ("e3b", 128, 128, 3),
    ("d2a", 192, 64, 3), ("d2b", 64, 64, 3),
    ("d1a", 96, 32, 3), ("d1b", 32, 32, 3),
    ("d0a", 48, 16, 3), ("d0b", 16, 16, 3),
    ("head", 16, 1, 1),
]


def init_params(seed=0, dtype=np.float64):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co, k in LAYERS:
        std = np.sqrt(2.0 / (ci * k * k))
        if name == "head":
            std = 0.1 / np.sqrt(ci)
        p[name + ".w"] = (std * rng.standard_normal((k, k, ci, co))).astype(dtype)
        p[name + ".b"] = np.zeros(co, dtype=dtype)
    return p


def conv(x, w, b):
    """'same' convolution, zero padding: x (N,H,W,Ci), w (k,k,Ci,Co)."""
    k = w.shape[0]
    r = k // 2
    N, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (r, r), (r, r), (0, 0)))
    out = np.zeros((N, H, W, w.shape[3]), dtype=x.dtype)
    for ky in range(k):
        for kx in range(k):
            out += xp[:, ky:ky + H, kx:kx + W, :] @ w[ky, kx]
    return out + b


def conv_backward(x, w, dy):
    """Gradients of conv w.r.t. x, w, b given dy."""
    k = w.shape[0]
    r = k // 2
    N, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (r, r), (r, r), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(k):
        for kx in range(k):
            patch = xp[:, ky:ky + H, kx:kx + W, :]
            dw[ky, kx] = np.einsum("nhwc,nhwd->cd", patch, dy)
            dxp[:, ky:ky + H, kx:kx + W, :] += dy @ w[ky, kx].T
    dx = dxp[:, r:r + H, r:r + W, :]
    db = dy.sum(axis=(0, 1, 2))
    return dx, dw, db


def pool(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_backward(dy):
    N, H, W, C = dy.shape
    return dy.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def relu(x):
    return np.maximum(x, 0.0)


def forward(p, x):
    """Returns (delta, cache).  x: (N, H, W, 4), H and W divisible by 8."""
    cache = {}

    def cr(name, h):
        z = conv(h, p[name + ".w"], p[name + ".b"])
        a = relu(z)
        cache[name] = (h, z)
        return a

    s0 = cr("e0b", cr("e0a", x))
    s1 = cr("e1b", cr("e1a", pool(s0)))
    s2 = cr("e2b", cr("e2a", pool(s1)))
    bt = cr("e3b", cr("e3a", pool(s2)))
    u2 = cr("d2b", cr("d2a", np.concatenate([s2, up(bt)], axis=3)))
    u1 = cr("d1b", cr("d1a", np.concatenate([s1, up(u2)], axis=3)))
    u0 = cr("d0b", cr("d0a", np.concatenate([s0, up(u1)], axis=3)))
    delta = conv(u0, p["head.w"], p["head.b"])
    cache["head"] = (u0, delta)
    return delta, cache


def backward(p, cache, ddelta):
    """Gradients of a loss with dL/d(delta) = ddelta, for every parameter."""
    g = {}

    def crb(name, da):
        h, z = cache[name]
        dz = da * (z > 0)
        dh, dw, db = conv_backward(h, p[name + ".w"], dz)
        g[name + ".w"], g[name + ".b"] = dw, db
        return dh

    u0, _ = cache["head"]
    du0, g["head.w"], g["head.b"] = conv_backward(u0, p["head.w"], ddelta)
    dc0 = crb("d0a", crb("d0b", du0))
    ds0 = dc0[..., :16]
    du1 = up_backward(dc0[..., 16:])
    dc1 = crb("d1a", crb("d1b", du1))
    ds1 = dc1[..., :32]
    du2 = up_backward(dc1[..., 32:])
    dc2 = crb("d2a", crb("d2b", du2))
    ds2 = dc2[..., :64]
    dbt = up_backward(dc2[..., 64:])
    dp2 = crb("e3a", crb("e3b", dbt))
    ds2 = ds2 + pool_backward(dp2)
    dp1 = crb("e2a", crb("e2b", ds2))
    ds1 = ds1 + pool_backward(dp1)
    dp0 = crb("e1a", crb("e1b", ds1))
    ds0 = ds0 + pool_backward(dp0)
    dx = crb("e0a", crb("e0b", ds0))
    return g, dx


def mse_loss(delta, target):
    d = delta - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def energy_loss(delta, target, feats):
    """Energy-norm loss of the guess error, and its gradient in delta.

    With E = exp(f0) (E^n up to the image's scale) and the face coefficients
    alpha_x = expm1(4 f2), alpha_y = expm1(4 f3) read back from the
    features, the guess E (1 + delta) misses the solve E (1 + target) by
    e = E (delta - target), whose energy norm under the backward-Euler
    operator A = I + sum_faces alpha (difference)^2 is
        |e|_A^2 = sum_i e_i^2 + sum_faces alpha_f (e_left - e_right)^2.
    The loss is the mean over images of |e|_A^2 / |e0|_A^2, e0 = E target
    being the error of the plain guess E^n.  A face exists between a pixel
    and its +x (+y) neighbour inside the image (no wrap).
    delta, target: (N, H, W, 1); feats: (N, H, W, 4).
    """
    E = np.exp(feats[..., 0])
    ax = np.expm1(4.0 * feats[..., 2])
    ay = np.expm1(4.0 * feats[..., 3])
    d = delta[..., 0]
    t = target[..., 0]
    e = E * (d - t)
    e0 = E * t

    def quad(v):
        q = np.sum(v * v, axis=(1, 2))
        q = q + np.sum(ax[:, :, :-1] * (v[:, :, :-1] - v[:, :, 1:]) ** 2,
                       axis=(1, 2))
        q = q + np.sum(ay[:, :-1, :] * (v[:, :-1, :] - v[:, 1:, :]) ** 2,
                       axis=(1, 2))
        return q

    def apply_A(v):
        out = v.copy()
        fx = ax[:, :, :-1] * (v[:, :, :-1] - v[:, :, 1:])
        out[:, :, :-1] += fx
        out[:, :, 1:] -= fx
        fy = ay[:, :-1, :] * (v[:, :-1, :] - v[:, 1:, :])
        out[:, :-1, :] += fy
        out[:, 1:, :] -= fy
        return out

    num, den = quad(e), quad(e0)
    N = delta.shape[0]
    loss = float(np.mean(num / den))
    grad = 2.0 * E * apply_A(e) / den[:, None, None] / N
    return loss, grad[..., None]


def features(E, rhokappa_dx, alpha_x, alpha_y):
    """Network inputs from the step's data (all float64, shape (H, W)).

    log E minus its mean over the grid, log of the optical depth of a cell,
    log(1 + alpha) of the two face coefficients (diffusion numbers), each
    scaled to order one.
    """
    lE = np.log(E)
    f0 = lE - lE.mean()
    f1 = np.log(rhokappa_dx) / 4.0
    f2 = np.log1p(alpha_x) / 4.0
    f3 = np.log1p(alpha_y) / 4.0
    return np.stack([f0, f1, f2, f3], axis=-1)[None]


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), in place."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
