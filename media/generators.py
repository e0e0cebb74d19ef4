"""Seeded synthetic inputs shaped like the FLD workloads.

Every field is a numpy float64 array in C order with x fastest: shape (nx,)
in 1D, (ny, nx) in 2D and (nz, ny, nx) in 3D, so that the flat index is
i + nx*(j + ny*k).  Code units: c = a_R = R_g = 1, gamma = 5/3, unit box.

Random fields come from ``grf``: white noise from numpy's PCG64
(``default_rng(seed)``) filtered in Fourier space by exp(-k^2 l^2 / 2), with
l in cells, then shifted and scaled to zero mean and unit variance.

The time step of a workload is fixed by a diffusion number nu with respect
to the optically thick diffusion coefficient c/(3 rho kappa) of the initial
state: dt = nu * dx^2 / median(c / (3 rho kappa0)).  This is part of the
input recipe (it only chooses dt); the update itself recomputes its own
flux-limited coefficients every step.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# Kramers-like opacity law of the 2D/3D workloads: kappa = k0 rho^a T^b,
# clipped to [kmin, kmax].
KRAMERS = dict(k0=1.0e2, a=1.0, b=-3.5, kmin=1.0e-2, kmax=1.0e6)

SIDES_C4 = (128, 192, 256, 384, 512, 768, 1024)


@dataclasses.dataclass
class Medium:
    """One synthetic problem: grid, constants, fields and stepping recipe."""

    ndim: int
    n: tuple  # (nx, ny, nz) with unused sides = 1
    dx: tuple  # (dx, dy, dz)
    bc: tuple  # per dimension: "periodic" or "neumann"
    rho: np.ndarray
    E: np.ndarray
    e: np.ndarray
    kappa: Optional[np.ndarray]  # None when the opacity law is used
    opacity: Optional[dict]  # Kramers parameters, or None for fixed kappa
    dt: float
    steps: int
    rtol: float
    c: float = 1.0
    a_rad: float = 1.0
    gamma: float = 5.0 / 3.0
    gas_const: float = 1.0
    limiter: str = "lp"  # "lp" (Levermore-Pomraning), "diffusion" (1/3) or
    #                      "minerbo"
    face_mean: str = "arith"  # "arith" or "harmonic"
    name: str = ""

    @property
    def shape(self):
        return self.rho.shape

    @property
    def cells(self):
        return int(self.rho.size)


def grf(shape, ell, rng):
    """Gaussian random field, correlation length ``ell`` cells, unit variance.

    Periodic by construction (filtered white noise on the full grid).
    """
    w = rng.standard_normal(shape)
    f = np.fft.fftn(w)
    k2 = np.zeros(shape)
    for ax, n in enumerate(shape):
        k = 2.0 * np.pi * np.fft.fftfreq(n)
        sh = [1] * len(shape)
        sh[ax] = n
        k2 = k2 + (k.reshape(sh)) ** 2
    f *= np.exp(-0.5 * k2 * ell * ell)
    g = np.real(np.fft.ifftn(f))
    g -= g.mean()
    s = g.std()
    return g / s if s > 0 else g


def _temperature_gas(e, rho, gamma, gas_const):
    return (gamma - 1.0) * e / (rho * gas_const)


def _kramers(rho, T, p):
    return np.clip(p["k0"] * rho ** p["a"] * T ** p["b"], p["kmin"], p["kmax"])


def _dt_from_nu(nu, dx, rho, kappa, c):
    d_thick = c / (3.0 * rho * kappa)
    return float(nu * dx * dx / np.median(d_thick))


def config_c1():
    """1D, 512 cells on [-0.5, 0.5], rho = 1, kappa = 1e3, periodic.

    E = 1 + 10 exp(-x^2 / (2 * 0.02^2)), gas in equilibrium T_gas = T_rad,
    diffusion number 100 w.r.t. c/(3 rho kappa), 10 steps to 1e-10.
    """
    n = 512
    dx = 1.0 / n
    x = -0.5 + (np.arange(n) + 0.5) * dx
    rho = np.ones(n)
    kappa = np.full(n, 1.0e3)
    E = 1.0 + 10.0 * np.exp(-x * x / (2.0 * 0.02 ** 2))
    T = E ** 0.25
    gamma = 5.0 / 3.0
    e = rho * T / (gamma - 1.0)
    dt = _dt_from_nu(100.0, dx, rho, kappa, 1.0)
    return Medium(ndim=1, n=(n, 1, 1), dx=(dx, 1.0, 1.0), bc=("periodic",),
                  rho=rho, E=E, e=e, kappa=kappa, opacity=None, dt=dt,
                  steps=10, rtol=1e-10, name="c1-1d-512-gaussian")


def _c2_fields(n, seed, nu):
    rng = np.random.default_rng(seed)
    g1 = grf((n, n), 32.0, rng)
    g2 = grf((n, n), 32.0, rng)
    g3 = grf((n, n), 32.0, rng)
    rho = np.exp(0.5 * g1 - 0.125)
    T = 1.0 + 0.1 * g2
    E = T ** 4 * (1.0 + 0.05 * g3)
    gamma = 5.0 / 3.0
    e = rho * T / (gamma - 1.0)
    kappa0 = _kramers(rho, T, KRAMERS)
    dx = 1.0 / n
    dt = _dt_from_nu(nu, dx, rho, kappa0, 1.0)
    return rho, E, e, dt


def config_c2(n=1024, seed=2, nu=100.0, steps=100, rtol=1e-8):
    """2D n x n, log-normal rho, T = 1 + 0.1 g, Kramers kappa, Neumann."""
    rho, E, e, dt = _c2_fields(n, seed, nu)
    return Medium(ndim=2, n=(n, n, 1), dx=(1.0 / n, 1.0 / n, 1.0),
                  bc=("neumann", "neumann"), rho=rho, E=E, e=e, kappa=None,
                  opacity=dict(KRAMERS), dt=dt, steps=steps, rtol=rtol,
                  name=f"c2-2d-{n}sq-kramers-lognormal")


def config_c3(n=256, seed=3, nu=100.0, steps=50, rtol=1e-8):
    """3D n^3, rho = exp(-z/0.1), T = 1 + 0.01 g, Kramers kappa.

    Periodic in x and y, Neumann in z, radiation in equilibrium E = T^4.
    """
    rng = np.random.default_rng(seed)
    g = grf((n, n, n), 32.0, rng)
    dx = 1.0 / n
    z = (np.arange(n) + 0.5) * dx
    rho = np.broadcast_to(np.exp(-z / 0.1)[:, None, None], (n, n, n)).copy()
    T = 1.0 + 0.01 * g
    E = T ** 4
    gamma = 5.0 / 3.0
    e = rho * T / (gamma - 1.0)
    kappa0 = _kramers(rho, T, KRAMERS)
    dt = _dt_from_nu(nu, dx, rho, kappa0, 1.0)
    return Medium(ndim=3, n=(n, n, n), dx=(dx, dx, dx),
                  bc=("periodic", "periodic", "neumann"), rho=rho, E=E, e=e,
                  kappa=None, opacity=dict(KRAMERS), dt=dt, steps=steps,
                  rtol=rtol, name=f"c3-3d-{n}cube-stratified")


def c4_sides(count=96, seed=4):
    rng = np.random.default_rng(seed)
    return [int(s) for s in rng.choice(SIDES_C4, size=count)]


def config_c4(count=96, seed=4, steps=20, rtol=1e-8, sides=None):
    """``count`` independent 2D grids with C2 statistics and their own dt.

    Sides are drawn uniformly from {128, ..., 1024} with ``seed``; grid g
    uses seed 4000 + g for its fields and a diffusion number log-uniform in
    [10, 1000].
    """
    if sides is None:
        sides = c4_sides(count, seed)
    rng = np.random.default_rng(seed + 100)
    nus = np.exp(rng.uniform(np.log(10.0), np.log(1000.0), size=len(sides)))
    out = []
    for g, (n, nu) in enumerate(zip(sides, nus)):
        rho, E, e, dt = _c2_fields(n, 4000 + g, float(nu))
        out.append(Medium(ndim=2, n=(n, n, 1), dx=(1.0 / n, 1.0 / n, 1.0),
                          bc=("neumann", "neumann"), rho=rho, E=E, e=e,
                          kappa=None, opacity=dict(KRAMERS), dt=dt,
                          steps=steps, rtol=rtol, name=f"c4-grid{g}-{n}sq"))
    return out


def config_c5_train(index, n=256):
    """Training medium ``index``: C2 statistics on n^2, seed 5e6 + index.

    Diffusion number log-uniform in [10, 1000]; the box side log-uniform in
    [0.25, 1], so that the cell width spans that of the 1024^2 workload
    (1/1024) up to the unit box at n = 256 (the optical depth per cell and
    the time step scale with it; the fields keep their 32-cell correlation
    length).
    """
    rng = np.random.default_rng(5_000_000 + index)
    nu = float(np.exp(rng.uniform(np.log(10.0), np.log(1000.0))))
    box = float(np.exp(rng.uniform(np.log(0.25), 0.0)))
    rho, E, e, dt = _c2_fields(n, 5_000_000 + index, nu)
    dx = box / n
    return Medium(ndim=2, n=(n, n, 1), dx=(dx, dx, 1.0),
                  bc=("neumann", "neumann"), rho=rho, E=E, e=e, kappa=None,
                  opacity=dict(KRAMERS), dt=dt * box * box, steps=1,
                  rtol=1e-8, name=f"c5-train{index}-{n}sq")


def random_small_medium(seed, n, bc, limiter="lp", face_mean="arith",
                        contrast=1.0, dt=None):
    """Random positive rho, kappa, E on a small grid (any dimension).

    ``n`` is a tuple (nx,), (nx, ny) or (nx, ny, nz); ``bc`` gives one entry
    per dimension.  ``contrast`` scales the log-amplitude of the fields.
    """
    rng = np.random.default_rng(seed)
    ndim = len(n)
    shape = tuple(reversed(n))
    rho = np.exp(contrast * 0.5 * rng.standard_normal(shape))
    kappa = np.exp(contrast * 1.0 * rng.standard_normal(shape)) * 20.0
    E = np.exp(contrast * 0.4 * rng.standard_normal(shape))
    gamma = 5.0 / 3.0
    T = np.exp(0.1 * rng.standard_normal(shape))
    e = rho * T / (gamma - 1.0)
    nn = tuple(list(n) + [1] * (3 - ndim))
    dx = tuple([1.0 / v for v in n] + [1.0] * (3 - ndim))
    if dt is None:
        dt = _dt_from_nu(float(np.exp(rng.uniform(0.0, np.log(300.0)))),
                         dx[0], rho, kappa, 1.0)
    return Medium(ndim=ndim, n=nn, dx=dx, bc=tuple(bc), rho=rho, E=E, e=e,
                  kappa=kappa, opacity=None, dt=dt, steps=1, rtol=1e-12,
                  limiter=limiter, face_mean=face_mean,
                  name=f"rand{seed}-{'x'.join(map(str, n))}")


def velocity_field(shape, ndim, seed, amplitude=0.1, ell=16.0):
    """Gas velocity for the explicit source terms: ndim components (x, y, z
    order), each amplitude * grf(shape, ell) from its own stream of `seed`.
    The update does not evolve v; it only differentiates it."""
    rng = np.random.default_rng(seed)
    return [amplitude * grf(tuple(shape), ell, rng) for _ in range(ndim)]


def _bilinear_up(f):
    """Fine-lattice values of a base field: 9/16 of the parent, 3/16 of the
    two edge neighbours towards the fine cell, 1/16 of the corner one
    (zero-gradient ghosts at the edges)."""
    p = np.pad(f, 1, mode="edge")
    ny, nx = f.shape
    out = np.empty((2 * ny, 2 * nx))
    for sy in (0, 1):
        for sx in (0, 1):
            oy, ox = (1 if sy else -1), (1 if sx else -1)
            c = p[1:-1, 1:-1]
            ex = p[1:-1, 1 + ox:1 + ox + nx]
            ey = p[1 + oy:1 + oy + ny, 1:-1]
            cr = p[1 + oy:1 + oy + ny, 1 + ox:1 + ox + nx]
            out[sy::2, sx::2] = (9 * c + 3 * ex + 3 * ey + cr) / 16.0
    return out


def config_amr(n=1024, b=16, frac=0.125, seed=2, nu=100.0, levels=1,
               frac_deeper=0.5):
    """The 2D n x n Kramers / log-normal medium as the base grid of a
    block-adaptive grid (b x b blocks, Neumann walls); the fraction `frac`
    of the blocks with the steepest mean |grad log E| refined; with
    `levels` > 1, on each further level the fraction `frac_deeper` of the
    steepest b x b patches of the level below whose four face-neighbouring
    patches also lie on that level (2:1 nesting) refined again.  Fine fields
    are interpolated bilinearly from the level below (rho, T, E), kappa from
    the Kramers law on each level.  Returns a dict of the grid and fields:
    `blocks` is one list of (bx, by) per refined level, the fine arrays hold
    level 1's blocks, then level 2's, ..."""
    rho, E, e, dt = _c2_fields(n, seed, nu)
    gamma = 5.0 / 3.0
    T = (gamma - 1.0) * e / rho
    s = 2 * b
    full = {"rho": rho, "T": T, "E": E}
    present = np.ones((n, n), dtype=bool)
    all_blocks, parts = [], {"rho": [], "T": [], "E": []}
    for lev in range(1, levels + 1):
        m = n << (lev - 1)  # the lattice being refined
        gy, gx = np.gradient(np.log(full["E"]))
        steep = np.sqrt(gx * gx + gy * gy) * m
        ub = m // b
        score = steep.reshape(ub, b, ub, b).mean(axis=(1, 3))
        inside = present.reshape(ub, b, ub, b).all(axis=(1, 3))
        if lev == 1:
            ok = inside
            k = int(round(frac * ub * ub))
        else:
            pad = np.pad(inside, 1, constant_values=True)  # walls end it
            ok = inside & pad[:-2, 1:-1] & pad[2:, 1:-1] & pad[1:-1, :-2] \
                & pad[1:-1, 2:]
            k = int(round(frac_deeper * np.count_nonzero(ok)))
        cand = np.flatnonzero(ok.ravel())
        order = cand[np.argsort(-score.ravel()[cand], kind="stable")][:k]
        blocks = sorted(((int(i % ub), int(i // ub)) for i in order),
                        key=lambda xy: (xy[1], xy[0]))
        all_blocks.append(blocks)
        up = {name: _bilinear_up(f) for name, f in full.items()}
        for name in parts:
            parts[name].append(np.stack(
                [up[name][by * s:(by + 1) * s, bx * s:(bx + 1) * s]
                 for bx, by in blocks]))
        present = np.zeros((2 * m, 2 * m), dtype=bool)
        for bx, by in blocks:
            present[by * s:(by + 1) * s, bx * s:(bx + 1) * s] = True
        full = up
    rho_f = np.concatenate(parts["rho"])
    T_f = np.concatenate(parts["T"])
    E_f = np.concatenate(parts["E"])
    counts = "-".join(str(len(bl)) for bl in all_blocks)
    return dict(n=n, b=b, blocks=all_blocks[0] if levels == 1 else all_blocks,
                dx=1.0 / n, dt=dt, bc=("neumann", "neumann"),
                rho_b=rho, E_b=E, kappa_b=_kramers(rho, T, KRAMERS),
                rho_f=rho_f, E_f=E_f, kappa_f=_kramers(rho_f, T_f, KRAMERS),
                name=f"amr-2d-{n}sq-base-b{b}-{counts}-refined-blocks")
