"""Held cells (an interior boundary whose cells take a prescribed new E) on
the GPU against the oracle, through the C ABI.

The library solves the system with the held cells eliminated: a free
cell's faces to held neighbours become diagonal and right-hand-side terms
and every face touching a held cell is cut, so a held row is x = E_hold;
on the coarse levels a cell with a held child is a point of zero
correction, coupled through the faces before the cut.  Solves
run to rtol 1e-12 and must meet the oracle's direct solve to relative L2
1e-10; the held cells come out at their values bit for bit.  Masks: a band
of the first columns (the overwritten first wavelength of the linear-wave
tests), scattered cells, a block inside the grid; with Neumann, periodic
and Dirichlet walls; 1D/2D/3D, even sizes over several levels and ragged
single-level ones.
"""
import numpy as np
import pytest

import media
from oracle import fldref as F

from gpu_common import announce, dev, host, params_for, rel_l2

pytestmark = pytest.mark.gpu


def _mask(kind, shape, seed):
    m = np.zeros(shape, dtype=bool)
    if kind == "band":
        m[..., : max(1, shape[-1] // 8)] = True
    elif kind == "scatter":
        m = np.random.default_rng(seed).random(shape) < 0.15
    elif kind == "block":
        sl = tuple(slice(s // 3, max(s // 3 + 1, s // 2)) for s in shape)
        m[sl] = True
    return m


CASES = [
    ((64,), ("neumann",), "band", {}),
    ((48,), ("periodic",), "scatter", {}),
    ((7,), ("neumann",), "block", {(0, 1): 1.3}),
    ((32, 24), ("periodic", "neumann"), "band", {}),
    ((40, 40), ("neumann", "neumann"), "scatter", {(1, 0): 2.0}),
    ((13, 10), ("periodic", "neumann"), "block", {}),
    ((16, 16, 16), ("periodic", "periodic", "neumann"), "band",
     {(2, 1): 0.6}),
    ((12, 8, 10), ("neumann", "periodic", "neumann"), "scatter", {}),
    ((6, 5, 9), ("neumann", "neumann", "periodic"), "block", {}),
]


def _prob(m, walls):
    return F.Problem(ndim=m.ndim, n=tuple(m.n), dx=tuple(m.dx),
                     bc=tuple(m.bc), c=m.c, a_rad=m.a_rad, gamma=m.gamma,
                     gas_const=m.gas_const, limiter=m.limiter,
                     face_mean=m.face_mean, dirichlet=dict(walls))


def _ctx(m, walls, **kw):
    from paper_2503_02764_amd import fld
    kw.setdefault("rtol", 1e-12)
    kw.setdefault("max_cycles", 200)
    return fld.fld_setup(params_for(m, dirichlet=walls or None,
                                    held_cells=True, **kw))


def _held_dev(mask, hold):
    import torch
    return (torch.from_numpy(mask.astype(np.uint8)).cuda(), dev(hold))


def _step(ctx, m, E, mask, hold, alias=False):
    from paper_2503_02764_amd import fld
    md, hd = _held_dev(mask, hold)
    fld.fld_set_held(ctx, md, hd)
    Ed = dev(E)
    out = Ed if alias else dev(np.zeros_like(E))
    _, stats = fld.fld_step(ctx, m.dt, dev(m.rho), dev(m.kappa), Ed, out)
    return host(out), stats


@pytest.mark.parametrize("n,bc,kind,walls", CASES)
@pytest.mark.parametrize("limiter,face", [("lp", "arith"),
                                          ("minerbo", "harmonic")])
def test_held_solve_vs_oracle(n, bc, kind, walls, limiter, face):
    m = media.random_small_medium(5 * sum(n) + len(kind), n, bc, limiter,
                                  face)
    mask = _mask(kind, m.E.shape, sum(n))
    hold = 0.5 + 2.0 * np.random.default_rng(len(n)).random(m.E.shape)
    announce(f"held solve n={n} bc={bc} {kind} walls={walls} {limiter}/{face}")
    x, stats = _step(_ctx(m, walls), m, m.E, mask, hold)
    ref = F.held_step(m.E, m.rho, m.kappa, m.dt, _prob(m, walls), mask, hold,
                      method="splu")
    assert stats["rel_res_final"] <= 1e-12, stats
    np.testing.assert_array_equal(x[mask], hold[mask])
    assert rel_l2(x, ref) <= 1e-10, (stats, rel_l2(x, ref))


def test_steady_line_between_two_held_cells():
    n = 64
    m = media.random_small_medium(9, (n,), ("neumann",), "diffusion")
    m.rho = np.ones(n)
    m.kappa = np.full(n, 3.0)
    m.dt = 1e10
    mask = np.zeros(n, dtype=bool)
    mask[[0, n - 1]] = True
    hold = np.zeros(n)
    hold[0], hold[-1] = 1.0, 4.0
    announce("held steady line n=64")
    x, _ = _step(_ctx(m, {}), m, np.full(n, 2.0), mask, hold)
    # the free cells' block of A is I plus a Laplacian (eigenvalues >= 1),
    # so the error is at most the residual, rtol |b| with |b| about |x|
    np.testing.assert_allclose(x, 1.0 + 3.0 * np.arange(n) / (n - 1),
                               rtol=1e-9)


def test_moving_held_values_over_steps():
    # the first wavelength of a 256 x 64 strip held at a travelling wave
    # of E, its values renewed in place between steps (one mask, one
    # registration), each step against the oracle from the same E
    nx, ny = 256, 64
    m = media.random_small_medium(31, (nx, ny), ("neumann", "periodic"),
                                  "lp")
    m.dt = 5e-3
    ctx = _ctx(m, {(0, 1): 1.0})
    prob = _prob(m, {(0, 1): 1.0})
    mask = np.zeros(m.E.shape, dtype=bool)
    mask[:, :32] = True
    xs = (np.arange(nx) + 0.5) / nx
    md, hd = _held_dev(mask, np.ones(m.E.shape))
    from paper_2503_02764_amd import fld
    fld.fld_set_held(ctx, md, hd)
    E = m.E.copy()
    Ed, out = dev(E), dev(np.zeros_like(E))
    for k in range(4):
        hold = np.broadcast_to(1.0 + 0.3 * np.sin(8 * np.pi * (xs - 0.05 * k)),
                               E.shape).copy()
        hd.copy_(dev(hold))
        announce(f"held moving wave step {k}")
        _, stats = fld.fld_step(ctx, m.dt, dev(m.rho), dev(m.kappa), Ed, out)
        got = host(out)
        ref = F.held_step(E, m.rho, m.kappa, m.dt, prob, mask, hold,
                          method="splu")
        np.testing.assert_array_equal(got[mask], hold[mask])
        assert rel_l2(got, ref) <= 1e-10, (k, stats)
        E = got
        Ed, out = out, Ed


@pytest.mark.parametrize("guess", ["prev", "zero"])
def test_alias_and_zero_guess(guess):
    n, bc, kind, walls = CASES[4][:4]
    m = media.random_small_medium(44, n, bc, "lp")
    mask = _mask(kind, m.E.shape, 3)
    hold = np.full(m.E.shape, 1.7)
    announce(f"held alias guess={guess}")
    ctx = _ctx(m, walls, guess=guess)
    x0, _ = _step(ctx, m, m.E, mask, hold)
    x1, _ = _step(ctx, m, m.E, mask, hold, alias=True)
    np.testing.assert_array_equal(x0, x1)
    ref = F.held_step(m.E, m.rho, m.kappa, m.dt, _prob(m, walls), mask, hold)
    assert rel_l2(x0, ref) <= 1e-10


def test_band_at_512sq():
    # the first wavelength (the first 64 of 512 columns) held, stratified
    # Kramers-like medium with Neumann walls top and bottom
    nx = ny = 512
    rng = np.random.default_rng(512)
    m = media.random_small_medium(2, (nx, ny), ("periodic", "neumann"), "lp")
    y = (np.arange(ny) + 0.5) / ny
    m.rho = np.exp(-1.5 * y)[:, None] * np.exp(0.3 * rng.standard_normal((ny, nx)))
    m.kappa = 20.0 * m.rho * np.exp(0.5 * rng.standard_normal((ny, nx)))
    m.E = np.exp(0.2 * rng.standard_normal((ny, nx)))
    m.dt = 1e-3
    mask = np.zeros((ny, nx), dtype=bool)
    mask[:, :64] = True
    hold = np.broadcast_to(1.0 + 0.5 * np.sin(2 * np.pi * (np.arange(nx) + 0.5)
                                              / 64), (ny, nx)).copy()
    announce("held band 512^2")
    x, stats = _step(_ctx(m, {}), m, m.E, mask, hold)
    ref = F.held_step(m.E, m.rho, m.kappa, m.dt, _prob(m, {}), mask, hold,
                      method="splu")
    np.testing.assert_array_equal(x[mask], hold[mask])
    assert rel_l2(x, ref) <= 1e-10, (stats, rel_l2(x, ref))


def test_step_needs_the_held_cells():
    from paper_2503_02764_amd import fld
    m = media.random_small_medium(3, (16, 16), ("periodic", "neumann"))
    ctx = _ctx(m, {})
    E, out = dev(m.E), dev(np.zeros_like(m.E))
    announce("held cells missing")
    with pytest.raises(fld.FldError):
        fld.fld_step(ctx, m.dt, dev(m.rho), dev(m.kappa), E, out)
    md, hd = _held_dev(np.zeros(m.E.shape, dtype=bool), np.ones(m.E.shape))
    # one of the two pointers alone
    assert fld.load().fld_set_held(ctx.ptr, fld._ptr(md, "mask"), None) == \
        fld.FLD_ERR_INVALID_ARG
    fld.fld_set_held(ctx, md, hd)  # no cell held: the plain step
    fld.fld_step(ctx, m.dt, dev(m.rho), dev(m.kappa), E, out)
    ref = F.diffusion_step(m.E, m.rho, m.kappa, m.dt, F.problem_from_medium(m))
    assert rel_l2(host(out), ref) <= 1e-10
    fld.fld_set_held(ctx, None, None)
    with pytest.raises(fld.FldError):
        fld.fld_step(ctx, m.dt, dev(m.rho), dev(m.kappa), E, out)
    plain = fld.fld_setup(params_for(m))
    with pytest.raises(fld.FldError):
        fld.fld_set_held(plain, md, hd)
