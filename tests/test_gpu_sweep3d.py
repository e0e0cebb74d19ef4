"""Fused red-black sweeps of the 3D levels (one launch per sweep, out of
place: z-marching on large levels, 32x8x4 tiles below them) against the
two colour passes per sweep they replace, and against the oracle.

The fused kernel applies the colour-pass update to every cell in the same
order (red from old black, then black from new red), so the solves agree bit
for bit: same V-cycle count, same iterate.  FLD_SWEEP3D=0 smooths by colour
passes only; a number > 1 forces fused sweeps with that many z planes per
block on every eligible level (nx % 64 == 0, ny % 16 == 0), small ones too.
"""
import numpy as np
import pytest

import media
from oracle import fldref as F
from gpu_common import announce, dev, host, params_for, rel_l2

pytestmark = pytest.mark.gpu

SHAPES = [
    ((64, 16, 12), ("neumann", "neumann", "neumann")),
    ((128, 32, 20), ("periodic", "periodic", "periodic")),
    ((64, 48, 10), ("neumann", "neumann", "periodic")),
    ((128, 64, 34), ("periodic", "neumann", "neumann")),
    ((64, 32, 16), ("neumann", "periodic", "neumann")),
]


def _solve(m, env, monkeypatch, **kw):
    from paper_2503_02764_amd import fld
    if env is None:
        monkeypatch.delenv("FLD_SWEEP3D", raising=False)
    else:
        monkeypatch.setenv("FLD_SWEEP3D", env)
    ctx = fld.fld_setup(params_for(m, **kw))
    x = dev(np.zeros_like(m.E))
    _, st = fld.fld_step(ctx, m.dt, dev(m.rho), dev(m.kappa), dev(m.E), x)
    return host(x), st


@pytest.mark.parametrize("n,bc", SHAPES)
@pytest.mark.parametrize("cycle", [(2, 2, 0, 0), (1, 2, 4, 4)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_fused_sweeps_match_colour_passes(n, bc, cycle, precision,
                                          monkeypatch):
    m = media.random_small_medium(7 * n[2] + n[0], n, bc)
    pre, post, cpre, cpost = cycle
    kw = dict(rtol=1e-10, precision=precision, max_cycles=200,
              pre_smooth=pre, post_smooth=post, coarse_pre_smooth=cpre,
              coarse_post_smooth=cpost)
    announce(f"fused sweep {n} {bc} V{cycle} {precision}")
    x0, s0 = _solve(m, "0", monkeypatch, **kw)
    x1, s1 = _solve(m, "5", monkeypatch, **kw)  # 5 planes: ragged last chunk
    assert s1["cycles"] == s0["cycles"] and s1["rel_res_final"] <= 1e-10, (s0, s1)
    np.testing.assert_array_equal(x1, x0)


@pytest.mark.parametrize("n,bc", [SHAPES[0], SHAPES[2], SHAPES[4]])
def test_fused_sweeps_vs_oracle(n, bc, monkeypatch):
    m = media.random_small_medium(3 * n[0] + n[2], n, bc)
    announce(f"fused sweep vs oracle {n} {bc}")
    x, st = _solve(m, "4", monkeypatch, rtol=1e-12, max_cycles=300)
    ref = F.diffusion_step(m.E, m.rho, m.kappa, m.dt,
                           F.problem_from_medium(m))
    assert st["rel_res_final"] <= 1e-12
    assert rel_l2(x, ref) <= 1e-10, st


@pytest.mark.parametrize("bc", [("neumann", "neumann", "neumann"),
                                ("periodic", "periodic", "neumann")])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_default_fused_levels(bc, precision, monkeypatch):
    """The default choice (levels of at least 2^22 cells, z chunk chosen
    from the shape) on a 256x128x128 grid: the finest level takes fused
    z-marching sweeps, the levels below it tiled ones, against colour passes
    everywhere (FLD_SWEEP3D=0); FLD_TILE3D=2 takes tiled sweeps on the
    finest level too."""
    n = (256, 128, 128)
    m = media.random_small_medium(128 + len(bc[0]), n, bc)
    kw = dict(rtol=1e-10, precision=precision, max_cycles=200,
              pre_smooth=1, post_smooth=2, coarse_pre_smooth=4,
              coarse_post_smooth=4)
    announce(f"default fused 256x128x128 {bc} {precision}")
    x0, s0 = _solve(m, "0", monkeypatch, **kw)
    x1, s1 = _solve(m, None, monkeypatch, **kw)
    assert s1["cycles"] == s0["cycles"] and s1["rel_res_final"] <= 1e-10, (s0, s1)
    np.testing.assert_array_equal(x1, x0)
    monkeypatch.setenv("FLD_TILE3D", "2")
    x2, s2 = _solve(m, None, monkeypatch, **kw)
    monkeypatch.delenv("FLD_TILE3D")
    assert s2["cycles"] == s0["cycles"], (s0, s2)
    np.testing.assert_array_equal(x2, x0)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_marching_residual_restriction_matches_plane_pairs(precision,
                                                           monkeypatch):
    """The z-marching residual + restriction (the default on 3D levels)
    against the one-plane-pair kernel (FLD_RR3_PAIRS): the same residuals
    and coarse right-hand sides up to the order of the norm's partial sums,
    so the same V-cycle counts and iterates to rounding, on a periodic-z and
    a Neumann-z medium with a ragged x tile."""
    for n, bc in (((96, 40, 24), ("periodic", "neumann", "periodic")),
                  ((64, 32, 32), ("periodic", "periodic", "neumann"))):
        m = media.random_small_medium(sum(n), n, bc)
        announce(f"marching residual+restriction n={n} {precision}")
        monkeypatch.setenv("FLD_RR3_PAIRS", "1")
        x0, s0 = _solve(m, "0", monkeypatch, rtol=1e-12, max_cycles=200,
                        precision=precision)
        monkeypatch.delenv("FLD_RR3_PAIRS")
        x1, s1 = _solve(m, "0", monkeypatch, rtol=1e-12, max_cycles=200,
                        precision=precision)
        assert s0["cycles"] == s1["cycles"], (n, s0, s1)
        assert np.linalg.norm(x1 - x0) <= 1e-13 * np.linalg.norm(x0), n


@pytest.mark.parametrize("n,bc", [
    ((32, 32, 32), ("periodic", "periodic", "periodic")),
    ((40, 24, 16), ("neumann", "periodic", "neumann")),
    ((64, 32, 16), ("neumann", "periodic", "neumann")),
])
@pytest.mark.parametrize("precision,krylov", [("fp64", False), ("fp32_ir", False),
                                              ("fp32_ir", True)])
def test_small_levels_in_one_workgroup_match_colour_passes(n, bc, precision,
                                                           krylov,
                                                           monkeypatch):
    """Coarse 3D levels of at most 4096 cells above the tail run their down
    and up passes in one workgroup each (the default); FLD_LEVEL_LDS=0 runs
    them by colour passes, the residual-restriction and the prolongation
    kernels.  Same operations in the same order: the same cycle counts and
    the same iterate, bit for bit."""
    m = media.random_small_medium(sum(n) + 5, n, bc)
    kw = dict(rtol=1e-12, max_cycles=300, precision=precision, krylov=krylov,
              coarse_pre_smooth=3, coarse_post_smooth=3)
    announce(f"small levels in one workgroup n={n} {precision} krylov={krylov}")
    monkeypatch.setenv("FLD_LEVEL_LDS", "0")
    x0, s0 = _solve(m, None, monkeypatch, **kw)
    monkeypatch.delenv("FLD_LEVEL_LDS")
    x1, s1 = _solve(m, None, monkeypatch, **kw)
    assert s0["cycles"] == s1["cycles"] and s0["outer_iters"] == s1["outer_iters"]
    np.testing.assert_array_equal(x0, x1)
    assert s1["rel_res_final"] <= 1e-12


@pytest.mark.parametrize("n,bc", [
    ((128, 64, 32), ("neumann", "neumann", "neumann")),
    ((64, 32, 32), ("periodic", "periodic", "periodic")),
    ((96, 48, 40), ("neumann", "periodic", "neumann")),
    ((64, 64, 16), ("periodic", "neumann", "periodic")),
])
@pytest.mark.parametrize("precision,krylov", [("fp64", False), ("fp32_ir", False),
                                              ("fp32_ir", True)])
def test_tiled_sweeps_match_colour_passes(n, bc, precision, krylov,
                                          monkeypatch):
    """3D levels below the marching sweeps (fewer than 2^22 cells) with
    nx % 32 == ny % 8 == nz % 4 == 0 sweep by 32x8x4 tiles, one launch per
    sweep (the default); FLD_TILE3D=0 takes two colour passes per sweep.
    Same operations in the same order: the same cycle counts and the same
    iterate, bit for bit."""
    m = media.random_small_medium(2 * n[0] + n[2], n, bc)
    kw = dict(rtol=1e-11, max_cycles=300, precision=precision, krylov=krylov,
              pre_smooth=2, post_smooth=2, coarse_pre_smooth=4,
              coarse_post_smooth=4)
    announce(f"tiled 3D sweeps n={n} {bc} {precision} krylov={krylov}")
    monkeypatch.setenv("FLD_TILE3D", "0")
    x0, s0 = _solve(m, None, monkeypatch, **kw)
    monkeypatch.delenv("FLD_TILE3D")
    x1, s1 = _solve(m, None, monkeypatch, **kw)
    assert s0["cycles"] == s1["cycles"] and s0["outer_iters"] == s1["outer_iters"]
    np.testing.assert_array_equal(x0, x1)
    assert s1["rel_res_final"] <= 1e-11


@pytest.mark.parametrize("n,bc", [((64, 32, 16), ("periodic", "periodic", "periodic")),
                                  ((32, 16, 24), ("neumann", "periodic", "neumann"))])
def test_tiled_sweeps_vs_oracle(n, bc, monkeypatch):
    m = media.random_small_medium(5 + n[2], n, bc)
    announce(f"tiled 3D sweeps vs oracle {n} {bc}")
    x, st = _solve(m, None, monkeypatch, rtol=1e-12, max_cycles=300,
                   pre_smooth=2, post_smooth=2)
    ref = F.diffusion_step(m.E, m.rho, m.kappa, m.dt,
                           F.problem_from_medium(m))
    assert st["rel_res_final"] <= 1e-12
    assert rel_l2(x, ref) <= 1e-10, st
