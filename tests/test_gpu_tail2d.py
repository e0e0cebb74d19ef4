"""The 2D single-workgroup tail started one level higher, on a level of
1025..4096 cells (k_tail2d_big: one block of 1024 threads owning that level
as 2x2 cell blocks), against the tiled down and up passes on that level
followed by the tail from the first level of at most 1024 cells
(FLD_TAIL_BIG=0).  The same operations in the same order: the same cycle
counts and the same iterate, bit for bit.  One case is also checked
against the oracle's exact solve (Sect. 3, the implicit diffusion solve of
the radiation energy).
"""
import numpy as np
import pytest

import media
from oracle import fldref as F
from gpu_common import announce, dev, host, params_for, rel_l2

pytestmark = pytest.mark.gpu

# (shape, boundaries): the level that moves into the tail and what follows
SHAPES = [
    ((128, 128), ("neumann", "neumann")),    # 64x64 -> 32x32, 16x16, 8x8, 4x4
    ((256, 64), ("periodic", "neumann")),    # 128x32 -> 64x16, 32x8, 16x4
    ((192, 128), ("neumann", "periodic")),   # 48x32 (3 levels down) -> 24x16 ...
    ((96, 64), ("periodic", "periodic")),    # 48x32 -> 24x16, 12x8, 6x4
    ((200, 136), ("periodic", "neumann")),   # no level fits: unchanged tail
]


def _solve(m, big, monkeypatch, **kw):
    from paper_2503_02764_amd import fld
    if big:
        monkeypatch.delenv("FLD_TAIL_BIG", raising=False)
    else:
        monkeypatch.setenv("FLD_TAIL_BIG", "0")
    ctx = fld.fld_setup(params_for(m, **kw))
    x = dev(np.zeros_like(m.E))
    _, st = fld.fld_step(ctx, m.dt, dev(m.rho), dev(m.kappa), dev(m.E), x)
    return host(x), st


@pytest.mark.parametrize("n,bc", SHAPES)
@pytest.mark.parametrize("cycle", [(1, 1, 3, 3), (2, 2, 2, 2), (1, 2, 1, 1)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_big_tail_matches_tiled_level(n, bc, cycle, precision, monkeypatch):
    m = media.random_small_medium(5 * n[0] + n[1], n, bc)
    pre, post, cpre, cpost = cycle
    kw = dict(rtol=1e-11, max_cycles=300, precision=precision,
              pre_smooth=pre, post_smooth=post, coarse_pre_smooth=cpre,
              coarse_post_smooth=cpost)
    announce(f"2D tail from 4096 cells {n} {bc} V{cycle} {precision}")
    x0, s0 = _solve(m, False, monkeypatch, **kw)
    x1, s1 = _solve(m, True, monkeypatch, **kw)
    assert s0["cycles"] == s1["cycles"], (s0, s1)
    assert s0["outer_iters"] == s1["outer_iters"]
    np.testing.assert_array_equal(x0, x1)
    assert s1["rel_res_final"] <= 1e-11


@pytest.mark.parametrize("n,bc", [SHAPES[0], SHAPES[3]])
def test_big_tail_vs_oracle(n, bc, monkeypatch):
    m = media.random_small_medium(3 + n[0], n, bc)
    announce(f"2D tail from 4096 cells vs oracle {n} {bc}")
    x, st = _solve(m, True, monkeypatch, rtol=1e-12, max_cycles=300)
    ref = F.diffusion_step(m.E, m.rho, m.kappa, m.dt, F.problem_from_medium(m))
    assert st["rel_res_final"] <= 1e-12
    assert rel_l2(x, ref) <= 1e-10, st


def test_big_tail_repeated_steps_identical(monkeypatch):
    """Two contexts, three steps each, with the big tail: identical bits
    (the tail's LDS scratch and stop flag leave nothing behind)."""
    from paper_2503_02764_amd import fld
    n, bc = (128, 128), ("periodic", "neumann")
    m = media.random_small_medium(77, n, bc)
    monkeypatch.delenv("FLD_TAIL_BIG", raising=False)
    announce("2D big tail repeated steps")
    runs = []
    for _ in range(2):
        ctx = fld.fld_setup(params_for(m, rtol=1e-10, max_cycles=200,
                                       coarse_pre_smooth=3,
                                       coarse_post_smooth=3))
        E = dev(m.E)
        outs = []
        for _ in range(3):
            x = dev(np.zeros_like(m.E))
            fld.fld_step(ctx, m.dt, dev(m.rho), dev(m.kappa), E, x)
            outs.append(host(x))
            E = x
        runs.append(outs)
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a, b)
