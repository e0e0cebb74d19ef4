"""Oracle pins of the block-adaptive composite step (oracle/amr.py).

Reductions to the uniform grid: no refined block is the base grid's own
step; every block refined is the step of a uniform grid at half the
spacing.  Closed forms and invariants: a linear field in x with uniform D
has no flux divergence, so (A E)_i = E_i on every leaf cell away from the
walls, including the cells on both sides of a block edge (this fixes the
2/3 and 1/4 of the coarse-fine faces); the volume-weighted operator is
symmetric; the step conserves sum V E with periodic and Neumann walls; a
uniform medium at a uniform E stays there.
"""
import numpy as np
import pytest

from oracle import amr as M
from oracle import fldref as F


def _grid(blocks, bc=(F.PERIODIC, F.NEUMANN), limiter="lp", nx=16, ny=16,
          b=4):
    return M.AmrGrid(nx=nx, ny=ny, dx=1.0 / nx, dy=1.5 / ny, b=b, bc=bc,
                     blocks=list(blocks), limiter=limiter)


def _fields(grid, seed):
    rng = np.random.default_rng(seed)
    nbk = len(grid.blocks)
    s = 2 * grid.b

    def pair(lo, amp):
        return (lo + amp * rng.random((grid.ny, grid.nx)),
                lo + amp * rng.random((nbk, s, s)))
    return pair(1.0, 1.0), pair(1.0, 1.0), pair(1.0, 3.0)


def test_no_refinement_is_the_base_step():
    g = _grid([])
    (Eb, Ef), (rb, rf), (kb, kf) = _fields(g, 1)
    xb, _ = M.amr_step(g, Eb, rb, kb, Ef, rf, kf, 0.2)
    ref = F.diffusion_step(Eb, rb, kb, 0.2, g.base_problem())
    np.testing.assert_allclose(xb, ref, rtol=1e-13)


def test_everything_refined_is_the_fine_uniform_step():
    g = _grid([(bx, by) for by in range(4) for bx in range(4)])
    (Eb, Ef), (rb, rf), (kb, kf) = _fields(g, 2)
    _, xf = M.amr_step(g, Eb, rb, kb, Ef, rf, kf, 0.2)
    full = lambda f: M.fine_to_full(g, f, np.zeros((2 * g.ny, 2 * g.nx)))  # noqa: E731
    ref = F.diffusion_step(full(Ef), full(rf), full(kf), 0.2, g.fine_problem())
    np.testing.assert_allclose(M.fine_to_full(g, xf, np.zeros_like(ref)), ref,
                               rtol=1e-13)


def _linear(g, axis, slope=2.0):
    """E = 3 + slope * coordinate along `axis` on both levels."""
    cb = (np.arange((g.nx, g.ny)[axis]) + 0.5) * (g.dx, g.dy)[axis]
    cf = (np.arange(2 * (g.nx, g.ny)[axis]) + 0.5) * (g.dx, g.dy)[axis] / 2
    if axis == 0:
        Eb = np.broadcast_to(3.0 + slope * cb, (g.ny, g.nx)).copy()
        Ff = np.broadcast_to(3.0 + slope * cf, (2 * g.ny, 2 * g.nx)).copy()
    else:
        Eb = np.broadcast_to((3.0 + slope * cb)[:, None], (g.ny, g.nx)).copy()
        Ff = np.broadcast_to((3.0 + slope * cf)[:, None],
                             (2 * g.ny, 2 * g.nx)).copy()
    return Eb, M.full_to_fine(g, Ff)


def _divergence(g, Eb, Ef, dt=0.7):
    one_b, one_f = np.ones_like(Eb), np.ones_like(Ef)
    Db, Df = M.coefficients(g, Eb, one_b, 3 * one_b, Ef, one_f, 3 * one_f)
    np.testing.assert_allclose(Db, 1.0 / 9.0, rtol=1e-15)
    A, _ = M.assemble(g, Db, Df, dt)
    e = M.to_leaf(g, Eb, Ef)
    ab, af = M.from_leaf(g, A @ e - e)
    return ab, M.fine_to_full(g, af, np.zeros((2 * g.ny, 2 * g.nx)))


@pytest.mark.parametrize("axis", [0, 1])
def test_linear_field_across_block_edges(axis):
    # uniform D (diffusion limiter, uniform rho and kappa) and E linear
    # along `axis`, with a strip of refined blocks across the other axis so
    # that every block edge is normal to `axis`: every face carries the
    # same flux, so the operator leaves E unchanged on every leaf cell whose
    # faces along `axis` are not walls; this fixes the 2/3 of the fine side
    # and the 1/4 of the base side of a block edge
    strip = [(1, k) for k in range(4)] if axis == 0 else \
        [(k, 2) for k in range(4)]
    bc = (F.NEUMANN, F.PERIODIC) if axis == 0 else (F.PERIODIC, F.NEUMANN)
    g = _grid(strip, bc=bc, limiter="diffusion")
    ab, af = _divergence(g, *_linear(g, axis))
    ref = g.refined()
    inner_b = np.ones((g.ny, g.nx), dtype=bool)
    inner_f = np.ones_like(af, dtype=bool)
    if axis == 0:
        inner_b[:, [0, -1]] = inner_f[:, [0, -1]] = False
    else:
        inner_b[[0, -1], :] = inner_f[[0, -1], :] = False
    assert np.max(np.abs(ab[inner_b & ~ref])) < 1e-12
    assert np.max(np.abs(af[inner_f])) < 1e-12


def test_tangential_offset_at_a_block_edge():
    # E linear in x across one refined block: along the block's y edges the
    # coarse centre sits a quarter base cell off each fine centre along x,
    # so a fine cell there sees the flux beta (E_f - E_c) with
    # E_f - E_c = +-2 dx / 4 (the reading's two-point flux), while the two
    # fine cells of one base face cancel on the base side
    g = _grid([(1, 1)], bc=(F.NEUMANN, F.PERIODIC), limiter="diffusion")
    dt = 0.7
    ab, af = _divergence(g, *_linear(g, 0), dt=dt)
    beta = (2.0 / 3.0) * dt * (1.0 / 9.0) / (g.dy / 2) ** 2
    s = 2 * g.b
    y0, x0 = s * 1, s * 1
    for J in (y0, y0 + s - 1):  # the fine rows along the y edges
        for I in range(x0 + 1, x0 + s - 1):
            sign = 1.0 if I % 2 else -1.0  # right or left half of a base cell
            assert af[J, I] == pytest.approx(beta * sign * 2.0 * g.dx / 4,
                                             rel=1e-12)
    rows = [g.b - 1, 2 * g.b]  # base rows below and above the block
    assert np.max(np.abs(ab[rows][:, g.b + 1:2 * g.b - 1])) < 1e-12


def test_volume_weighted_operator_is_symmetric():
    g = _grid([(1, 1), (2, 1), (1, 3)], bc=(F.PERIODIC, F.PERIODIC))
    (Eb, Ef), (rb, rf), (kb, kf) = _fields(g, 3)
    Db, Df = M.coefficients(g, Eb, rb, kb, Ef, rf, kf)
    A, vol = M.assemble(g, Db, Df, 0.3)
    S = (sp_diag(vol) @ A).toarray()
    np.testing.assert_allclose(S, S.T, rtol=1e-13, atol=0)


def sp_diag(v):
    import scipy.sparse as sp
    return sp.diags(v)


@pytest.mark.parametrize("bc", [(F.PERIODIC, F.NEUMANN),
                                (F.NEUMANN, F.NEUMANN)])
def test_energy_is_conserved(bc):
    g = _grid([(0, 0), (1, 0), (2, 3)], bc=bc, limiter="minerbo")
    (Eb, Ef), (rb, rf), (kb, kf) = _fields(g, 4)
    xb, xf = M.amr_step(g, Eb, rb, kb, Ef, rf, kf, 0.5)
    _, vol = M.assemble(g, *M.coefficients(g, Eb, rb, kb, Ef, rf, kf), 0.5)
    before = vol @ M.to_leaf(g, Eb, Ef)
    after = vol @ M.to_leaf(g, xb, xf)
    assert after == pytest.approx(before, rel=1e-13)
    assert np.max(np.abs(M.to_leaf(g, xb, xf) - M.to_leaf(g, Eb, Ef))) > 1e-3


def test_uniform_state_stays():
    g = _grid([(1, 2), (2, 2)])
    Eb = np.full((g.ny, g.nx), 2.5)
    Ef = np.full((2, 2 * g.b, 2 * g.b), 2.5)
    xb, xf = M.amr_step(g, Eb, Eb, Eb, Ef, Ef, Ef, 3.0)
    np.testing.assert_allclose(xb, 2.5, rtol=1e-13)
    np.testing.assert_allclose(xf, 2.5, rtol=1e-13)


def test_covered_base_values_do_not_matter():
    # the base cells under refined blocks are not unknowns: their base
    # view is the mean of the fine children, whatever the input holds
    g = _grid([(1, 1), (2, 1)])
    (Eb, Ef), (rb, rf), (kb, kf) = _fields(g, 5)
    x0 = M.amr_step(g, Eb, rb, kb, Ef, rf, kf, 0.4)
    ref = g.refined()
    Eb2 = np.where(ref, 7.0 * Eb, Eb)
    x1 = M.amr_step(g, Eb2, rb, kb, Ef, rf, kf, 0.4)
    np.testing.assert_array_equal(x0[0], x1[0])
    np.testing.assert_array_equal(x0[1], x1[1])


# ---- deeper hierarchies (hier_*) ------------------------------------------

def _hier_fields(g, levels, seed, lo=1.0):
    rng = np.random.default_rng(seed)
    s = 2 * g.b
    out = []
    for amp in (1.0, 1.0, 3.0):
        f = [lo + amp * rng.random((g.ny, g.nx))]
        f += [lo + amp * rng.random((len(bl), s, s)) for bl in levels]
        out.append(f)
    return out


def test_one_level_hierarchy_is_the_one_level_step():
    g = _grid([(1, 1), (2, 1), (0, 3)])
    (Eb, Ef), (rb, rf), (kb, kf) = _fields(g, 21)
    x1 = M.amr_step(g, Eb, rb, kb, Ef, rf, kf, 0.3)
    x2 = M.hier_step(g, [g.blocks], [Eb, Ef], [rb, rf], [kb, kf], 0.3)
    np.testing.assert_array_equal(x1[0], x2[0])
    np.testing.assert_array_equal(x1[1], x2[1])


def test_two_levels_everything_refined_is_the_uniform_step_at_4x():
    g = _grid([], nx=8, ny=8, b=4)
    lv1 = [(i, j) for j in range(2) for i in range(2)]
    lv2 = [(i, j) for j in range(4) for i in range(4)]
    E, rho, kap = _hier_fields(g, [lv1, lv2], 22)
    x = M.hier_step(g, [lv1, lv2], E, rho, kap, 0.05)
    z = np.zeros((32, 32))
    full = lambda a: M.blocks_to_full(g, lv2, a, z)  # noqa: E731
    ref = F.diffusion_step(full(E[2]), full(rho[2]), full(kap[2]), 0.05,
                           M.level_problem(g, 2))
    np.testing.assert_allclose(full(x[2]), ref, rtol=1e-12)


@pytest.mark.parametrize("axis", [0, 1])
def test_linear_field_across_two_levels_of_edges(axis):
    # strips across the other axis at both levels: every edge is normal to
    # `axis`; uniform D and a linear E give no flux divergence off the walls
    g = _grid([], bc=(F.NEUMANN, F.PERIODIC) if axis == 0 else
              (F.PERIODIC, F.NEUMANN), limiter="diffusion")
    if axis == 0:
        lv1 = [(1, k) for k in range(4)] + [(2, k) for k in range(4)]
        lv2 = [(3, k) for k in range(8)]   # inside level-1 column 1
    else:
        lv1 = [(k, 1) for k in range(4)] + [(k, 2) for k in range(4)]
        lv2 = [(k, 3) for k in range(8)]
    levels = [lv1, lv2]
    fields = []
    for f in (lambda c: 3.0 + 2.0 * c, lambda c: 1.0 + 0.0 * c,
              lambda c: 3.0 + 0.0 * c):
        per_level = []
        for l in range(3):
            ny, nx = M.level_lattice(g, l)
            h = (g.dx, g.dy)[axis] / (1 << l)
            c = (np.arange((nx, ny)[axis]) + 0.5) * h
            full = np.broadcast_to(f(c) if axis == 0 else f(c)[:, None],
                                   (ny, nx)).copy()
            per_level.append(full if l == 0 else
                             M.full_to_blocks(g, levels[l - 1], full))
        fields.append(per_level)
    E, rho, kap = fields
    D = M.hier_coefficients(g, levels, E, rho, kap)
    A, _ = M.hier_assemble(g, levels, D, 0.7)
    e = M.hier_to_leaf(g, levels, E)
    div = A @ e - e
    idx, _ = M.hier_numbering(g, levels)
    for l in range(3):
        ny, nx = idx[l].shape
        inner = np.ones((ny, nx), dtype=bool)
        if axis == 0:
            inner[:, [0, -1]] = False
        else:
            inner[[0, -1], :] = False
        m = (idx[l] >= 0) & inner
        assert np.max(np.abs(div[idx[l][m]])) < 1e-11, l


def test_two_levels_conserve_and_are_symmetric():
    g = _grid([], bc=(F.PERIODIC, F.NEUMANN), limiter="minerbo")
    lv1 = [(1, 1), (2, 1), (1, 2)]
    # the one unit of b level-1 cells whose face neighbours all lie in
    # level-1 blocks (2:1 nesting)
    lv2 = [(3, 3)]
    E, rho, kap = _hier_fields(g, [lv1, lv2], 23)
    D = M.hier_coefficients(g, [lv1, lv2], E, rho, kap)
    A, vol = M.hier_assemble(g, [lv1, lv2], D, 0.4)
    S = (sp_diag(vol) @ A).toarray()
    np.testing.assert_allclose(S, S.T, rtol=1e-13, atol=0)
    x = M.hier_step(g, [lv1, lv2], E, rho, kap, 0.4)
    before = vol @ M.hier_to_leaf(g, [lv1, lv2], E)
    assert vol @ M.hier_to_leaf(g, [lv1, lv2], x) == pytest.approx(before,
                                                                    rel=1e-13)


def test_unbalanced_levels_are_refused():
    # a level-2 block on the edge of its level-1 block whose outside
    # neighbour is a base cell: two levels across one face
    g = _grid([])
    lv1 = [(1, 1)]
    lv2 = [(2, 2)]                      # level-1 cells 8..11: edge of block (1,1)
    E, rho, kap = _hier_fields(g, [lv1, lv2], 24)
    with pytest.raises(ValueError):
        M.hier_step(g, [lv1, lv2], E, rho, kap, 0.1)


def test_views_of_an_injected_field():
    # fields that are the base field copied down to every level: each
    # level's view (inside and outside its blocks) is that copy, so each
    # level's D is the uniform grid's D of the copied field
    g = _grid([], limiter="lp")
    lv1 = [(1, 1), (2, 1), (1, 2)]
    lv2 = [(3, 3)]
    rng = np.random.default_rng(25)
    base = [1.0 + rng.random((g.ny, g.nx)) for _ in range(3)]
    fields = []
    for f in base:
        per_level, full = [f], f
        for l, bl in enumerate((lv1, lv2), start=1):
            full = M.inject(full)
            per_level.append(M.full_to_blocks(g, bl, full))
        fields.append(per_level)
    D = M.hier_coefficients(g, [lv1, lv2], *fields)
    full = [f for f in base]
    for l in (1, 2):
        full = [M.inject(f) for f in full]
        ref, _, _ = F.diffusion_coefficient(*full, M.level_problem(g, l))
        np.testing.assert_allclose(D[l], ref, rtol=1e-14)
