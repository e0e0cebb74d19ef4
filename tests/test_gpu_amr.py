"""Block-adaptive 2D step on the GPU (fld_amr_*) against the oracle's
direct solve of the composite system (oracle/amr.py), through the C ABI.

The solve runs to a volume-weighted relative residual of 1e-12; in that
norm the composite operator (identity plus a positive semi-definite
diffusion part) has eigenvalues >= 1, so the error is at most the residual
and the leaf values must meet the oracle's to relative L2 1e-10.  Cases:
one block, neighbouring blocks, a strip, blocks across the periodic seams
and on the walls; all three limiters; everything refined (the uniform fine
grid) and nothing refined (the base grid); conservation of sum V E; in
place and from a zero guess; a 256 x 256 base with a refined band.
"""
import numpy as np
import pytest

from oracle import amr as M
from oracle import fldref as F

from gpu_common import announce, dev, host, rel_l2

pytestmark = pytest.mark.gpu


def _params(g, **kw):
    from paper_2503_02764_amd.solver import make_params
    bc = tuple("periodic" if b == F.PERIODIC else "neumann" for b in g.bc)
    kw.setdefault("rtol", 1e-12)
    kw.setdefault("max_cycles", 400)
    return make_params(2, (g.nx, g.ny), (g.dx, g.dy), bc, c=g.c,
                       limiter=g.limiter, face_mean=g.face_mean, **kw)


def _medium(g, seed, contrast=1.0):
    rng = np.random.default_rng(seed)
    s = 2 * g.b
    nb = len(g.blocks)

    def pair(scale, amp):
        return (scale * np.exp(amp * contrast * rng.standard_normal((g.ny, g.nx))),
                scale * np.exp(amp * contrast * rng.standard_normal((nb, s, s))))
    return pair(1.0, 0.3), pair(1.0, 0.4), pair(20.0, 0.8)


def _run(g, fields, dt, **kw):
    from paper_2503_02764_amd import fld
    (Eb, Ef), (rb, rf), (kb, kf) = fields
    ctx = fld.fld_amr_setup(_params(g, **kw), g.b, g.blocks)
    out_b = dev(np.zeros_like(Eb))
    out_f = dev(np.zeros_like(Ef)) if Ef.size else dev(np.zeros(1))[:0]
    ef = dev(Ef) if Ef.size else dev(np.zeros(1))[:0]
    rf_, kf_ = (dev(rf), dev(kf)) if Ef.size else (ef, ef)
    _, stats = fld.fld_amr_step(ctx, dt, dev(rb), dev(kb), dev(Eb), out_b,
                                rf_, kf_, ef, out_f)
    return host(out_b), host(out_f), stats


def _check(g, fields, dt, tol=1e-10, **kw):
    xb, xf, stats = _run(g, fields, dt, **kw)
    (Eb, Ef), (rb, rf), (kb, kf) = fields
    rb_, rf_ = M.amr_step(g, Eb, rb, kb, Ef, rf, kf, dt)
    got, ref = M.to_leaf(g, xb, xf), M.to_leaf(g, rb_, rf_)
    assert stats["rel_res_final"] <= 1e-12, stats
    assert rel_l2(got, ref) <= tol, (stats, rel_l2(got, ref))
    # covered base cells: the mean of their children
    ref_mask = g.refined()
    np.testing.assert_allclose(xb[ref_mask], rb_[ref_mask], rtol=1e-9)
    return got, ref, stats


CASES = [
    ("one", [(1, 1)], (F.PERIODIC, F.NEUMANN)),
    ("pair", [(1, 1), (2, 1)], (F.NEUMANN, F.NEUMANN)),
    ("strip", [(1, k) for k in range(4)], (F.NEUMANN, F.PERIODIC)),
    ("seams", [(0, 0), (3, 0), (0, 3), (3, 3)], (F.PERIODIC, F.PERIODIC)),
    ("walls", [(0, 1), (3, 2), (2, 0)], (F.NEUMANN, F.NEUMANN)),
]


@pytest.mark.parametrize("name,blocks,bc", CASES)
@pytest.mark.parametrize("limiter", ["lp", "minerbo", "diffusion"])
def test_amr_step_vs_oracle(name, blocks, bc, limiter):
    g = M.AmrGrid(nx=32, ny=32, dx=1.0 / 32, dy=1.0 / 32, b=8, bc=bc,
                  blocks=blocks, limiter=limiter)
    announce(f"amr step {name} {limiter}")
    _check(g, _medium(g, len(name) + len(limiter)), 0.02)


@pytest.mark.parametrize("dt", [1e-4, 1.0])
def test_amr_step_time_steps(dt):
    # from nearly the identity to far beyond the diffusion time
    g = M.AmrGrid(nx=24, ny=16, dx=1.0 / 24, dy=1.0 / 24, b=4,
                  bc=(F.PERIODIC, F.NEUMANN),
                  blocks=[(1, 1), (2, 1), (4, 3)], limiter="lp")
    announce(f"amr step dt={dt}")
    _check(g, _medium(g, 7), dt)


def test_nothing_and_everything_refined():
    g0 = M.AmrGrid(nx=16, ny=16, dx=1 / 16, dy=1 / 16, b=4,
                   bc=(F.PERIODIC, F.NEUMANN), blocks=[])
    f0 = _medium(g0, 3)
    announce("amr nothing refined")
    xb, _, _ = _run(g0, f0, 0.05)
    (Eb, _), (rb, _), (kb, _) = f0
    ref = F.diffusion_step(Eb, rb, kb, 0.05, g0.base_problem())
    assert rel_l2(xb, ref) <= 1e-10
    g1 = M.AmrGrid(nx=16, ny=16, dx=1 / 16, dy=1 / 16, b=4,
                   bc=(F.PERIODIC, F.NEUMANN),
                   blocks=[(i, j) for j in range(4) for i in range(4)])
    f1 = _medium(g1, 4)
    announce("amr everything refined")
    _, xf, _ = _run(g1, f1, 0.05)
    (_, Ef), (_, rf), (_, kf) = f1
    z = np.zeros((32, 32))
    full = lambda a: M.fine_to_full(g1, a, z)  # noqa: E731
    ref = F.diffusion_step(full(Ef), full(rf), full(kf), 0.05,
                           g1.fine_problem())
    assert rel_l2(full(xf), ref) <= 1e-10


def test_conservation_in_place_and_zero_guess():
    from paper_2503_02764_amd import fld
    g = M.AmrGrid(nx=32, ny=32, dx=1 / 32, dy=1 / 32, b=8,
                  bc=(F.PERIODIC, F.PERIODIC), blocks=[(1, 1), (1, 2), (2, 2)],
                  limiter="minerbo")
    fields = _medium(g, 9)
    (Eb, Ef), (rb, rf), (kb, kf) = fields
    announce("amr conservation / in place / zero guess")
    got, ref, _ = _check(g, fields, 0.05)
    _, vol = M.assemble(g, *M.coefficients(g, Eb, rb, kb, Ef, rf, kf), 0.05)
    e0 = M.to_leaf(g, Eb, Ef)
    assert vol @ got == pytest.approx(vol @ e0, rel=1e-11)
    ctx = fld.fld_amr_setup(_params(g), g.b, g.blocks)
    eb, ef = dev(Eb), dev(Ef)
    fld.fld_amr_step(ctx, 0.05, dev(rb), dev(kb), eb, eb, dev(rf), dev(kf),
                     ef, ef)
    np.testing.assert_allclose(M.to_leaf(g, host(eb), host(ef)), got,
                               rtol=1e-13)
    _check(g, fields, 0.05, guess="zero")


def test_band_at_256sq():
    # a refined band around a front of E across a 256 x 256 base (16 x 16
    # blocks of 16 base cells; 3 rows of blocks refined)
    nx = 256
    blocks = [(i, j) for j in (7, 8, 9) for i in range(16)]
    g = M.AmrGrid(nx=nx, ny=nx, dx=1 / nx, dy=1 / nx, b=16,
                  bc=(F.PERIODIC, F.NEUMANN), blocks=blocks, limiter="lp")
    rng = np.random.default_rng(256)
    s = 2 * g.b
    yb = (np.arange(nx) + 0.5) / nx
    yf = (np.arange(2 * nx) + 0.5) / (2 * nx)
    front = lambda y: 1.0 + 9.0 / (1.0 + np.exp((y - 0.5) / 0.02))  # noqa: E731
    Eb = np.broadcast_to(front(yb)[:, None], (nx, nx)).copy()
    Ef = M.full_to_fine(g, np.broadcast_to(front(yf)[:, None],
                                           (2 * nx, 2 * nx)).copy())
    rb = np.exp(0.3 * rng.standard_normal((nx, nx)))
    rf = np.exp(0.3 * rng.standard_normal((len(blocks), s, s)))
    kb = 20.0 * np.exp(0.5 * rng.standard_normal((nx, nx)))
    kf = 20.0 * np.exp(0.5 * rng.standard_normal((len(blocks), s, s)))
    announce("amr band 256^2")
    _check(g, ((Eb, Ef), (rb, rf), (kb, kf)), 2e-4)


def test_errors():
    from paper_2503_02764_amd import fld
    g = M.AmrGrid(nx=16, ny=16, dx=1 / 16, dy=1 / 16, b=4,
                  bc=(F.PERIODIC, F.NEUMANN), blocks=[(1, 1)])
    (Eb, Ef), (rb, rf), (kb, kf) = _medium(g, 2)
    ctx = fld.fld_amr_setup(_params(g), g.b, g.blocks)
    bad = Eb.copy()
    bad[3, 3] = -1.0
    announce("amr nonphysical input")
    st, _ = fld.fld_amr_step(ctx, 0.1, dev(rb), dev(kb), dev(bad),
                             dev(np.zeros_like(Eb)), dev(rf), dev(kf),
                             dev(Ef), dev(np.zeros_like(Ef)), check=False)
    assert st == fld.FLD_ERR_NONPHYSICAL
    with pytest.raises(fld.FldError):
        fld.fld_amr_step(ctx, -1.0, dev(rb), dev(kb), dev(Eb),
                         dev(np.zeros_like(Eb)), dev(rf), dev(kf), dev(Ef),
                         dev(np.zeros_like(Ef)))


def test_bench_workload_full_size():
    # the block-adaptive bench workload (1024^2 base, 512 refined blocks of
    # 16^2 base cells, 1.44 M leaf cells) in the bench's configuration: the
    # oracle's own composite operator, assembled from the same inputs,
    # judges the GPU's iterate (its relative residual bounds the relative
    # error, the operator's eigenvalues being >= 1 in the volume norm)
    import media
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import make_params
    w = media.config_amr()
    n, b = w["n"], w["b"]
    g = M.AmrGrid(nx=n, ny=n, dx=w["dx"], dy=w["dx"], b=b,
                  bc=(F.NEUMANN, F.NEUMANN), blocks=w["blocks"])
    p = make_params(2, (n, n), (w["dx"], w["dx"]), w["bc"], rtol=1e-8,
                    pre_smooth=1, post_smooth=1, max_cycles=200)
    ctx = fld.fld_amr_setup(p, b, w["blocks"])
    ob, of = dev(np.zeros_like(w["E_b"])), dev(np.zeros_like(w["E_f"]))
    announce("amr bench workload 1024^2 base")
    _, stats = fld.fld_amr_step(ctx, w["dt"], dev(w["rho_b"]),
                                dev(w["kappa_b"]), dev(w["E_b"]), ob,
                                dev(w["rho_f"]), dev(w["kappa_f"]),
                                dev(w["E_f"]), of)
    Db, Df = M.coefficients(g, w["E_b"], w["rho_b"], w["kappa_b"], w["E_f"],
                            w["rho_f"], w["kappa_f"])
    A, vol = M.assemble(g, Db, Df, w["dt"])
    x = M.to_leaf(g, host(ob), host(of))
    bvec = M.to_leaf(g, w["E_b"], w["E_f"])
    r = bvec - A @ x
    rel = np.sqrt(vol @ (r * r) / (vol @ (bvec * bvec)))
    assert stats["rel_res_final"] <= 1e-8, stats
    assert rel <= 2e-8, (rel, stats)
    assert vol @ x == pytest.approx(vol @ bvec, rel=1e-7)


def test_split_step_opacity_diffusion_exchange():
    # opacity (Kramers law) -> diffusion -> exchange on a block-adaptive
    # grid, every stage against the oracle on the same cells: the per-cell
    # stages on the base and fine arrays, the diffusion on the leaf cells
    from paper_2503_02764_amd import fld
    import media
    g = M.AmrGrid(nx=32, ny=32, dx=1 / 32, dy=1 / 32, b=8,
                  bc=(F.PERIODIC, F.NEUMANN), blocks=[(1, 1), (2, 1), (1, 2)],
                  limiter="lp")
    (Eb, Ef), (rb, rf), _ = _medium(g, 12)
    rng = np.random.default_rng(13)
    eb = rb * (1.0 + 0.1 * rng.random(rb.shape)) * 1.5
    ef = rf * (1.0 + 0.1 * rng.random(rf.shape)) * 1.5
    o = media.KRAMERS
    prob = F.Problem(ndim=2, n=(g.nx, g.ny, 1), dx=(g.dx, g.dy, 1.0),
                     bc=tuple(g.bc))
    ctx = fld.fld_amr_setup(_params(g), g.b, g.blocks)
    d = {k: dev(v) for k, v in dict(Eb=Eb, Ef=Ef, rb=rb, rf=rf, eb=eb,
                                    ef=ef).items()}
    kb, kf = dev(np.zeros_like(Eb)), dev(np.zeros_like(Ef))
    announce("amr split step")
    fld.fld_amr_opacity_powerlaw(ctx, d["rb"], d["eb"], d["rf"], d["ef"],
                                 o["k0"], o["a"], o["b"], o["kmin"], o["kmax"],
                                 kb, kf)
    kap_b = F.opacity_powerlaw(rb, eb, prob, o["k0"], o["a"], o["b"],
                               o["kmin"], o["kmax"])
    kap_f = F.opacity_powerlaw(rf, ef, prob, o["k0"], o["a"], o["b"],
                               o["kmin"], o["kmax"])
    np.testing.assert_allclose(host(kb), kap_b, rtol=1e-13)
    np.testing.assert_allclose(host(kf), kap_f, rtol=1e-13)
    dt = 0.02
    fld.fld_amr_step(ctx, dt, d["rb"], kb, d["Eb"], d["Eb"], d["rf"], kf,
                     d["Ef"], d["Ef"])
    xb, xf = M.amr_step(g, Eb, rb, kap_b, Ef, rf, kap_f, dt)
    got_b, got_f = host(d["Eb"]), host(d["Ef"])
    assert rel_l2(M.to_leaf(g, got_b, got_f), M.to_leaf(g, xb, xf)) <= 1e-10
    fld.fld_amr_exchange(ctx, dt, d["rb"], kb, d["Eb"], d["eb"], d["rf"], kf,
                         d["Ef"], d["ef"])
    for E_in, e_in, rho, kap, E_d, e_d in (
            (got_b, eb, rb, kap_b, d["Eb"], d["eb"]),
            (got_f, ef, rf, kap_f, d["Ef"], d["ef"])):
        E_ref, e_ref = F.exchange(E_in, e_in, rho, kap, dt, prob)
        np.testing.assert_allclose(host(E_d), E_ref, rtol=1e-12)
        np.testing.assert_allclose(host(e_d), e_ref, rtol=1e-12)


# ---- deeper hierarchies ----------------------------------------------------

def _hier_run(g, levels, E, rho, kap, dt, **kw):
    from paper_2503_02764_amd import fld
    cat = lambda fs: np.concatenate([f.reshape(-1) for f in fs[1:]]) \
        if len(fs) > 1 else np.zeros(0)  # noqa: E731
    ctx = fld.fld_amr_setup(_params(g, **kw), g.b, levels)
    ob = dev(np.zeros_like(E[0]))
    ef = cat(E)
    of = dev(np.zeros_like(ef))
    _, stats = fld.fld_amr_step(ctx, dt, dev(rho[0]), dev(kap[0]), dev(E[0]),
                                ob, dev(cat(rho)), dev(cat(kap)), dev(ef), of)
    out_f, k = host(of), 0
    per_level = [host(ob)]
    s = 2 * g.b
    for bl in levels:
        n = len(bl) * s * s
        per_level.append(out_f[k:k + n].reshape(len(bl), s, s))
        k += n
    return per_level, stats


def _hier_medium(g, levels, seed):
    rng = np.random.default_rng(seed)
    s = 2 * g.b
    out = []
    for scale, amp in ((1.0, 0.3), (1.0, 0.4), (20.0, 0.8)):
        f = [scale * np.exp(amp * rng.standard_normal((g.ny, g.nx)))]
        f += [scale * np.exp(amp * rng.standard_normal((len(bl), s, s)))
              for bl in levels]
        out.append(f)
    return out


@pytest.mark.parametrize("limiter", ["lp", "minerbo"])
@pytest.mark.parametrize("bc", [(F.PERIODIC, F.NEUMANN),
                                (F.NEUMANN, F.NEUMANN)])
def test_two_levels_vs_oracle(limiter, bc):
    g = M.AmrGrid(nx=32, ny=32, dx=1 / 32, dy=1 / 32, b=4, bc=bc, blocks=[],
                  limiter=limiter)
    lv1 = [(i, j) for j in range(2, 6) for i in range(2, 6)]   # base 8..23
    lv2 = [(i, j) for j in range(5, 11) for i in range(5, 11)]  # inside, 2:1
    E, rho, kap = _hier_medium(g, [lv1, lv2], 31)
    announce(f"amr two levels {limiter} {bc}")
    got, stats = _hier_run(g, [lv1, lv2], E, rho, kap, 0.02)
    ref = M.hier_step(g, [lv1, lv2], E, rho, kap, 0.02)
    assert stats["rel_res_final"] <= 1e-12, stats
    r = rel_l2(M.hier_to_leaf(g, [lv1, lv2], got),
               M.hier_to_leaf(g, [lv1, lv2], ref))
    assert r <= 1e-10, (r, stats)
    for l in (0, 1):  # cells under finer blocks: their children's mean
        np.testing.assert_allclose(got[l], ref[l], rtol=1e-9)


def test_two_levels_everything_refined_is_the_uniform_step():
    g = M.AmrGrid(nx=8, ny=8, dx=1 / 8, dy=1 / 8, b=4,
                  bc=(F.PERIODIC, F.NEUMANN), blocks=[])
    lv1 = [(i, j) for j in range(2) for i in range(2)]
    lv2 = [(i, j) for j in range(4) for i in range(4)]
    E, rho, kap = _hier_medium(g, [lv1, lv2], 32)
    announce("amr two levels everything refined")
    got, _ = _hier_run(g, [lv1, lv2], E, rho, kap, 0.01)
    z = np.zeros((32, 32))
    full = lambda a: M.blocks_to_full(g, lv2, a, z)  # noqa: E731
    ref = F.diffusion_step(full(E[2]), full(rho[2]), full(kap[2]), 0.01,
                           M.level_problem(g, 2))
    assert rel_l2(full(got[2]), ref) <= 1e-10


def test_three_levels_around_a_front():
    g = M.AmrGrid(nx=64, ny=64, dx=1 / 64, dy=1 / 64, b=8,
                  bc=(F.PERIODIC, F.NEUMANN), blocks=[], limiter="lp")
    lv1 = [(i, j) for j in (2, 3, 4, 5) for i in range(8)]        # base rows 16..47
    lv2 = [(i, j) for j in (5, 6, 7, 8, 9, 10) for i in range(16)]  # l1 rows 40..87
    lv3 = [(i, j) for j in (12, 13, 14, 15, 16, 17, 18, 19) for i in range(32)]
    levels = [lv1, lv2, lv3]
    E, rho, kap = _hier_medium(g, levels, 33)
    announce("amr three levels")
    got, stats = _hier_run(g, levels, E, rho, kap, 0.005)
    ref = M.hier_step(g, levels, E, rho, kap, 0.005)
    r = rel_l2(M.hier_to_leaf(g, levels, got), M.hier_to_leaf(g, levels, ref))
    assert stats["rel_res_final"] <= 1e-12 and r <= 1e-10, (r, stats)


def test_unbalanced_levels_are_refused():
    from paper_2503_02764_amd import fld
    g = M.AmrGrid(nx=16, ny=16, dx=1 / 16, dy=1 / 16, b=4,
                  bc=(F.PERIODIC, F.NEUMANN), blocks=[])
    p = _params(g)
    assert fld.fld_amr_workspace_bytes(p, 4, [[(1, 1)], [(2, 2)]]) == 0
    assert fld.fld_amr_workspace_bytes(p, 4, [[(1, 1)], [(5, 5)]]) == 0
    ok = [[(1, 1), (2, 1), (1, 2), (2, 2), (0, 1), (3, 1), (1, 0), (1, 3),
           (0, 2), (3, 2), (2, 0), (2, 3)], [(3, 3)]]
    assert fld.fld_amr_workspace_bytes(p, 4, ok) > 0
