"""Batched grids: one launch per phase over many independent grids.

Each grid of a batch must get what the single-grid entry points give it
(same operator and stop test), and the captured hipGraph must replay the
same work: every replay is compared with an eager batched step, with other
eager work on the stream in between.
"""
import numpy as np
import pytest

import media
from oracle import fldref as F
from gpu_common import announce, dev, host, params_for, rel_l2

pytestmark = pytest.mark.gpu

SIDES = [128, 192, 256, 160, 384]


def _media():
    ms = media.config_c4(count=len(SIDES), sides=SIDES)
    for m in ms:
        prob = F.problem_from_medium(m)
        m.kappa = F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
    return ms


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_batch_matches_single_grids(precision):
    from paper_2503_02764_amd import fld
    ms = _media()
    announce(f"batch vs single {precision}")
    params = [params_for(m, rtol=1e-11, precision=precision, max_cycles=200)
              for m in ms]
    bctx = fld.fld_setup_batch(params)
    rho = [dev(m.rho) for m in ms]
    kap = [dev(m.kappa) for m in ms]
    E = [dev(m.E) for m in ms]
    out = [dev(np.zeros_like(m.E)) for m in ms]
    st, stats = fld.fld_step_batch(bctx, [m.dt for m in ms], rho, kap, E, out)
    for g, m in enumerate(ms):
        assert stats[g]["rel_res_final"] <= 1e-11, (g, stats[g])
        ctx = fld.fld_setup(params[g])
        o1 = dev(np.zeros_like(m.E))
        fld.fld_step(ctx, m.dt, rho[g], kap[g], E[g], o1)
        assert rel_l2(host(out[g]), host(o1)) <= 1e-10, g
    # the oracle on the two smallest grids
    for g in (0, 3):
        m = ms[g]
        ref = F.diffusion_step(m.E, m.rho, m.kappa, m.dt,
                               F.problem_from_medium(m))
        assert rel_l2(host(out[g]), ref) <= 1e-10, g


def test_batch_in_place_and_exchange_opacity():
    from paper_2503_02764_amd import fld
    ms = _media()
    announce("batch in place + exchange + opacity")
    params = [params_for(m, rtol=1e-10, precision="fp32_ir") for m in ms]
    bctx = fld.fld_setup_batch(params)
    rho = [dev(m.rho) for m in ms]
    e = [dev(m.e) for m in ms]
    E = [dev(m.E) for m in ms]
    kap = [dev(np.zeros_like(m.E)) for m in ms]
    o = ms[0].opacity
    fld.fld_opacity_powerlaw_batch(bctx, rho, e, o["k0"], o["a"], o["b"],
                                   o["kmin"], o["kmax"], kap)
    dts = [m.dt for m in ms]
    fld.fld_step_batch(bctx, dts, rho, kap, E, E)
    fld.fld_exchange_batch(bctx, dts, rho, kap, E, e)
    for g, m in enumerate(ms):
        prob = F.problem_from_medium(m)
        np.testing.assert_allclose(host(kap[g]), m.kappa, rtol=1e-13)
        En, en, Es = F.step(m.E, m.e, m.rho, prob, m.dt, kappa=m.kappa)
        assert rel_l2(host(E[g]), En) <= 1e-9, g
        assert rel_l2(host(e[g]), en) <= 1e-9, g


def test_batch_graph_replays_match_eager():
    from paper_2503_02764_amd import fld
    import torch
    ms = _media()
    announce("batch graph replays")
    params = [params_for(m, rtol=1e-8, precision="fp32_ir") for m in ms]
    dts = [m.dt for m in ms]
    eager = fld.fld_setup_batch(params)
    with pytest.raises(fld.FldError):  # the null stream cannot be captured
        fld.fld_batch_set_graph(eager, True)
    stream = torch.cuda.Stream()
    graph = fld.fld_setup_batch(params, stream=stream)
    fld.fld_batch_set_graph(graph, True)
    rho = [dev(m.rho) for m in ms]
    kap = [dev(m.kappa) for m in ms]
    Ea = [dev(m.E) for m in ms]
    Eb = [dev(m.E) for m in ms]
    for step in range(4):
        _, sa = fld.fld_step_batch(eager, dts, rho, kap, Ea, Ea)
        # unrelated eager work on the stream between replays
        junk = torch.ones(1 << 20, dtype=torch.float64, device="cuda")
        junk.mul_(3.0).sum().item()
        torch.cuda.synchronize()
        _, sb = fld.fld_step_batch(graph, dts, rho, kap, Eb, Eb)
        torch.cuda.synchronize()
        for g in range(len(ms)):
            assert np.array_equal(host(Ea[g]), host(Eb[g])), (step, g)
            assert sa[g]["cycles"] == sb[g]["cycles"]


def test_batch_rejects_bad_setups():
    from paper_2503_02764_amd import fld
    ms = _media()
    announce("batch validation")
    p3 = params_for(media.random_small_medium(1, (16, 16, 16),
                                              ("periodic",) * 3))
    with pytest.raises(fld.FldError):
        fld.fld_setup_batch([params_for(ms[0]), p3])
    tiny = params_for(media.random_small_medium(1, (16, 16),
                                                ("neumann", "neumann")))
    with pytest.raises(fld.FldError):
        fld.fld_setup_batch([tiny])


@pytest.mark.parametrize("variant", [2, 3])
def test_batch_tile_shapes_give_identical_iterates(variant, monkeypatch):
    from paper_2503_02764_amd import fld
    ms = _media()
    announce(f"batch tile shape {variant} vs 0")
    out = {}
    for v in (0, variant):
        monkeypatch.setenv("FLD_TILE_VARIANT", str(v))
        for prec in ("fp64", "fp32_ir"):
            params = [params_for(m, rtol=1e-10, precision=prec) for m in ms]
            bctx = fld.fld_setup_batch(params)
            o = [dev(np.zeros_like(m.E)) for m in ms]
            fld.fld_step_batch(bctx, [m.dt for m in ms],
                               [dev(m.rho) for m in ms],
                               [dev(m.kappa) for m in ms],
                               [dev(m.E) for m in ms], o)
            out[(v, prec)] = [host(x) for x in o]
    for prec in ("fp64", "fp32_ir"):
        for g in range(len(ms)):
            np.testing.assert_array_equal(out[(0, prec)][g],
                                          out[(variant, prec)][g],
                                          err_msg=f"{prec} grid {g}")


def test_batch_autotune_keeps_results_and_graph():
    """Tuned shapes give the same iterates; a graph captured before the
    tuning is dropped and captured again with the new launch shapes."""
    from paper_2503_02764_amd import fld
    import torch
    ms = _media()
    announce("batch autotune + graph")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        params = [params_for(m, rtol=1e-10, precision="fp32_ir") for m in ms]
        bctx = fld.fld_setup_batch(params, stream=stream)
        fld.fld_batch_set_graph(bctx, True)
        rho = [dev(m.rho) for m in ms]
        kap = [dev(m.kappa) for m in ms]
        E = [dev(m.E) for m in ms]
        dts = [m.dt for m in ms]
        out0 = [torch.zeros_like(x) for x in E]
        fld.fld_step_batch(bctx, dts, rho, kap, E, out0)
        shapes = fld.fld_autotune(bctx)
        out1 = [torch.zeros_like(x) for x in E]
        fld.fld_step_batch(bctx, dts, rho, kap, E, out1)
        stream.synchronize()
    assert shapes[0][0] != "invalid"
    for g in range(len(ms)):
        np.testing.assert_array_equal(host(out1[g]), host(out0[g]))


def test_c4_full_size_batch_configuration():
    """The 96-grid batch (36.8 M cells, sides 128..1024) in the bench's
    configuration: FP32 V-cycles in FP64 refinement, V(2,3), autotuned tile
    shapes, hipGraph replay on a stream of its own.  The oracle assembles
    each grid's operator from the same inputs and measures the GPU iterate's
    residual (<= rtol, which bounds the error against the exact solve since
    A >= I); the exchange is checked on sampled cells of every grid."""
    import torch
    import bench
    from paper_2503_02764_amd import fld
    ms = media.config_c4()
    announce("c4 full size: 96 grids, graph, autotuned")
    o = ms[0].opacity
    params = [params_for(m, rtol=1e-8, precision="fp32_ir",
                         pre_smooth=bench.PRE, post_smooth=bench.POST,
                         coarse_pre_smooth=bench.COARSE_PRE,
                         coarse_post_smooth=bench.COARSE_POST)
              for m in ms]
    dts = [m.dt for m in ms]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        bctx = fld.fld_setup_batch(params, stream=stream)
        fld.fld_batch_set_graph(bctx, True)
        fld.fld_autotune(bctx)
        rho = [dev(m.rho) for m in ms]
        e = [dev(m.e) for m in ms]
        E = [dev(m.E) for m in ms]
        kap = [dev(np.zeros_like(m.E)) for m in ms]
        out = [dev(np.zeros_like(m.E)) for m in ms]
        fld.fld_opacity_powerlaw_batch(bctx, rho, e, o["k0"], o["a"], o["b"],
                                       o["kmin"], o["kmax"], kap)
        st, stats = fld.fld_step_batch(bctx, dts, rho, kap, E, out)
        stream.synchronize()
        xs = [host(x) for x in out]
        fld.fld_exchange_batch(bctx, dts, rho, kap, out, e)
        stream.synchronize()
        e_h = [host(v) for v in e]
        out_h = [host(v) for v in out]
    rng = np.random.default_rng(2)
    for g, m in enumerate(ms):
        prob = F.problem_from_medium(m)
        k_ref = F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
        alphas = F.face_coefficients(m.E, m.rho, k_ref, m.dt, prob)
        rr = F.relative_residual(xs[g], m.E, alphas, prob)
        assert rr <= 1.0e-8 * 1.001, (g, rr, stats[g])
        assert abs(rr / stats[g]["rel_res_final"] - 1) < 1e-3, (g, rr, stats[g])
        idx = rng.choice(xs[g].size, 256, replace=False)
        x = xs[g].ravel()[idx]
        En, en = F.exchange(x, m.e.ravel()[idx], m.rho.ravel()[idx],
                            k_ref.ravel()[idx], m.dt, prob)
        S = x + m.e.ravel()[idx]
        assert np.all(np.abs(e_h[g].ravel()[idx] - en) <= 8 * np.spacing(S)), g
        assert np.all(np.abs(out_h[g].ravel()[idx] - En) <= 8 * np.spacing(S)), g
