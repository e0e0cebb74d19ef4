"""GPU path vs the FP64 oracle, through the C ABI.

Diffusion solves run to rtol 1e-12, which by lambda_min(A) >= 1 bounds the
relative error by rtol * sqrt(N) |b| / sum(b) (a factor near 1 for these
media); the bar is relative L2 <= 1e-10 against the oracle's exact solve.
The exchange is checked per cell to a few ulp of the conserved total S.
"""
import numpy as np
import pytest

import media
from oracle import fldref as F
from gpu_common import announce, dev, host, params_for, rel_l2

pytestmark = pytest.mark.gpu

TINY = [
    ((8,), ("periodic",)), ((64,), ("neumann",)), ((5,), ("periodic",)),
    ((6,), ("neumann",)), ((48,), ("periodic",)),
    ((8, 8), ("periodic", "periodic")), ((32, 32), ("neumann", "neumann")),
    ((24, 20), ("periodic", "neumann")), ((12, 7), ("neumann", "neumann")),
    ((4, 4, 4), ("periodic", "periodic", "periodic")),
    ((12, 12, 12), ("periodic", "periodic", "neumann")),
    ((8, 6, 10), ("neumann", "periodic", "neumann")),
]


def _solve_gpu(m, **kw):
    from paper_2503_02764_amd import fld
    ctx = fld.fld_setup(params_for(m, **kw))
    rho, kap, E = dev(m.rho), dev(m.kappa), dev(m.E)
    out = dev(np.zeros_like(m.E))
    st, stats = fld.fld_step(ctx, m.dt, rho, kap, E, out)
    return host(out), stats


@pytest.mark.parametrize("n,bc", TINY)
@pytest.mark.parametrize("limiter,face", [("lp", "arith"),
                                          ("diffusion", "harmonic"),
                                          ("minerbo", "arith")])
def test_tiny_solve_vs_dense(n, bc, limiter, face):
    m = media.random_small_medium(sum(n) + len(n), n, bc, limiter, face)
    announce(f"tiny solve n={n} bc={bc} {limiter}/{face}")
    x, stats = _solve_gpu(m, rtol=1e-12)
    ref = F.diffusion_step(m.E, m.rho, m.kappa, m.dt,
                           F.problem_from_medium(m), method="dense")
    assert stats["rel_res_final"] <= 1e-12
    assert rel_l2(x, ref) <= 1e-10, (stats, rel_l2(x, ref))


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_minerbo_limiter_c2_statistics_vs_oracle(precision):
    """Minerbo's limiter on a 256^2 medium of the 2D workload's statistics
    with a fifth of its opacity, so that R spans both branches of the
    limiter (R = 3/2 falls inside its range): the LDS-tiled coefficient
    stage and the solve against the oracle's sparse direct solve."""
    m = media.config_c2(n=256)
    m.limiter = "minerbo"
    prob = F.problem_from_medium(m)
    kap = 0.2 * F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
    _, R, _ = F.diffusion_coefficient(m.E, m.rho, kap, prob)
    assert R.min() < 1.5 < R.max()
    m.kappa = kap
    announce(f"minerbo c2 statistics 256^2 {precision}")
    x, stats = _solve_gpu(m, rtol=1e-12 if precision == "fp64" else 1e-10,
                          precision=precision, max_cycles=200)
    ref = F.diffusion_step(m.E, m.rho, kap, m.dt, prob, method="splu")
    assert rel_l2(x, ref) <= (1e-10 if precision == "fp64" else 1e-8), stats


@pytest.mark.parametrize("n", [128, 256])
def test_c2_media_solve_vs_oracle(n):
    from paper_2503_02764_amd import fld
    m = media.config_c2(n=n)
    prob = F.problem_from_medium(m)
    kap = F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
    announce(f"c2 media n={n}")
    ctx = fld.fld_setup(params_for(m, rtol=1e-12))
    rho, E, e = dev(m.rho), dev(m.E), dev(m.e)
    kap_d = dev(np.zeros_like(m.E))
    o = m.opacity
    fld.fld_opacity_powerlaw(ctx, rho, e, o["k0"], o["a"], o["b"], o["kmin"],
                             o["kmax"], kap_d)
    np.testing.assert_allclose(host(kap_d), kap, rtol=1e-13)
    out = dev(np.zeros_like(m.E))
    _, stats = fld.fld_step(ctx, m.dt, rho, kap_d, E, out)
    ref = F.diffusion_step(m.E, m.rho, kap, m.dt, prob)
    assert rel_l2(host(out), ref) <= 1e-10, stats
    # exchange on the same cells
    fld.fld_exchange(ctx, m.dt, rho, kap_d, out, e)
    En, en = F.exchange(ref, m.e, m.rho, kap, m.dt, prob)
    S = ref + m.e
    assert np.abs(host(e) - en).max() <= 1e-10 * S.max()


def test_c1_ten_steps_vs_oracle():
    from paper_2503_02764_amd.solver import Stepper
    m = media.config_c1()
    prob = F.problem_from_medium(m)
    announce("c1 ten steps")
    st = Stepper(params_for(m, rtol=1e-12))
    rho, kap, E, e = dev(m.rho), dev(m.kappa), dev(m.E), dev(m.e)
    En, en = m.E.copy(), m.e.copy()
    for _ in range(m.steps):
        st.step(m.dt, rho, kap, E, e)
        En, en, _ = F.step(En, en, m.rho, prob, m.dt, kappa=m.kappa)
    assert rel_l2(host(E), En) <= 1e-10
    assert rel_l2(host(e), en) <= 1e-10
    # mirror symmetry of the symmetric pulse is kept
    x = host(E)
    assert np.abs(x - x[::-1]).max() <= 1e-10 * x.max()


def test_exchange_per_cell_vs_oracle():
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import make_params
    rng = np.random.default_rng(9)
    n = 100_000
    rho = np.exp(2 * rng.standard_normal(n))
    kap = np.exp(3 * rng.standard_normal(n))
    E = np.exp(3 * rng.standard_normal(n))
    e = np.exp(3 * rng.standard_normal(n))
    prob = F.Problem(ndim=1, n=(n, 1, 1), dx=(1, 1, 1), bc=("periodic",),
                     gamma=1.4, gas_const=0.8, a_rad=1.3, c=2.0)
    announce("exchange per cell 1e5")
    ctx = fld.fld_setup(make_params(1, (n,), (1.0,), ("periodic",), c=2.0,
                                    a_rad=1.3, gamma=1.4, gas_const=0.8))
    for dt in (1e-3, 1.0, 1e3):
        Ed, ed = dev(E), dev(e)
        fld.fld_exchange(ctx, dt, dev(rho), dev(kap), Ed, ed)
        En, en = F.exchange(E, e, rho, kap, dt, prob)
        S = E + e
        assert np.all(np.abs(host(ed) - en) <= 8 * np.spacing(S)), dt
        assert np.all(np.abs(host(Ed) - En) <= 8 * np.spacing(S)), dt
        # per-cell conservation on the GPU
        assert np.all(np.abs(host(Ed) + host(ed) - S) <= 2 * np.spacing(S))


def test_equilibrium_preserved_on_gpu():
    """Uniform T_gas = T_rad with random rho, kappa: nothing moves.

    The diffusion solve needs no V-cycle and returns E^n bit for bit; the
    exchange moves each cell by at most a couple of ulp of e + E per step.
    """
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import Stepper
    n = (64, 48)
    m = media.random_small_medium(5, n, ("neumann", "periodic"))
    T = 1.7
    m.E = np.full(m.rho.shape, T ** 4)
    m.e = m.rho * T / (m.gamma - 1)
    announce("equilibrium preserved")
    st = Stepper(params_for(m, rtol=1e-12))
    E, e = dev(m.E), dev(m.e)
    rho, kap = dev(m.rho), dev(m.kappa)
    out = dev(np.zeros_like(m.E))
    _, stats = fld.fld_step(st.ctx, m.dt, rho, kap, E, out)
    assert stats["cycles"] == 0 and np.array_equal(host(out), m.E)
    S = m.E + m.e
    for k in range(100):
        stats = st.step(m.dt, rho, kap, E, e)
        assert stats["cycles"] == 0
    ulp = np.spacing(S)
    assert np.all(np.abs(host(E) - m.E) <= 2 * 100 * ulp)
    assert np.all(np.abs(host(e) - m.e) <= 2 * 100 * ulp)
    assert np.all(np.abs(host(E) + host(e) - S) <= 2 * 100 * ulp)


def test_solve_conserves_total_energy():
    m = media.random_small_medium(21, (96, 80), ("neumann", "periodic"))
    announce("global conservation")
    x, stats = _solve_gpu(m, rtol=1e-12)
    assert abs(x.sum() - m.E.sum()) <= 1e-11 * m.E.sum()


def test_alias_and_determinism():
    from paper_2503_02764_amd import fld
    m = media.config_c2(n=128)
    prob = F.problem_from_medium(m)
    kap = F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
    announce("alias/determinism")
    ctx = fld.fld_setup(params_for(m, rtol=1e-10))
    rho, kd = dev(m.rho), dev(kap)
    outs = []
    for _ in range(3):
        E = dev(m.E)
        out = dev(np.zeros_like(m.E))
        fld.fld_step(ctx, m.dt, rho, kd, E, out)
        outs.append(host(out))
    E = dev(m.E)
    fld.fld_step(ctx, m.dt, rho, kd, E, E)  # in place
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    assert np.array_equal(host(E), outs[0])


def test_zero_guess_same_solution():
    m = media.random_small_medium(3, (40, 40), ("neumann", "neumann"))
    announce("zero guess")
    x0, _ = _solve_gpu(m, rtol=1e-12)
    x1, s1 = _solve_gpu(m, rtol=1e-12, guess="zero")
    assert s1["rel_res_initial"] == pytest.approx(1.0)
    assert rel_l2(x1, x0) <= 1e-10


@pytest.mark.parametrize("n,bc", [((96, 80), ("periodic", "neumann")),
                                  ((130, 70), ("neumann", "periodic"))])
def test_initial_residual_of_previous_energy(n, bc):
    """The coefficient stage of a 2D grid also forms |b - A E^n| / |b| for
    the default guess (x0 = E^n): equal to the oracle's residual of E^n with
    the oracle's coefficients, to rounding (each term alpha (E - E_f) loses
    digits to the difference of neighbouring E, a few ulp of |E| / |E - E_f|
    on these media, far inside the 1e-12 bar)."""
    m = media.random_small_medium(17 + n[0], n, bc)
    prob = F.problem_from_medium(m)
    alphas = F.face_coefficients(m.E, m.rho, m.kappa, m.dt, prob)
    ref = F.relative_residual(m.E, m.E, alphas, prob)
    announce(f"initial residual n={n} bc={bc}")
    from paper_2503_02764_amd import fld
    ctx = fld.fld_setup(params_for(m, rtol=1e-10))
    rho, kap = dev(m.rho), dev(m.kappa)
    for aliased in (False, True):
        E = dev(m.E)
        out = E if aliased else dev(np.zeros_like(m.E))
        _, stats = fld.fld_step(ctx, m.dt, rho, kap, E, out)
        assert stats["rel_res_initial"] == pytest.approx(ref, rel=1e-12,
                                                         abs=1e-15), aliased
        assert stats["rel_res_final"] <= 1e-10


def test_error_paths():
    from paper_2503_02764_amd import fld
    m = media.random_small_medium(4, (32, 32), ("neumann", "neumann"))
    announce("error paths")
    ctx = fld.fld_setup(params_for(m, rtol=1e-14, max_cycles=1))
    rho, kap, E = dev(m.rho), dev(m.kappa), dev(m.E)
    out = dev(np.zeros_like(m.E))
    st, stats = fld.fld_step(ctx, m.dt, rho, kap, E, out, check=False)
    assert st == fld.FLD_ERR_NOT_CONVERGED
    assert stats["cycles"] == 1 and stats["rel_res_final"] > 1e-14
    ctx = fld.fld_setup(params_for(m, rtol=1e-10))
    Ebad = m.E.copy()
    Ebad[3, 4] = -1.0
    st, stats = fld.fld_step(ctx, m.dt, rho, kap, dev(Ebad), out, check=False)
    assert st == fld.FLD_ERR_NONPHYSICAL and stats["flagged_cells"] == 1
    kbad = m.kappa.copy()
    kbad[0, 0] = np.nan
    kbad[7, 7] = 0.0
    st, stats = fld.fld_step(ctx, m.dt, rho, dev(kbad), E, out, check=False)
    assert st == fld.FLD_ERR_NONPHYSICAL and stats["flagged_cells"] == 2
    # the context stays usable after an error
    st, stats = fld.fld_step(ctx, m.dt, rho, kap, E, out)
    assert st == fld.FLD_OK
    with pytest.raises(fld.FldError):
        fld.fld_step(ctx, -1.0, rho, kap, E, out)


def test_c2_full_size_bench_configuration():
    """1024^2 at the benchmark's rtol: oracle-side residual and sampled cells.

    The oracle assembles its own operator from the same inputs and measures
    the GPU iterate's residual; the exchange is checked cell by cell on a
    sample (it is pointwise, so the oracle can compute single cells).
    """
    from paper_2503_02764_amd.solver import Stepper
    m = media.config_c2(n=1024)
    prob = F.problem_from_medium(m)
    kap = F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
    announce("c2 full size 1024^2")
    import bench
    from paper_2503_02764_amd import fld
    # the cycle and the autotuned tile shapes the bench runs with
    st = Stepper(params_for(m, rtol=1e-8, pre_smooth=bench.PRE,
                            post_smooth=bench.POST,
                            coarse_pre_smooth=bench.COARSE_PRE,
                            coarse_post_smooth=bench.COARSE_POST),
                 opacity=m.opacity)
    fld.fld_autotune(st.ctx)
    rho, E, e = dev(m.rho), dev(m.E), dev(m.e)
    kap_d = dev(np.zeros_like(m.E))
    o = m.opacity
    fld.fld_opacity_powerlaw(st.ctx, rho, e, o["k0"], o["a"], o["b"],
                             o["kmin"], o["kmax"], kap_d)
    Estar = dev(np.zeros_like(m.E))
    _, stats = fld.fld_step(st.ctx, m.dt, rho, kap_d, E, Estar)
    x = host(Estar)
    alphas = F.face_coefficients(m.E, m.rho, kap, m.dt, prob)
    rr = F.relative_residual(x, m.E, alphas, prob)
    assert rr <= 1.0e-8 * 1.001, (rr, stats)
    assert abs(rr / stats["rel_res_final"] - 1) < 1e-3
    fld.fld_exchange(st.ctx, m.dt, rho, kap_d, Estar, e)
    idx = np.random.default_rng(0).choice(x.size, 4096, replace=False)
    xs = x.ravel()[idx]
    En, en = F.exchange(xs, m.e.ravel()[idx], m.rho.ravel()[idx],
                        kap.ravel()[idx], m.dt, prob)
    S = xs + m.e.ravel()[idx]
    assert np.all(np.abs(host(e).ravel()[idx] - en) <= 8 * np.spacing(S))
    assert np.all(np.abs(host(Estar).ravel()[idx] - En) <= 8 * np.spacing(S))



@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_c3_full_size_bench_configuration(precision):
    """256^3 stratified medium in the bench's configuration (its V-cycle,
    rtol 1e-8): the oracle assembles its own operator from the same inputs and
    measures the GPU iterate's residual.  A has every eigenvalue >= 1, so
    |x - A^-1 b| <= |b - A x|: a relative residual of 1e-8 bounds the error
    against the exact solve as well.  The exchange is checked on sampled
    cells."""
    from paper_2503_02764_amd.solver import make_params
    from paper_2503_02764_amd import fld
    m = media.config_c3()
    prob = F.problem_from_medium(m)
    kap = F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
    announce(f"c3 full size 256^3 {precision}")
    import bench
    params = make_params(3, m.n, m.dx, m.bc, rtol=1e-8, precision=precision,
                         max_cycles=300, pre_smooth=bench.PRE3,
                         post_smooth=bench.POST3,
                         coarse_pre_smooth=bench.COARSE_PRE3,
                         coarse_post_smooth=bench.COARSE_POST3)
    ctx = fld.fld_setup(params)
    rho, E, e = dev(m.rho), dev(m.E), dev(m.e)
    kap_d = dev(np.zeros_like(m.E))
    o = m.opacity
    fld.fld_opacity_powerlaw(ctx, rho, e, o["k0"], o["a"], o["b"],
                             o["kmin"], o["kmax"], kap_d)
    np.testing.assert_allclose(host(kap_d), kap, rtol=1e-13)
    Estar = dev(np.zeros_like(m.E))
    _, stats = fld.fld_step(ctx, m.dt, rho, kap_d, E, Estar)
    x = host(Estar)
    alphas = F.face_coefficients(m.E, m.rho, kap, m.dt, prob)
    rr = F.relative_residual(x, m.E, alphas, prob)
    assert rr <= 1.0e-8 * 1.001, (rr, stats)
    assert abs(rr / stats["rel_res_final"] - 1) < 1e-3, (rr, stats)
    fld.fld_exchange(ctx, m.dt, rho, kap_d, Estar, e)
    idx = np.random.default_rng(1).choice(x.size, 4096, replace=False)
    xs = x.ravel()[idx]
    En, en = F.exchange(xs, m.e.ravel()[idx], m.rho.ravel()[idx],
                        kap.ravel()[idx], m.dt, prob)
    S = xs + m.e.ravel()[idx]
    assert np.all(np.abs(host(e).ravel()[idx] - en) <= 8 * np.spacing(S))
    assert np.all(np.abs(host(Estar).ravel()[idx] - En) <= 8 * np.spacing(S))


TILED_2D = [
    ((96, 80), ("periodic", "periodic")),
    ((200, 136), ("neumann", "neumann")),
    ((384, 192), ("periodic", "neumann")),
    ((130, 66), ("neumann", "periodic")),
]


@pytest.mark.parametrize("n,bc", TILED_2D)
@pytest.mark.parametrize("nu", [1, 2, 3])
def test_2d_tiled_levels_vs_oracle(n, bc, nu):
    """Grids large enough for the LDS-tiled kernels, ragged tile edges."""
    m = media.random_small_medium(n[0] + 7 * n[1], n, bc, contrast=1.0)
    announce(f"tiled 2d n={n} bc={bc} nu={nu}")
    x, stats = _solve_gpu(m, rtol=1e-12, pre_smooth=nu, post_smooth=nu,
                          max_cycles=200)
    ref = F.diffusion_step(m.E, m.rho, m.kappa, m.dt,
                           F.problem_from_medium(m))
    assert rel_l2(x, ref) <= 1e-10, stats


@pytest.mark.parametrize("n,bc", TILED_2D[:2] + [((12, 12, 12),
                                                  ("periodic",) * 3)])
def test_fast_and_simple_kernel_paths_agree(n, bc, monkeypatch):
    m = media.random_small_medium(3 * n[0] + n[1], n, bc)
    announce(f"fast vs simple n={n}")
    x_fast, s_fast = _solve_gpu(m, rtol=1e-12)
    monkeypatch.setenv("FLD_KERNEL_PATH", "simple")
    x_simple, s_simple = _solve_gpu(m, rtol=1e-12)
    assert rel_l2(x_fast, x_simple) <= 1e-10, (s_fast, s_simple)


@pytest.mark.parametrize("nu", [1, 2])
def test_fast_and_simple_paths_same_cycles(nu, monkeypatch):
    """Both kernel paths run the same V-cycle: equal residual histories.

    Rough, high-contrast white-noise coefficients converge slowly with the
    rediscretised coarse operators; this pins that the tiled kernels and
    the one-pass-per-colour kernels take the same iterates there.
    """
    from paper_2503_02764_amd import fld
    m = media.random_small_medium(11, (96, 80), ("periodic", "periodic"),
                                  contrast=1.5)
    announce(f"fast vs simple residual history nu={nu}")
    res = {}
    for path in ("fast", "simple"):
        if path == "simple":
            monkeypatch.setenv("FLD_KERNEL_PATH", "simple")
        ctx = fld.fld_setup(params_for(m, rtol=1e-15, max_cycles=6,
                                       pre_smooth=nu, post_smooth=nu))
        out = dev(np.zeros_like(m.E))
        st, stats = fld.fld_step(ctx, m.dt, dev(m.rho), dev(m.kappa),
                                 dev(m.E), out, check=False)
        assert st == fld.FLD_ERR_NOT_CONVERGED
        res[path] = stats["rel_res_final"]
    assert abs(res["fast"] / res["simple"] - 1) < 1e-6, res


MIXED = [
    ((512,), ("periodic",)),
    ((128, 128), ("neumann", "neumann")),
    ((200, 136), ("periodic", "neumann")),
    ((16, 16, 16), ("periodic", "periodic", "neumann")),
    ((24, 20, 12), ("neumann", "neumann", "neumann")),
]


@pytest.mark.parametrize("n,bc", MIXED)
def test_mixed_precision_refinement_vs_oracle(n, bc):
    """FP32 V-cycles inside FP64 iterative refinement reach FP64 accuracy."""
    m = media.random_small_medium(5 * n[0] + len(n), n, bc)
    announce(f"mixed n={n} bc={bc}")
    x, stats = _solve_gpu(m, rtol=1e-11, precision="fp32_ir", max_cycles=200)
    ref = F.diffusion_step(m.E, m.rho, m.kappa, m.dt,
                           F.problem_from_medium(m))
    assert stats["rel_res_final"] <= 1e-11
    assert stats["outer_iters"] >= 1
    assert rel_l2(x, ref) <= 1e-10, stats


def test_mixed_precision_c3_like_stratified():
    """Stratified 3D medium (the 3D workload's statistics, 32^3)."""
    m = media.config_c3(n=32)
    prob = F.problem_from_medium(m)
    kap = F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
    m.kappa = kap
    announce("mixed c3-like 32^3")
    x, stats = _solve_gpu(m, rtol=1e-9, precision="fp32_ir", max_cycles=400)
    ref = F.diffusion_step(m.E, m.rho, kap, m.dt, prob)
    assert rel_l2(x, ref) <= 1e-8, stats
    x64, s64 = _solve_gpu(m, rtol=1e-9, max_cycles=400)
    assert rel_l2(x64, ref) <= 1e-8, s64


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6])
def test_tile_shapes_give_identical_iterates(variant, monkeypatch):
    """Every tile shape performs the same red-black sweeps, residuals and
    transfers cell by cell: the same iterate bit for bit (the residual norm
    is summed in another order, so the stop test could differ only at a
    tie; the cycle count is checked too)."""
    from paper_2503_02764_amd import fld
    m = media.config_c2(n=256)
    prob = F.problem_from_medium(m)
    kap = F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
    announce(f"tile shape {variant} vs 0 on c2 256")
    out = {}
    for v in (0, variant):
        monkeypatch.setenv("FLD_TILE_VARIANT", str(v))
        for prec in ("fp64", "fp32_ir"):
            ctx = fld.fld_setup(params_for(m, rtol=1e-10, precision=prec))
            x = dev(np.zeros_like(m.E))
            _, st = fld.fld_step(ctx, m.dt, dev(m.rho), dev(kap), dev(m.E), x)
            out[(v, prec)] = (host(x), st["cycles"])
    for prec in ("fp64", "fp32_ir"):
        assert out[(0, prec)][1] == out[(variant, prec)][1]
        np.testing.assert_array_equal(out[(0, prec)][0],
                                      out[(variant, prec)][0])


def test_autotune_keeps_results():
    from paper_2503_02764_amd import fld
    m = media.config_c2(n=256)
    prob = F.problem_from_medium(m)
    kap = F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
    ref = F.diffusion_step(m.E, m.rho, kap, m.dt, prob)
    announce("autotune c2 256")
    ctx = fld.fld_setup(params_for(m, rtol=1e-12))
    x0 = dev(np.zeros_like(m.E))
    fld.fld_step(ctx, m.dt, dev(m.rho), dev(kap), dev(m.E), x0)
    shapes = fld.fld_autotune(ctx)
    names = {"64x48/256", "64x64/512", "64x64/1024", "32x32/256", "128x48/512",
             "32x64/256", "64x32/512"}
    assert all(d in names and u in names for d, u in shapes[:4]), shapes
    x1 = dev(np.zeros_like(m.E))
    fld.fld_step(ctx, m.dt, dev(m.rho), dev(kap), dev(m.E), x1)
    assert rel_l2(host(x1), ref) <= 1e-10
    np.testing.assert_array_equal(host(x1), host(x0))


@pytest.mark.parametrize("case", [((16, 12), (0, 1)), ((8, 8, 6), (1, 0, 1)),
                                  ((40,), (1,))])
def test_same_calls_on_both_sides(case):
    """One parameter mapping drives the library (fld_setup / fld_step /
    fld_exchange) and the oracle's calls of the same names."""
    from paper_2503_02764_amd import fld
    from oracle.fldref_api import fldref_exchange, fldref_setup, fldref_step
    n, codes = case
    nd = len(n)
    bcs = tuple("periodic" if c == 0 else "neumann" for c in codes)
    m = media.random_small_medium(7 + nd, n, bcs)
    spec = dict(ndim=nd, n=tuple(n) + (1,) * (3 - nd), dx=m.dx,
                bc_lo=tuple(codes) + (0,) * (3 - nd),
                bc_hi=tuple(codes) + (0,) * (3 - nd), c=1.0, a_rad=1.0,
                gamma=5.0 / 3.0, gas_const=1.0, limiter=0, face_mean=0,
                rtol=1e-12)
    announce(f"same calls on both sides n={n}")
    ctx = fld.fld_setup(fld.fld_params_default(**spec))
    ref_ctx = fldref_setup(spec)
    rho, kap = dev(m.rho), dev(m.kappa)
    E = dev(m.E)
    out = dev(np.zeros_like(m.E))
    fld.fld_step(ctx, m.dt, rho, kap, E, out)
    x, _ = fldref_step(ref_ctx, m.dt, m.rho, m.kappa, m.E)
    assert rel_l2(host(out).reshape(x.shape), x) <= 1e-10
    e = dev(m.e)
    fld.fld_exchange(ctx, m.dt, rho, kap, out, e)
    En, en = fldref_exchange(ref_ctx, m.dt, m.rho, m.kappa, x, m.e)
    S = x + m.e
    assert np.abs(host(e).reshape(en.shape) - en).max() <= 1e-9 * S.max()
    assert np.abs(host(out).reshape(En.shape) - En).max() <= 1e-9 * S.max()


@pytest.mark.parametrize("n,bc", [((96, 80), ("periodic", "neumann")),
                                  ((130, 70), ("neumann", "periodic")),
                                  ((200, 136), ("periodic", "periodic")),
                                  ((1000, 520), ("neumann", "neumann")),
                                  ((384, 256), ("neumann", "periodic")),
                                  ((512, 512), ("neumann", "neumann"))])
def test_multilevel_coarsening_matches_per_level(n, bc, monkeypatch):
    """The 2D coarse coefficients computed several levels per launch (pair
    tiles, whole small levels in one block, single-level fallback) are those
    of one launch per level: the same iterate bit for bit, in FP64 and in
    the FP32 hierarchy."""
    from paper_2503_02764_amd import fld
    m = media.random_small_medium(31 + n[0], n, bc)
    announce(f"multi-level coarsening {n} {bc}")
    out = {}
    for per_level in (False, True):
        if per_level:
            monkeypatch.setenv("FLD_COARSEN_PER_LEVEL", "1")
        else:
            monkeypatch.delenv("FLD_COARSEN_PER_LEVEL", raising=False)
        for prec in ("fp64", "fp32_ir"):
            ctx = fld.fld_setup(params_for(m, rtol=1e-10, precision=prec,
                                           max_cycles=200))
            x = dev(np.zeros_like(m.E))
            _, st = fld.fld_step(ctx, m.dt, dev(m.rho), dev(m.kappa),
                                 dev(m.E), x)
            out[(per_level, prec)] = (host(x), st["cycles"])
    for prec in ("fp64", "fp32_ir"):
        assert out[(False, prec)][1] == out[(True, prec)][1]
        np.testing.assert_array_equal(out[(False, prec)][0],
                                      out[(True, prec)][0])


@pytest.mark.parametrize("n,bc", [((75,), ("periodic",)),
                                  ((1501,), ("periodic",)),
                                  ((65, 35), ("periodic", "periodic")),
                                  ((200, 136), ("periodic", "periodic")),
                                  ((130, 70), ("neumann", "periodic")),
                                  ((96, 80), ("periodic", "periodic")),
                                  ((20, 12, 28), ("periodic", "neumann",
                                                  "periodic"))])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_odd_periodic_levels_are_deterministic(n, bc, precision):
    """A periodic dimension of odd length (on the finest level or on the
    coarsest one that coarsening reaches) has same-parity neighbours across
    the wrap; the sweeps then use the extra colour classes.  A data race
    there would show as run-to-run differences in the last bits; the answer
    must also be the oracle's.  (1501,) and (65, 35) are single levels too
    large for the LDS tail: the whole solve runs in the global-memory tail,
    whose outcome the host reads from the control block's mirror.)"""
    from paper_2503_02764_amd import fld
    m = media.random_small_medium(7 + sum(n), n, bc)
    announce(f"odd periodic determinism {n} {bc} {precision}")
    outs = []
    for _ in range(3):
        ctx = fld.fld_setup(params_for(m, rtol=1e-11, precision=precision,
                                       max_cycles=400))
        x = dev(np.zeros_like(m.E))
        _, st = fld.fld_step(ctx, m.dt, dev(m.rho), dev(m.kappa), dev(m.E), x)
        assert st["rel_res_final"] <= 1e-11, st
        outs.append(host(x))
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])
    ref = F.diffusion_step(m.E, m.rho, m.kappa, m.dt, F.problem_from_medium(m))
    assert rel_l2(outs[0], ref) <= 1e-9


@pytest.mark.parametrize("n,bc", [((200, 136), ("neumann", "neumann")),
                                  ((96, 80), ("periodic", "neumann"))])
@pytest.mark.parametrize("coarse", [(1, 1), (3, 3), (3, 1)])
def test_coarse_level_smoothing_counts(n, bc, coarse):
    """Coarse levels may smooth more or less than the finest one (tiled
    levels, register tail and the FP32 hierarchy alike); the answer is the
    oracle's whatever the counts."""
    m = media.random_small_medium(61 + n[0] + coarse[0], n, bc)
    announce(f"coarse smoothing {coarse} {n} {bc}")
    ref = F.diffusion_step(m.E, m.rho, m.kappa, m.dt, F.problem_from_medium(m))
    for prec, tol in (("fp64", 1e-10), ("fp32_ir", 1e-8)):
        x, stats = _solve_gpu(m, rtol=1e-12 if prec == "fp64" else 1e-10,
                              precision=prec, pre_smooth=2, post_smooth=3,
                              coarse_pre_smooth=coarse[0],
                              coarse_post_smooth=coarse[1], max_cycles=200)
        assert rel_l2(x, ref) <= tol, (prec, stats)
