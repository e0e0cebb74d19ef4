"""FP64 parity at the workloads' full sizes, solved to 1e-12.

The backward-Euler operator is A = I + dt L with L symmetric positive
semi-definite, so every eigenvalue of A is at least 1 and the error against
the exact solve obeys |x - A^-1 b|_2 <= |b - A x|_2.  Since the column sums
of A are 1, sum(x) = sum(b) and |x|_2 >= sum(b) / sqrt(N); together

    rel-L2 error <= rel-residual * sqrt(N) |b|_2 / sum(b).

The oracle assembles its own operator from the same inputs and measures the
residual of the GPU iterate, so each test below bounds the element-wise
error against the exact solve by a figure the oracle computes itself, at
sizes where the exact solve is out of its reach.  On the 64^3 stratified
medium (the 3D workload's statistics, small enough for the oracle's
conjugate gradients to 1e-14) the error is measured element by element.
"""
import numpy as np
import pytest

import media
from oracle import fldref as F

from gpu_common import announce, dev, host, params_for, rel_l2

pytestmark = pytest.mark.gpu


def _bound_factor(b):
    b = b.ravel()
    return float(np.sqrt(b.size) * np.linalg.norm(b) / b.sum())


def _oracle_check(m, x, kap, rtol, err_bar):
    prob = F.problem_from_medium(m)
    alphas = F.face_coefficients(m.E, m.rho, kap, m.dt, prob)
    rr = F.relative_residual(x, m.E, alphas, prob)
    bound = rr * _bound_factor(m.E)
    assert rr <= rtol * 1.001, rr
    assert bound <= err_bar, (rr, bound)
    return rr, bound


def test_c2_full_size_fp64_rtol_1e12():
    """1024^2 Kramers/log-normal medium, the benchmark's V-cycle and
    autotuned tiles, FP64 to 1e-12: error bound <= 1e-10 from the oracle's
    residual."""
    import bench
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import Stepper
    m = media.config_c2(n=1024)
    prob = F.problem_from_medium(m)
    kap = F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
    announce("c2 full size 1024^2 fp64 rtol 1e-12")
    st = Stepper(params_for(m, rtol=1e-12, max_cycles=100,
                            pre_smooth=bench.PRE, post_smooth=bench.POST,
                            coarse_pre_smooth=bench.COARSE_PRE,
                            coarse_post_smooth=bench.COARSE_POST),
                 opacity=m.opacity)
    fld.fld_autotune(st.ctx)
    rho, E, e = dev(m.rho), dev(m.E), dev(m.e)
    kap_d = dev(np.zeros_like(m.E))
    o = m.opacity
    fld.fld_opacity_powerlaw(st.ctx, rho, e, o["k0"], o["a"], o["b"],
                             o["kmin"], o["kmax"], kap_d)
    np.testing.assert_allclose(host(kap_d), kap, rtol=1e-13)
    out = dev(np.zeros_like(m.E))
    _, stats = fld.fld_step(st.ctx, m.dt, rho, kap_d, E, out)
    rr, _ = _oracle_check(m, host(out), kap, 1e-12, 1e-10)
    # near 1e-13 the two residuals differ by the rounding of the residual
    # itself (about eps times the sum of the face coefficients per cell)
    assert abs(rr - stats["rel_res_final"]) <= max(1e-3 * rr, 1e-13), \
        (rr, stats)


@pytest.mark.parametrize("precision,rtol,bar", [("fp64", 1e-12, 1e-10),
                                                ("fp32_ir", 1e-10, 1e-8)])
def test_c3_full_size_tight(precision, rtol, bar):
    """256^3 stratified medium in the benchmark's V-cycle, FP64 to 1e-12
    (error bound <= 1e-10) and FP32 V-cycles in FP64 refinement to 1e-10
    (bound <= 1e-8)."""
    import bench
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import make_params
    m = media.config_c3()
    prob = F.problem_from_medium(m)
    kap = F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
    announce(f"c3 full size 256^3 {precision} rtol {rtol}")
    params = make_params(3, m.n, m.dx, m.bc, rtol=rtol, precision=precision,
                         max_cycles=400, pre_smooth=bench.PRE3,
                         post_smooth=bench.POST3,
                         coarse_pre_smooth=bench.COARSE_PRE3,
                         coarse_post_smooth=bench.COARSE_POST3)
    ctx = fld.fld_setup(params)
    out = dev(np.zeros_like(m.E))
    _, stats = fld.fld_step(ctx, m.dt, dev(m.rho), dev(kap), dev(m.E), out)
    rr, _ = _oracle_check(m, host(out), kap, rtol, bar)
    assert abs(rr - stats["rel_res_final"]) <= max(1e-3 * rr, 1e-13), \
        (rr, stats)


@pytest.mark.parametrize("fused", ["0", "8"])
@pytest.mark.parametrize("precision,rtol,bar", [("fp64", 1e-12, 1e-10),
                                                ("fp32_ir", 1e-9, 1e-8)])
def test_c3_statistics_64cube_elementwise(precision, rtol, bar, fused,
                                          monkeypatch):
    """64^3 medium with the 3D workload's statistics (exponential
    stratification, Kramers opacity, periodic x, y and Neumann z), the
    benchmark's V-cycle, colour passes ("0") or fused one-launch sweeps
    ("8" planes per block) on every level: relative L2 error against the
    oracle's exact solve (conjugate gradients to 1e-14) <= 1e-10 in FP64 and
    <= 1e-8 after FP32 V-cycles in FP64 refinement."""
    import bench
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import make_params
    monkeypatch.setenv("FLD_SWEEP3D", fused)
    m = media.config_c3(n=64)
    prob = F.problem_from_medium(m)
    kap = F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
    alphas = F.face_coefficients(m.E, m.rho, kap, m.dt, prob)
    ref = F.solve(alphas, m.E, prob, method="cg", rtol=1e-14)
    announce(f"c3 statistics 64^3 {precision} fused={fused}")
    params = make_params(3, m.n, m.dx, m.bc, rtol=rtol, precision=precision,
                         max_cycles=400, pre_smooth=bench.PRE3,
                         post_smooth=bench.POST3,
                         coarse_pre_smooth=bench.COARSE_PRE3,
                         coarse_post_smooth=bench.COARSE_POST3)
    ctx = fld.fld_setup(params)
    out = dev(np.zeros_like(m.E))
    _, stats = fld.fld_step(ctx, m.dt, dev(m.rho), dev(kap), dev(m.E), out)
    assert rel_l2(host(out), ref) <= bar, stats
