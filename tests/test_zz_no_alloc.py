"""The allocation-free step (fld_step_noalloc) against fld_step.

Both run the same kernels with the default tile shape on every level, so
the iterates must agree bit for bit.  Two calls in a row, the second on a
smaller grid, check that the shared static scratch carries nothing from one
call into the next; a grid whose workspace exceeds the scratch is rejected
on the host before anything is launched.
"""
import numpy as np
import pytest

import media

from gpu_common import announce, dev, host, params_for

pytestmark = pytest.mark.gpu


def _both(m, **kw):
    from paper_2503_02764_amd import fld
    from oracle import fldref as F
    prob = F.problem_from_medium(m)
    kap = m.kappa if m.kappa is not None else \
        F.opacity_powerlaw(m.rho, m.e, prob, **m.opacity)
    params = params_for(m, **kw)
    rho, kd, E = dev(m.rho), dev(kap), dev(m.E)
    ctx = fld.fld_setup(params)
    out_ref = dev(np.zeros_like(m.E))
    _, s_ref = fld.fld_step(ctx, m.dt, rho, kd, E, out_ref)
    out = dev(np.full_like(m.E, -1.0))
    _, s = fld.fld_step_noalloc(params, m.dt, rho, kd, E, out)
    return host(out_ref), s_ref, host(out), s


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_noalloc_matches_fld_step_two_calls(precision):
    for n in (512, 128):  # the second call is smaller
        m = media.config_c2(n=n)
        announce(f"noalloc c2 n={n} {precision}")
        ref, s_ref, got, s = _both(m, rtol=1e-10, precision=precision)
        np.testing.assert_array_equal(got, ref)
        assert s["cycles"] == s_ref["cycles"]
        assert s["rel_res_final"] == s_ref["rel_res_final"] <= 1e-10


def test_noalloc_3d_then_1d_and_aliased():
    from paper_2503_02764_amd import fld
    m = media.config_c3(n=32)
    announce("noalloc c3 32^3")
    ref, s_ref, got, s = _both(m, rtol=1e-10, max_cycles=200)
    np.testing.assert_array_equal(got, ref)
    m1 = media.config_c1()
    announce("noalloc c1 512, E_out aliasing E_in")
    params = params_for(m1, rtol=1e-10)
    ctx = fld.fld_setup(params)
    rho, kd = dev(m1.rho), dev(m1.kappa)
    out_ref = dev(m1.E)
    fld.fld_step(ctx, m1.dt, rho, kd, out_ref, out_ref)
    E = dev(m1.E)
    fld.fld_step_noalloc(params, m1.dt, rho, kd, E, E)
    np.testing.assert_array_equal(host(E), host(out_ref))


def test_noalloc_rejects_grids_beyond_the_scratch():
    from paper_2503_02764_amd import fld
    from paper_2503_02764_amd.solver import make_params
    import torch
    p = make_params(3, (128, 128, 128), (1 / 128,) * 3,
                    ("periodic", "periodic", "neumann"))
    assert fld.fld_workspace_bytes(p) > 64 << 20
    z = torch.ones(128 ** 3, dtype=torch.float64, device="cuda")
    st, _ = fld.fld_step_noalloc(p, 1e-3, z, z, z, z, check=False)
    assert st == fld.FLD_ERR_WORKSPACE
    assert "static scratch" in fld.load().fld_last_error(None).decode()
    p2 = make_params(2, (64, 64), (1 / 64,) * 2, ("neumann", "neumann"),
                     guess="learned")
    z2 = z[: 64 * 64]
    st, _ = fld.fld_step_noalloc(p2, 1e-3, z2, z2, z2, z2, check=False)
    assert st == fld.FLD_ERR_INVALID_ARG
