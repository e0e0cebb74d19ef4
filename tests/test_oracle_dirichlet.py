"""Oracle pins of the Dirichlet wall (E held at E_w on a boundary face; the
radiation temperature tied to the gas temperature on the boundary of the
magnetoconvection case, Sect. 4.5).

Closed forms: with a uniform diffusion coefficient and a step long enough
to reach the steady state, the solution between two Dirichlet walls is the
straight line through the wall values at the wall faces (half a cell
outside the first and last centres); a medium at the wall value stays
there; the odd-reflection ghosts make the five-point gradient exact on a
line that meets the wall value at the wall face; the wall's diagonal and
right-hand-side terms by hand on three cells; and the step conserves
energy up to the flux through the Dirichlet walls.
"""
import numpy as np
import pytest

from oracle import fldref as F


def _prob_1d(n, dirichlet, dx=None, limiter="diffusion", face_mean="arith"):
    dx = 1.0 / n if dx is None else dx
    return F.Problem(ndim=1, n=(n, 1, 1), dx=(dx, 1.0, 1.0), bc=(F.NEUMANN,),
                     limiter=limiter, face_mean=face_mean,
                     dirichlet=dict(dirichlet))


def test_steady_state_is_the_line_through_the_wall_values():
    n = 8
    prob = _prob_1d(n, {(0, 0): 1.0, (0, 1): 3.0})
    E = np.full(n, 2.0)
    rho = np.full(n, 1.0)
    kap = np.full(n, 3.0)  # D = c / (3 rho kappa) = 1/9, uniform
    x = F.diffusion_step(E, rho, kap, 1e12, prob)
    centres = (np.arange(n) + 0.5) / n
    line = 1.0 + 2.0 * centres
    np.testing.assert_allclose(x, line, rtol=1e-9, atol=0)


def test_one_wall_steady_state_is_the_wall_value():
    # Neumann on the left, Dirichlet on the right: the steady state is flat
    # at the wall value whatever the start and the medium
    n = 6
    prob = _prob_1d(n, {(0, 1): 0.5}, limiter="lp")
    rng = np.random.default_rng(4)
    E = 1.0 + rng.random(n)
    rho = 1.0 + rng.random(n)
    kap = 1.0 + rng.random(n)
    x = F.diffusion_step(E, rho, kap, 1e13, prob)
    np.testing.assert_allclose(x, 0.5, rtol=1e-8)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_medium_at_the_wall_value_stays_there(ndim):
    n = (6, 5, 4)[:ndim] + (1,) * (3 - ndim)
    shape = tuple(reversed(n[:ndim]))
    bc = (F.NEUMANN, F.PERIODIC, F.NEUMANN)[:ndim]
    walls = {(0, 0): 2.5, (0, 1): 2.5}
    if ndim == 3:
        walls[(2, 1)] = 2.5
    prob = F.Problem(ndim=ndim, n=n, dx=(0.1, 0.2, 0.3), bc=bc,
                     dirichlet=walls)
    rng = np.random.default_rng(ndim)
    E = np.full(shape, 2.5)
    rho = 1.0 + rng.random(shape)
    kap = 1.0 + rng.random(shape)
    x = F.diffusion_step(E, rho, kap, 0.7, prob)
    np.testing.assert_allclose(x, 2.5, rtol=1e-13)


def test_gradient_exact_on_a_line_meeting_the_wall_value():
    # E = 2 + 3 x on cell centres x_i = (i + 1/2) dx, walls at x = 0 and
    # x = n dx holding the line's values there: the odd reflection continues
    # the line, so every cell's five-point gradient is 3; mirror ghosts
    # (Neumann) are not
    n = 7
    dx = 0.25
    x = (np.arange(n) + 0.5) * dx
    E = 2.0 + 3.0 * x
    prob = _prob_1d(n, {(0, 0): 2.0, (0, 1): 2.0 + 3.0 * n * dx}, dx=dx)
    (G,) = F.gradient(E, prob)
    np.testing.assert_allclose(G, 3.0, rtol=1e-13)
    (Gn,) = F.gradient(E, _prob_1d(n, {}, dx=dx))
    assert abs(Gn[0] - 3.0) > 0.5 and abs(Gn[-1] - 3.0) > 0.5


def test_wall_terms_hand_values_three_cells():
    # three cells, dx = 0.5, dt = 0.2, Dirichlet E_w = 4 on the upper wall
    # only; diffusion limiter, c = 1: D = 1 / (3 rho kappa)
    prob = _prob_1d(3, {(0, 1): 4.0}, dx=0.5)
    E = np.array([1.0, 2.0, 3.0])
    rho = np.array([1.0, 1.0, 2.0])
    kap = np.array([1.0, 2.0, 1.0])
    dt = 0.2
    D = np.array([1 / 3, 1 / 6, 1 / 6])
    diag, rhs = F.dirichlet_terms(E, rho, kap, dt, prob)
    aw = 2.0 * dt * D[2] / 0.25  # 2 dt D / dx^2 = 4/15
    np.testing.assert_allclose(diag, [0.0, 0.0, aw], rtol=1e-15)
    np.testing.assert_allclose(rhs, [0.0, 0.0, 4.0 * aw], rtol=1e-15)
    alphas = F.face_coefficients(E, rho, kap, dt, prob)
    a01 = dt * 0.5 * (D[0] + D[1]) / 0.25
    a12 = dt * 0.5 * (D[1] + D[2]) / 0.25
    A = F.assemble(alphas, prob, diag).toarray()
    expect = np.array([[1 + a01, -a01, 0.0],
                       [-a01, 1 + a01 + a12, -a12],
                       [0.0, -a12, 1 + a12 + aw]])
    np.testing.assert_allclose(A, expect, rtol=1e-14)
    x = F.diffusion_step(E, rho, kap, dt, prob)
    np.testing.assert_allclose(expect @ x, E + rhs, rtol=1e-13)


def test_energy_balance_through_the_walls():
    # sum(E* - E^n) is the net inflow through the Dirichlet walls,
    # sum over wall cells of alpha_w (E_w - E*_i); interior faces cancel
    n = (12, 9)
    prob = F.Problem(ndim=2, n=n + (1,), dx=(0.1, 0.1, 1.0),
                     bc=(F.PERIODIC, F.NEUMANN), limiter="lp",
                     dirichlet={(1, 0): 5.0, (1, 1): 0.5})
    rng = np.random.default_rng(7)
    shape = prob.shape
    E = 1.0 + rng.random(shape)
    rho = 1.0 + rng.random(shape)
    kap = 1.0 + rng.random(shape)
    dt = 0.05
    x = F.diffusion_step(E, rho, kap, dt, prob)
    diag, rhs = F.dirichlet_terms(E, rho, kap, dt, prob)
    inflow = np.sum(rhs - diag * x)
    assert np.sum(x - E) == pytest.approx(inflow, rel=1e-11)
    assert inflow != 0.0
