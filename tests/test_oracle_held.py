"""Oracle pins of held cells (an interior boundary: cells whose new E is
prescribed, as the linear-wave tests of Sect. 4.3 overwrite the first
wavelength of the domain).

Closed forms: with a uniform diffusion coefficient and a step far beyond
the diffusion time, the free cells between two held cells lie on the
straight line through the held cells' centres, and a periodic ring with one
held cell settles at the held value.  Elimination: the free cells'
values equal the solution of the plain system restricted to the free cells
with the held values moved to the right-hand side (the plain operator is
pinned on its own).  Energy balance: the free cells gain what flows in
through their faces with held cells and through Dirichlet walls.
"""
import numpy as np
import pytest

from oracle import fldref as F


def _medium(shape, seed):
    rng = np.random.default_rng(seed)
    E = 1.0 + rng.random(shape)
    rho = 1.0 + rng.random(shape)
    kap = 1.0 + 2.0 * rng.random(shape)
    return rng, E, rho, kap


def _prob_2d(limiter="lp", dirichlet=None):
    return F.Problem(ndim=2, n=(12, 9, 1), dx=(0.1, 0.15, 1.0),
                     bc=(F.PERIODIC, F.NEUMANN), limiter=limiter,
                     dirichlet=dict(dirichlet or {}))


def test_held_cells_take_their_values():
    prob = _prob_2d(dirichlet={(1, 0): 2.0})
    rng, E, rho, kap = _medium(prob.shape, 1)
    held = rng.random(prob.shape) < 0.25
    E_hold = 0.5 + 3.0 * rng.random(prob.shape)
    x = F.held_step(E, rho, kap, 0.3, prob, held, E_hold)
    np.testing.assert_allclose(x[held], E_hold[held], rtol=1e-14)
    assert np.all(np.abs(x[~held] - E[~held]) > 0)


def test_steady_line_between_two_held_cells():
    n = 10
    prob = F.Problem(ndim=1, n=(n, 1, 1), dx=(1.0 / n, 1.0, 1.0),
                     bc=(F.NEUMANN,), limiter="diffusion")
    E = np.full(n, 2.0)
    rho = np.ones(n)
    kap = np.full(n, 3.0)
    held = np.zeros(n, dtype=bool)
    held[[0, n - 1]] = True
    E_hold = np.zeros(n)
    E_hold[0], E_hold[-1] = 1.0, 4.0
    x = F.held_step(E, rho, kap, 1e12, prob, held, E_hold)
    np.testing.assert_allclose(x, 1.0 + 3.0 * np.arange(n) / (n - 1),
                               rtol=1e-9)


def test_periodic_ring_settles_at_the_held_value():
    n = 16
    prob = F.Problem(ndim=1, n=(n, 1, 1), dx=(1.0 / n, 1.0, 1.0),
                     bc=(F.PERIODIC,), limiter="lp")
    _, E, rho, kap = _medium((n,), 3)
    held = np.zeros(n, dtype=bool)
    held[5] = True
    x = F.held_step(E, rho, kap, 1e13, prob, held, np.full(n, 0.75))
    np.testing.assert_allclose(x, 0.75, rtol=1e-8)


@pytest.mark.parametrize("walls", [{}, {(1, 0): 2.0, (1, 1): 0.5}])
def test_elimination_of_the_held_cells(walls):
    prob = _prob_2d(dirichlet=walls)
    rng, E, rho, kap = _medium(prob.shape, 4)
    held = rng.random(prob.shape) < 0.3
    E_hold = 0.5 + 3.0 * rng.random(prob.shape)
    dt = 0.4
    x = F.held_step(E, rho, kap, dt, prob, held, E_hold)
    alphas = F.face_coefficients(E, rho, kap, dt, prob)
    diag, rhs = F.dirichlet_terms(E, rho, kap, dt, prob)
    A = F.assemble(alphas, prob, diag).toarray()
    h = held.ravel()
    f = ~h
    b_f = (E + rhs).ravel()[f] - A[np.ix_(f, h)] @ E_hold.ravel()[h]
    x_f = np.linalg.solve(A[np.ix_(f, f)], b_f)
    np.testing.assert_allclose(x.ravel()[f], x_f, rtol=1e-12)


def test_energy_balance_through_held_faces():
    prob = _prob_2d(limiter="minerbo", dirichlet={(1, 1): 1.5})
    rng, E, rho, kap = _medium(prob.shape, 6)
    held = np.zeros(prob.shape, dtype=bool)
    held[:, :3] = True  # a band of columns, as the overwritten wavelength
    E_hold = np.full(prob.shape, 3.0)
    dt = 0.2
    x = F.held_step(E, rho, kap, dt, prob, held, E_hold)
    alphas = F.face_coefficients(E, rho, kap, dt, prob)
    diag, rhs = F.dirichlet_terms(E, rho, kap, dt, prob)
    free = ~held
    inflow = np.sum((rhs - diag * x)[free])
    for d in range(prob.ndim):
        ax = prob.axis(d)
        up = lambda a: np.roll(a, -1, axis=ax)  # noqa: E731
        flux = alphas[d] * (x - up(x))  # through face i+1/2, i -> i+1
        inflow += np.sum(flux[held & up(free)]) - np.sum(flux[free & up(held)])
    assert np.sum((x - E)[free]) == pytest.approx(inflow, rel=1e-11)
    assert inflow > 0


def test_no_held_cell_is_the_plain_step_and_all_held_is_the_values():
    prob = _prob_2d(dirichlet={(1, 0): 2.0})
    rng, E, rho, kap = _medium(prob.shape, 8)
    none = np.zeros(prob.shape, dtype=bool)
    x = F.held_step(E, rho, kap, 0.3, prob, none, np.zeros(prob.shape))
    np.testing.assert_allclose(x, F.diffusion_step(E, rho, kap, 0.3, prob),
                               rtol=1e-13)
    hold = 0.5 + rng.random(prob.shape)
    x = F.held_step(E, rho, kap, 0.3, prob, ~none, hold)
    np.testing.assert_array_equal(x, hold)
