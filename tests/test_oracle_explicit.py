"""Pins of the oracle's explicit FLD source terms (oracle/explicit.py).

- the Eddington tensor of eq. fld_Eddington_tensor has trace 1, the value f
  along n and (1 - f)/2 across it; 1/3 I in the thick limit and n n in the
  free-streaming limit (Sect. 2 after eq. fld_f);
- the radiation force f_r = -lambda grad E (eq. rad_force with eq. fld_F)
  on a linear profile, where lambda(R) is known in closed form, and its sign
  (down the gradient of E);
- photon tiring P : grad v (eq. fld_P) in the two limits: E div(v) / 3 for
  an optically thick medium and E n.(grad v).n for a free-streaming one, on
  linear velocity fields the five-point stencil differentiates exactly; a
  pure shear across a diagonal gradient, worked by hand; uniform motion
  does no work;
- the work term v . f_r.
"""
import numpy as np
import pytest

from oracle import explicit as X
from oracle import fldref as F


def _prob(n, bc, limiter="lp"):
    nd = len(n)
    return F.Problem(ndim=nd, n=tuple(list(n) + [1] * (3 - nd)),
                     dx=tuple([1.0 / v for v in n] + [1.0] * (3 - nd)),
                     bc=tuple(bc), limiter=limiter)


def _xy(n):
    ny, nx = n[1], n[0]
    y, x = np.meshgrid((np.arange(ny) + 0.5) / ny, (np.arange(nx) + 0.5) / nx,
                       indexing="ij")
    return x, y


INNER = (slice(2, -2), slice(2, -2))  # cells whose stencils touch no ghost


@pytest.mark.parametrize("f", [1.0 / 3.0, 0.5, 0.8, 1.0])
def test_eddington_tensor_trace_and_eigenvalues(f):
    rng = np.random.default_rng(3)
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    T = X.eddington_tensor(f, n)
    assert np.trace(T) == pytest.approx(1.0, abs=1e-15)
    assert n @ T @ n == pytest.approx(f, abs=1e-15)
    w = np.linalg.eigvalsh(T)
    np.testing.assert_allclose(sorted(w), sorted([f, (1 - f) / 2, (1 - f) / 2]),
                               atol=1e-15)
    if f == 1.0 / 3.0:
        np.testing.assert_allclose(T, np.eye(3) / 3.0, atol=1e-16)
    if f == 1.0:
        np.testing.assert_allclose(T, np.outer(n, n), atol=1e-16)


def test_force_on_linear_profile():
    """E = 1 + s x with rho kappa = 2: inside, grad E = (s, 0) exactly, so
    R = s / (2 E) and f_r = -(2 + R) / (6 + 3 R + R^2) s along x, 0 along
    y; it points down the gradient; the work of v = (1, 2) is f_r_x."""
    n = (24, 16)
    prob = _prob(n, ["neumann", "periodic"])
    x, _ = _xy(n)
    s = 3.0
    E = 1.0 + s * x
    rho = np.full_like(E, 2.0)
    kap = np.ones_like(E)
    v = [np.ones_like(E), 2.0 * np.ones_like(E)]
    fr, work, _, f = X.explicit_sources(E, rho, kap, v, prob)
    R = s / (2.0 * E)
    lam = (2.0 + R) / (6.0 + 3.0 * R + R * R)
    np.testing.assert_allclose(fr[0][:, 2:-2], -lam[:, 2:-2] * s, rtol=1e-12)
    np.testing.assert_allclose(fr[1], 0.0, atol=1e-12)
    assert np.all(fr[0][:, 2:-2] < 0)
    np.testing.assert_allclose(work[:, 2:-2], fr[0][:, 2:-2], rtol=1e-12)
    np.testing.assert_allclose(f[:, 2:-2], lam[:, 2:-2] + lam[:, 2:-2] ** 2 *
                               R[:, 2:-2] ** 2, rtol=1e-12)


def test_tiring_thick_limit_is_isotropic_pressure_work():
    """rho kappa = 1e12: R ~ 1e-12, f = 1/3 to 1e-24, so P = E I / 3 and
    P : grad v = E div(v) / 3; v = (a x, b y) has div v = a + b, exact for
    the stencil away from the walls.  Expansion (a + b > 0) gives a positive
    term, which eq. mhd_r_e subtracts from dE/dt."""
    n = (20, 18)
    prob = _prob(n, ["neumann", "neumann"])
    x, y = _xy(n)
    E = 2.0 + 0.3 * x - 0.2 * y
    rho = np.full_like(E, 1e6)
    kap = np.full_like(E, 1e6)
    a, b = 0.7, 0.4
    _, _, tir, f = X.explicit_sources(E, rho, kap, [a * x, b * y], prob)
    np.testing.assert_allclose(f, 1.0 / 3.0, rtol=1e-12)
    np.testing.assert_allclose(tir[INNER], (E * (a + b) / 3.0)[INNER],
                               rtol=1e-10)
    assert np.all(tir[INNER] > 0)


def test_tiring_free_streaming_limit_projects_on_n():
    """rho kappa = 1e-12 and E = exp(4 x): grad E is along x only, R ~ 1e12,
    f = 1 - O(1/R), so P = E n n with n = x: P : grad v = E d v_x / d x; with
    v = (a x, b y) the result is E a and b drops out."""
    n = (24, 12)
    prob = _prob(n, ["neumann", "periodic"])
    x, y = _xy(n)
    E = np.exp(4.0 * x)
    rho = np.full_like(E, 1e-6)
    kap = np.full_like(E, 1e-6)
    a, b = 0.7, 5.0
    _, _, tir, f = X.explicit_sources(E, rho, kap, [a * x, b * np.sin(2 * np.pi * y)],
                                      prob)
    np.testing.assert_allclose(f[:, 2:-2], 1.0, rtol=1e-9)
    np.testing.assert_allclose(tir[:, 2:-2], (E * a)[:, 2:-2], rtol=1e-9)


def test_tiring_of_a_shear_across_a_diagonal_gradient():
    """E = exp(k (x + y)) on a square grid: the stencil gives G_x = G_y, so
    n = (1, 1)/sqrt 2 everywhere inside; v = (c y, 0) is a pure shear
    (div v = 0, only d v_x / d y = c), so P : grad v = E f_xy c with
    f_xy = (3 f - 1)/2 n_x n_y = (3 f - 1)/4."""
    n = (32, 32)
    prob = _prob(n, ["neumann", "neumann"])
    x, y = _xy(n)
    E = np.exp(0.8 * (x + y))
    rho = np.full_like(E, 0.5)
    kap = np.full_like(E, 2.0)
    c = 1.3
    _, _, tir, f = X.explicit_sources(E, rho, kap, [c * y, np.zeros_like(E)],
                                      prob)
    np.testing.assert_allclose(tir[INNER], (E * (3 * f - 1) / 4 * c)[INNER],
                               rtol=1e-12)
    assert np.all(f[INNER] > 1.0 / 3.0)


def test_tiring_of_a_shear_across_an_oblique_gradient():
    """E = exp(kx x + ky y) with kx != ky: the five-point stencil gives
    G = E (gx, gy) with gx = (16 sinh(kx h) - 2 sinh(2 kx h)) / (12 h) (and
    gy likewise), so n = (gx, gy)/|g| is constant and oblique; R = |g| /
    (rho kappa).  The pure shear v = (c y, 0) gives P : grad v =
    E (3 f - 1)/2 n_x n_y c, which tells n_x n_y from n_y^2 (the off-axis
    entry of the Eddington tensor)."""
    n = (40, 40)
    h = 1.0 / 40
    prob = _prob(n, ["neumann", "neumann"])
    x, y = _xy(n)
    kx, ky = 2.0, 0.5
    E = np.exp(kx * x + ky * y)
    rho = np.full_like(E, 0.5)
    kap = np.full_like(E, 3.0)
    c = 0.9
    _, _, tir, f = X.explicit_sources(E, rho, kap, [c * y, np.zeros_like(E)],
                                      prob)
    g = [(16.0 * np.sinh(k * h) - 2.0 * np.sinh(2.0 * k * h)) / (12.0 * h)
         for k in (kx, ky)]
    gm = np.hypot(g[0], g[1])
    R = gm / 1.5
    lam = (2.0 + R) / (6.0 + 3.0 * R + R * R)
    fe = lam + lam * lam * R * R
    expect = E * 0.5 * (3.0 * fe - 1.0) * (g[0] / gm) * (g[1] / gm) * c
    np.testing.assert_allclose(f[INNER], fe, rtol=1e-12)
    np.testing.assert_allclose(tir[INNER], expect[INNER], rtol=1e-11)


def test_uniform_motion_does_no_work_on_radiation():
    """A uniform velocity has grad v = 0: no photon tiring (3D, periodic)."""
    n = (8, 6, 10)
    prob = _prob(n, ["periodic"] * 3)
    rng = np.random.default_rng(5)
    E = np.exp(0.3 * rng.standard_normal((10, 6, 8)))
    rho = np.exp(rng.standard_normal(E.shape))
    kap = np.exp(rng.standard_normal(E.shape))
    v = [np.full_like(E, 0.3), np.full_like(E, -1.2), np.full_like(E, 2.0)]
    fr, work, tir, _ = X.explicit_sources(E, rho, kap, v, prob)
    np.testing.assert_allclose(tir, 0.0, atol=1e-12)
    np.testing.assert_allclose(work, 0.3 * fr[0] - 1.2 * fr[1] + 2.0 * fr[2],
                               rtol=1e-13, atol=1e-14)
