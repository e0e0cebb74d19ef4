"""Pins of the oracle's coefficient stage (limiter, gradient, R, faces).

Checked against closed forms: the limits of eq. fld_lambda stated in
Sect. 2, the Eddington-factor limits of eq. fld_f, exactness of the
five-point stencil on quartic polynomials and its 4th-order convergence,
and the equivalence of mirror (Neumann) ghosts with a periodic, mirrored
domain of twice the size.
"""
import numpy as np
import pytest

from oracle import fldref as F


def test_limiter_limits():
    # optically thick limit lambda -> 1/3 (Sect. 2)
    assert F.limiter(0.0) == pytest.approx(1.0 / 3.0, rel=0, abs=0)
    R = np.logspace(-4, 8, 400)
    lam = F.limiter(R)
    # lambda decreasing in R (below 1e-4 the steps drown in rounding)
    assert np.all(np.diff(lam) < 0)
    # optically thin limit lambda -> 1/R, so |F| = D |grad E| -> c E
    assert abs(F.limiter(1e9) * 1e9 - 1.0) < 1e-8
    # diffusion-limit mode lambda == 1/3
    assert np.all(F.limiter(R, "diffusion") == 1.0 / 3.0)


def test_eddington_factor_limits():
    R = np.logspace(-8, 8, 400)
    f = F.eddington_factor(F.limiter(R), R)
    # thick limit f -> 1/3, thin limit f -> 1 (Sect. 2, eq. fld_f)
    assert abs(f[0] - 1.0 / 3.0) < 1e-8
    assert abs(f[-1] - 1.0) < 1e-7
    assert np.all(f >= 1.0 / 3.0 - 1e-15) and np.all(f <= 1.0 + 1e-15)


def _prob(n, bc, dx=None):
    ndim = len(n)
    nn = tuple(list(n) + [1] * (3 - ndim))
    if dx is None:
        dx = tuple([1.0 / v for v in n] + [1.0] * (3 - ndim))
    return F.Problem(ndim=ndim, n=nn, dx=dx, bc=tuple(bc))


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4])
def test_gradient_exact_on_quartics(deg):
    """The five-point stencil is exact for polynomials of degree <= 4."""
    rng = np.random.default_rng(deg)
    n = (12, 10, 9)
    prob = _prob(n, ["neumann"] * 3, dx=(0.3, 0.7, 1.1))
    coef = rng.standard_normal((3, deg + 1))
    z, y, x = np.meshgrid(*[np.arange(v) * prob.dx[d] for d, v in
                            reversed(list(enumerate(n)))], indexing="ij")
    coords = [x, y, z]
    E = sum(np.polyval(coef[d], coords[d]) for d in range(3))
    G = F.gradient(E, prob)
    for d in range(3):
        exact = np.polyval(np.polyder(coef[d]), coords[d])
        ax = prob.axis(d)
        sl = [slice(None)] * 3
        sl[ax] = slice(2, -2)  # interior: the stencil does not touch ghosts
        err = np.abs(G[d][tuple(sl)] - exact[tuple(sl)]).max()
        assert err <= 1e-10 * (1 + np.abs(exact).max())


def test_gradient_fourth_order_periodic():
    errs = []
    for n in (32, 64, 128):
        prob = _prob((n,), ["periodic"])
        x = np.arange(n) / n
        E = 2.0 + np.sin(2 * np.pi * x)
        G = F.gradient(E, prob)[0]
        errs.append(np.abs(G - 2 * np.pi * np.cos(2 * np.pi * x)).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 4.0) < 0.1), rates


def _mirror_double(f, axis):
    return np.concatenate([f, np.flip(f, axis=axis)], axis=axis)


@pytest.mark.parametrize("limiter", ["lp", "diffusion"])
@pytest.mark.parametrize("face_mean", ["arith", "harmonic"])
def test_neumann_equals_mirrored_periodic(limiter, face_mean):
    """Mirror ghosts + wall faces == periodic domain of the even extension."""
    rng = np.random.default_rng(7)
    ny, nx = 6, 10
    E = np.exp(0.4 * rng.standard_normal((ny, nx)))
    rho = np.exp(0.3 * rng.standard_normal((ny, nx)))
    kap = 5.0 * np.exp(rng.standard_normal((ny, nx)))
    pn = F.Problem(ndim=2, n=(nx, ny, 1), dx=(0.1, 0.2, 1.0),
                   bc=("neumann", "periodic"), limiter=limiter,
                   face_mean=face_mean)
    pp = F.Problem(ndim=2, n=(2 * nx, ny, 1), dx=(0.1, 0.2, 1.0),
                   bc=("periodic", "periodic"), limiter=limiter,
                   face_mean=face_mean)
    Dn, Rn, _ = F.diffusion_coefficient(E, rho, kap, pn)
    Dp, Rp, _ = F.diffusion_coefficient(_mirror_double(E, 1),
                                        _mirror_double(rho, 1),
                                        _mirror_double(kap, 1), pp)
    np.testing.assert_allclose(Rn, Rp[:, :nx], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(Dn, Dp[:, :nx], rtol=1e-13)
    # and the solve: Neumann solution equals the mirrored periodic solution
    dt = 3e-3
    xn = F.diffusion_step(E, rho, kap, dt, pn)
    xp = F.diffusion_step(_mirror_double(E, 1), _mirror_double(rho, 1),
                          _mirror_double(kap, 1), dt, pp)
    np.testing.assert_allclose(xn, xp[:, :nx], rtol=1e-12)


def test_R_closed_form_linear_profile():
    """E = 1 + s x with constant rho kappa: R = |s| / (rho kappa E) inside."""
    n = 40
    prob = _prob((n,), ["neumann"])
    x = (np.arange(n) + 0.5) / n
    s = 3.0
    E = 1.0 + s * x
    rho = np.full(n, 2.0)
    kap = np.full(n, 1.5)
    _, R, lam = F.diffusion_coefficient(E, rho, kap, prob)
    Rex = s / (rho * kap * E)
    np.testing.assert_allclose(R[2:-2], Rex[2:-2], rtol=1e-12)
    np.testing.assert_allclose(lam[2:-2], (2 + Rex[2:-2]) /
                               (6 + 3 * Rex[2:-2] + Rex[2:-2] ** 2),
                               rtol=1e-12)


def test_face_means_order_and_walls():
    rng = np.random.default_rng(3)
    n = (9, 8)
    E = np.exp(0.3 * rng.standard_normal((8, 9)))
    rho = np.exp(rng.standard_normal((8, 9)))
    kap = np.exp(rng.standard_normal((8, 9)))
    pa = F.Problem(ndim=2, n=(9, 8, 1), dx=(1 / 9, 1 / 8, 1),
                   bc=("neumann", "neumann"), face_mean="arith")
    ph = F.Problem(ndim=2, n=(9, 8, 1), dx=(1 / 9, 1 / 8, 1),
                   bc=("neumann", "neumann"), face_mean="harmonic")
    aa = F.face_coefficients(E, rho, kap, 0.1, pa)
    ah = F.face_coefficients(E, rho, kap, 0.1, ph)
    for d in range(2):
        # harmonic mean <= arithmetic mean (AM-HM inequality)
        assert np.all(ah[d] <= aa[d] * (1 + 1e-15))
    # wall faces carry no flux
    assert np.all(aa[0][:, -1] == 0) and np.all(aa[1][-1, :] == 0)
    del n


# ---------------------------------------------------------------------------
# Hand-computed face coefficients (distinct D on every face)
#
# With the diffusion limiter (lambda = 1/3), rho = 1 and c = 3 the cell
# value is D = c lambda / (rho kappa) = 1 / kappa (eq. fld_F), so kappa
# fixes D exactly.  alpha_d = dt D_face / dx_d^2 on the face between a cell
# and its upper neighbour along d; a Neumann wall face carries 0.
#   arithmetic mean:  (D_L + D_R) / 2
#   harmonic mean:    2 D_L D_R / (D_L + D_R)
# Every expected value below was worked out by hand from those two lines.
# ---------------------------------------------------------------------------

def _hand_problem(n, bc, dx, face_mean):
    ndim = len(n)
    return F.Problem(ndim=ndim, n=tuple(list(n) + [1] * (3 - ndim)),
                     dx=tuple(list(dx) + [1.0] * (3 - ndim)), bc=tuple(bc),
                     c=3.0, limiter="diffusion", face_mean=face_mean)


@pytest.mark.parametrize("face_mean,expect_neu,expect_per", [
    # D = (1, 1/2, 1/4), dt / dx^2 = 1
    ("arith", [0.75, 0.375, 0.0], [0.75, 0.375, 0.625]),
    ("harmonic", [2.0 / 3.0, 1.0 / 3.0, 0.0], [2.0 / 3.0, 1.0 / 3.0, 0.4]),
])
def test_face_means_hand_values_1d(face_mean, expect_neu, expect_per):
    kap = np.array([1.0, 2.0, 4.0])
    rho = np.ones(3)
    E = np.array([1.0, 3.0, 2.0])  # any positive E: lambda = 1/3 here
    for bc, expect in (("neumann", expect_neu), ("periodic", expect_per)):
        prob = _hand_problem((3,), [bc], (0.5,), face_mean)
        a = F.face_coefficients(E, rho, kap, 0.25, prob)[0]
        np.testing.assert_allclose(a, expect, rtol=1e-15, atol=0)


def test_operator_entries_hand_values_1d():
    """A = I + sum_faces alpha (difference)^T (difference), written out for
    the Neumann case above (arithmetic mean): alpha = (0.75, 0.375, wall)."""
    kap = np.array([1.0, 2.0, 4.0])
    prob = _hand_problem((3,), ["neumann"], (0.5,), "arith")
    al = F.face_coefficients(np.ones(3), np.ones(3), kap, 0.25, prob)
    A = F.assemble(al, prob).toarray()
    expect = np.array([[1.75, -0.75, 0.0],
                       [-0.75, 2.125, -0.375],
                       [0.0, -0.375, 1.375]])
    np.testing.assert_allclose(A, expect, rtol=1e-15, atol=0)
    v = np.array([2.0, -1.0, 0.5])
    # A v by hand: 1.75*2 + 0.75 = 4.25; -1.5 - 2.125 - 0.1875 = -3.8125;
    # 0.375 + 0.6875 = 1.0625
    np.testing.assert_allclose(F.apply_operator(v, al, prob),
                               [4.25, -3.8125, 1.0625], rtol=1e-15)
    # and the periodic case couples cell 2 to cell 0 through 0.625
    pp = _hand_problem((3,), ["periodic"], (0.5,), "arith")
    Ap = F.assemble(F.face_coefficients(np.ones(3), np.ones(3), kap, 0.25,
                                        pp), pp).toarray()
    np.testing.assert_allclose(Ap, [[2.375, -0.75, -0.625],
                                    [-0.75, 2.125, -0.375],
                                    [-0.625, -0.375, 2.0]], rtol=1e-15)


@pytest.mark.parametrize("face_mean,ax_expect,ay_expect", [
    ("arith",
     [[0.75, 0.375, 0.0], [0.375, 0.1875, 0.0]],
     [[3.0, 1.5, 0.75], [0.0, 0.0, 0.0]]),
    ("harmonic",
     [[2.0 / 3.0, 1.0 / 3.0, 0.0], [1.0 / 3.0, 1.0 / 6.0, 0.0]],
     [[8.0 / 3.0, 4.0 / 3.0, 2.0 / 3.0], [0.0, 0.0, 0.0]]),
])
def test_face_means_hand_values_2d(face_mean, ax_expect, ay_expect):
    """nx = 3, ny = 2, Neumann; kappa rows (1, 2, 4) and (2, 4, 8), so
    D rows (1, 1/2, 1/4) and (1/2, 1/4, 1/8); dx = 0.5, dy = 0.25, dt = 0.25:
    dt/dx^2 = 1 along x, dt/dy^2 = 4 along y (a swapped axis or spacing
    changes every entry)."""
    kap = np.array([[1.0, 2.0, 4.0], [2.0, 4.0, 8.0]])
    prob = _hand_problem((3, 2), ["neumann", "neumann"], (0.5, 0.25),
                         face_mean)
    ax, ay = F.face_coefficients(np.ones((2, 3)), np.ones((2, 3)), kap, 0.25,
                                 prob)
    np.testing.assert_allclose(ax, ax_expect, rtol=1e-15, atol=0)
    np.testing.assert_allclose(ay, ay_expect, rtol=1e-15, atol=0)


def test_minerbo_limiter_hand_values_and_limits():
    """Minerbo's limiter (its published piecewise form; Sect. 2 names it
    without a formula): lambda(0) = 1/3; at R = 1 the lower branch gives
    2 / (3 + sqrt 21) = 0.263763...; at R = 3/2 both branches give 2/9
    (2 / (3 + 6) and 1 / (1 + 3/2 + 2)); at R = 4, 1 / (5 + 3) = 1/8;
    decreasing; lambda R -> 1 in the free-streaming limit; below LP's
    value for R > 0."""
    lam = F.limiter
    assert lam(0.0, "minerbo") == pytest.approx(1.0 / 3.0, rel=1e-15)
    assert lam(1.0, "minerbo") == pytest.approx(2.0 / (3.0 + np.sqrt(21.0)),
                                                rel=1e-15)
    # between R = 1 and 3/2 the lower branch still holds: at R = 6/5,
    # 2 / (3 + sqrt(9 + 17.28)) = 0.246105..., not the upper branch's
    # 1 / (2.2 + sqrt 3.4) = 0.247285...
    assert lam(1.2, "minerbo") == pytest.approx(
        2.0 / (3.0 + np.sqrt(26.28)), rel=1e-15)
    assert abs(lam(1.2, "minerbo") - 1.0 / (2.2 + np.sqrt(3.4))) > 1e-3
    assert lam(1.5, "minerbo") == pytest.approx(2.0 / 9.0, rel=1e-15)
    assert lam(1.5 + 1e-12, "minerbo") == pytest.approx(2.0 / 9.0, rel=1e-10)
    assert lam(4.0, "minerbo") == pytest.approx(0.125, rel=1e-15)
    R = np.logspace(-4, 8, 400)
    m = lam(R, "minerbo")
    assert np.all(np.diff(m) < 0)
    assert abs(lam(1e9, "minerbo") * 1e9 - 1.0) < 1e-4
    assert np.all(m < lam(R, "lp"))
