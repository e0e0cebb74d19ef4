"""Pins of the oracle's backward-Euler diffusion solve.

Closed forms: with lambda = 1/3 and uniform rho kappa the operator is
diagonal in Fourier (periodic) and cosine (Neumann, DCT-II) modes, with
eigenvalues 1 + sum_d 4 alpha_d sin^2(theta_d / 2); these are computed
with scipy's FFT/DCT, independently of the oracle's assembly and solver.
Invariants: symmetry and lambda_min >= 1 of A, exact global conservation
(1^T A = 1^T), mirror symmetry, and the error bound |e| <= |r| that
follows from lambda_min(A) >= 1.
"""
import numpy as np
import pytest
import scipy.fft as sfft

from oracle import fldref as F


def _uniform(n, bc, dx, rhok=40.0, dt=2e-3, seed=0):
    ndim = len(n)
    shape = tuple(reversed(n))
    rng = np.random.default_rng(seed)
    prob = F.Problem(ndim=ndim, n=tuple(list(n) + [1] * (3 - ndim)),
                     dx=tuple(list(dx) + [1.0] * (3 - ndim)), bc=tuple(bc),
                     limiter="diffusion", c=1.7)
    rho = np.full(shape, 2.0)
    kap = np.full(shape, rhok / 2.0)
    E = 1.0 + 0.5 * rng.random(shape)
    return prob, rho, kap, E, dt


def _closed_form(prob, E, alpha):
    """Solve by transforming each axis (FFT periodic, DCT-II Neumann)."""
    Eh = E.astype(complex)
    denom = np.ones(E.shape)
    for d in range(prob.ndim):
        ax = prob.axis(d)
        n = E.shape[ax]
        sh = [1] * prob.ndim
        sh[ax] = n
        k = np.arange(n)
        if prob.bc[d] == "periodic":
            Eh = sfft.fft(Eh, axis=ax)
            theta = 2 * np.pi * k / n
        else:
            Eh = sfft.dct(Eh.real, type=2, axis=ax, norm="ortho") + \
                1j * sfft.dct(Eh.imag, type=2, axis=ax, norm="ortho")
            theta = np.pi * k / n
        denom = denom + (4 * alpha[d] * np.sin(theta / 2) ** 2).reshape(sh)
    Xh = Eh / denom
    for d in reversed(range(prob.ndim)):
        ax = prob.axis(d)
        if prob.bc[d] == "periodic":
            Xh = sfft.ifft(Xh, axis=ax)
        else:
            Xh = sfft.idct(Xh.real, type=2, axis=ax, norm="ortho") + \
                1j * sfft.idct(Xh.imag, type=2, axis=ax, norm="ortho")
    return Xh.real


CASES = [
    ((64,), ["periodic"], (1 / 64,)),
    ((64,), ["neumann"], (1 / 64,)),
    ((16, 12), ["periodic", "periodic"], (1 / 16, 1 / 12)),
    ((16, 12), ["neumann", "neumann"], (1 / 16, 1 / 12)),
    ((16, 12), ["periodic", "neumann"], (0.05, 0.11)),
    ((8, 6, 10), ["periodic", "periodic", "neumann"], (1 / 8, 1 / 6, 1 / 10)),
    ((8, 6, 10), ["neumann", "periodic", "neumann"], (0.2, 0.1, 0.15)),
]


@pytest.mark.parametrize("n,bc,dx", CASES)
def test_uniform_closed_form(n, bc, dx):
    prob, rho, kap, E, dt = _uniform(n, bc, dx)
    D = prob.c / (3.0 * rho.flat[0] * kap.flat[0])
    alpha = [dt * D / dx[d] ** 2 for d in range(len(n))]
    x = F.diffusion_step(E, rho, kap, dt, prob)
    ref = _closed_form(prob, E, alpha)
    assert np.abs(x - ref).max() / np.abs(ref).max() < 1e-13


def _random(n, bc, seed, limiter="lp", face_mean="arith"):
    ndim = len(n)
    shape = tuple(reversed(n))
    rng = np.random.default_rng(seed)
    prob = F.Problem(ndim=ndim, n=tuple(list(n) + [1] * (3 - ndim)),
                     dx=tuple([1.0 / v for v in n] + [1.0] * (3 - ndim)),
                     bc=tuple(bc), limiter=limiter, face_mean=face_mean)
    rho = np.exp(0.5 * rng.standard_normal(shape))
    kap = 10 * np.exp(rng.standard_normal(shape))
    E = np.exp(0.4 * rng.standard_normal(shape))
    return prob, rho, kap, E


@pytest.mark.parametrize("n,bc,dx", CASES)
def test_operator_spd_and_conservative(n, bc, dx):
    prob, rho, kap, E = _random(n, bc, 11)
    a = F.face_coefficients(E, rho, kap, 0.05, prob)
    A = F.assemble(a, prob).toarray()
    assert np.abs(A - A.T).max() == 0.0
    assert np.linalg.eigvalsh(A).min() >= 1.0 - 1e-12
    # column sums are one: sum(A x) = sum(x), so the solve conserves sum(E)
    np.testing.assert_allclose(A.sum(axis=0), 1.0, rtol=0, atol=1e-12)
    x = F.solve(a, E, prob)
    assert abs(x.sum() - E.sum()) <= 1e-12 * E.sum()
    # matrix-free operator agrees with the assembled matrix
    np.testing.assert_allclose(F.apply_operator(x, a, prob).ravel(),
                               A @ x.ravel(), rtol=1e-13)


def test_mirror_symmetry_c1():
    """A mirror-symmetric input gives a mirror-symmetric output."""
    import media
    m = media.config_c1()
    prob = F.problem_from_medium(m)
    x = F.diffusion_step(m.E, m.rho, m.kappa, m.dt, prob)
    # C1 is symmetric about x = 0 (cell centres at +-(i+1/2) dx)
    assert np.abs(x - x[::-1]).max() <= 1e-12 * x.max()


def test_solvers_agree_and_error_bound():
    prob, rho, kap, E = _random((48, 40), ["neumann", "periodic"], 5)
    a = F.face_coefficients(E, rho, kap, 0.3, prob)
    xd = F.solve(a, E, prob, method="dense")
    xs = F.solve(a, E, prob, method="splu")
    xc = F.solve(a, E, prob, method="cg", rtol=1e-14)
    for x in (xs, xc):
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-12
    # |x - x*| <= |b - A x| for any x, because lambda_min(A) >= 1
    y = xd + 1e-6 * np.random.default_rng(0).standard_normal(xd.shape)
    r = E - F.apply_operator(y, a, prob)
    assert np.linalg.norm(y - xd) <= np.linalg.norm(r) * (1 + 1e-9)


def test_gaussian_pulse_analytic():
    """Thick-limit diffusion of the 1D Gaussian pulse against the continuum.

    Diffusion only (no exchange), lambda = 1/3: E(x, t) is the periodic sum
    of spreading Gaussians with sigma_t^2 = sigma_0^2 + 2 D t.  Backward
    Euler converges at first order in dt; the LP limiter differs from 1/3 by
    about R^2/6 relative.
    """
    import media
    m = media.config_c1()
    D = m.c / (3.0 * 1.0 * 1.0e3)
    s0 = 0.02
    t_end = 10 * m.dt
    x = -0.5 + (np.arange(512) + 0.5) / 512

    def exact(t):
        st = np.sqrt(s0 ** 2 + 2 * D * t)
        return 1.0 + 10.0 * sum((s0 / st) * np.exp(-(x - k) ** 2 / (2 * st ** 2))
                                for k in (-2, -1, 0, 1, 2))

    errs = []
    for nsub in (1, 2, 4):
        prob = F.Problem(ndim=1, n=(512, 1, 1), dx=(1 / 512, 1, 1),
                         bc=("periodic",), limiter="diffusion")
        E = m.E.copy()
        dt = m.dt / nsub
        for _ in range(10 * nsub):
            E = F.diffusion_step(E, m.rho, m.kappa, dt, prob)
        errs.append(np.abs(E - exact(t_end)).max())
    # first order in dt (space error O(dx^2) ~ 1e-5 is far smaller)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.7 < r1 < 2.3 and 1.7 < r2 < 2.3, errs
    assert errs[2] < 0.02
    # LP limiter stays within R^2/6 of the diffusion value here
    prob = F.problem_from_medium(m)
    _, R, lam = F.diffusion_coefficient(m.E, m.rho, m.kappa, prob)
    assert R.max() < 0.07
    assert np.all(np.abs(3 * lam - 1) <= R ** 2 / 6 + 1e-15)


def test_fldref_api_drives_the_oracle_like_the_library():
    """The oracle's three calls (host arrays, library parameter names and
    codes) give what the oracle's functions give."""
    import numpy as np
    import media
    from oracle import fldref as F
    from oracle.fldref_api import fldref_exchange, fldref_setup, fldref_step
    m = media.random_small_medium(5, (12, 10), ("periodic", "neumann"))
    prob = F.problem_from_medium(m)
    ctx = fldref_setup(dict(ndim=2, n=(12, 10, 1), dx=m.dx, bc_lo=(0, 1, 0),
                            bc_hi=(0, 1, 0), c=1.0, a_rad=1.0, gamma=5 / 3,
                            gas_const=1.0, limiter=0, face_mean=0))
    x, st = fldref_step(ctx, m.dt, m.rho.ravel(), m.kappa.ravel(), m.E.ravel())
    ref = F.diffusion_step(m.E, m.rho, m.kappa, m.dt, prob, method="dense")
    assert np.allclose(x, ref, rtol=1e-12, atol=0)
    assert st["rel_res_final"] <= 1e-13
    En, en = fldref_exchange(ctx, m.dt, m.rho, m.kappa, x, m.e)
    En2, en2 = F.exchange(x, m.e, m.rho, m.kappa, m.dt, prob)
    assert np.array_equal(En, En2) and np.array_equal(en, en2)
