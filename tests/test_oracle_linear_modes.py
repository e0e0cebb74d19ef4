"""Pins from the linear analysis of Appendix B and Tables 2-3.

1. The octic dispersion relation, written out with numpy, reproduces the
   eigenfrequencies the paper prints in Tables 2 and 3, and the equilibrium
   radiation energies E0 printed in Sect. 4.3 (this fixes the CGS constants
   and the two readings of the printed relation).
2. The static part of that linearisation (no flow) has two decaying modes,
   radiative diffusion and thermal; their rates match the paper's values.
3. The oracle's full split step (diffusion solve + exchange) on a small
   single-mode perturbation of the same uniform medium has exactly the
   amplification matrix predicted by the static linearisation for the
   discrete operators, and its rates approach the paper's numbers.
"""
import numpy as np
import pytest

from oracle import fldref as F
from oracle import linear_modes as L
from paper_pins import cgs, paper_values


def _case(name):
    pv = paper_values()[name]
    kw = dict(rho0=pv["rho0"], p0=pv["p0"], mu=pv["mu"], gamma=pv["gamma"],
              kappa=pv["kappa"], k=pv["k"], **cgs())
    return pv, kw


@pytest.mark.parametrize("name", ["linear_weak", "linear_strong"])
def test_octic_reproduces_tables(name):
    pv, kw = _case(name)
    roots = L.octic_roots(B0=pv["B0"], **kw)
    table = pv["roots"]
    for mode, (re, im) in table.items():
        target = complex(re, im)
        d = np.abs(roots - target)
        best = roots[np.argmin(d)]
        tol = 1e-3 if mode == "radiative_diffusion" else 1e-4
        assert abs(best - target) <= tol * abs(target), (mode, best, target)
        if re != 0.0:  # the mirrored root
            tgt2 = complex(-re, im)
            assert np.min(np.abs(roots - tgt2)) <= tol * abs(tgt2)
    bg = L.background(pv["rho0"], pv["p0"], pv["mu"], pv["gamma"],
                      pv["kappa"], cgs()["k_B"], cgs()["m_p"], cgs()["a_r"],
                      cgs()["c"])
    assert abs(bg["E0"] / pv["E0"] - 1) < 2e-5


@pytest.mark.parametrize("name,thermal_tol", [("linear_weak", 0.01),
                                               ("linear_strong", 0.03)])
def test_static_rates_vs_tables(name, thermal_tol):
    pv, kw = _case(name)
    rates = np.sort(-np.linalg.eigvals(L.static_rate_matrix(**kw)).real)
    thermal = -pv["roots"]["thermal"][1]
    radiative = -pv["roots"]["radiative_diffusion"][1]
    assert abs(rates[1] / radiative - 1) < 1e-3
    # the thermal mode keeps some hydrodynamic coupling in the full octic
    assert abs(rates[0] / thermal - 1) < thermal_tol


def _oracle_amplification(name, dt, n=128, eps=1e-7):
    """2x2 amplification of the (e, E) cos(kx) mode by one oracle step."""
    pv, kw = _case(name)
    C = cgs()
    k = pv["k"]
    lam_w = 2 * np.pi / k
    dx = lam_w / n
    gas_const = C["k_B"] / (pv["mu"] * C["m_p"])
    prob = F.Problem(ndim=1, n=(n, 1, 1), dx=(dx, 1, 1), bc=("periodic",),
                     c=C["c"], a_rad=C["a_r"], gamma=pv["gamma"],
                     gas_const=gas_const)
    rho = np.full(n, pv["rho0"])
    kap = np.full(n, pv["kappa"])
    e0 = pv["p0"] / (pv["gamma"] - 1)
    T0 = pv["p0"] / (pv["rho0"] * gas_const)
    E0 = C["a_r"] * T0 ** 4
    x = (np.arange(n) + 0.5) * dx
    mode = np.cos(k * x)
    base_E, base_e, _ = F.step(np.full(n, E0), np.full(n, e0), rho, prob, dt,
                               kappa=kap)
    G = np.zeros((2, 2))
    for j, (de, dE) in enumerate(((eps * e0, 0.0), (0.0, eps * E0))):
        En, en, _ = F.step(E0 + dE * mode, e0 + de * mode, rho, prob, dt,
                           kappa=kap)
        # project the response on the mode, in units relative to (e0, E0)
        G[0, j] = 2 / n * np.dot(en - base_e, mode) / (eps * e0)
        G[1, j] = 2 / n * np.dot(En - base_E, mode) / (eps * E0)
    scale = np.diag([1.0, 1.0])
    return G, prob, dict(e0=e0, E0=E0, T0=T0, dx=dx, kw=kw, scale=scale)


def _predicted_amplification(prob, info, dt):
    """Discrete prediction: linearised exchange after the diffusion solve."""
    C = cgs()
    kw = info["kw"]
    rho0, kap = kw["rho0"], kw["kappa"]
    k, dx = kw["k"], info["dx"]
    kh2 = 4.0 / dx ** 2 * np.sin(k * dx / 2) ** 2
    D = C["c"] / (3 * rho0 * kap)
    Gd = np.diag([1.0, 1.0 / (1.0 + dt * D * kh2)])
    # d/dt (e1/e0, E1/E0) for qdot = c kappa rho (E - a_R T^4), T1/T0 = e1/e0
    ckr = C["c"] * kap * rho0
    e0, E0 = info["e0"], info["E0"]
    M = np.array([[-4 * ckr * E0 / e0, ckr * E0 / e0],
                  [4 * ckr, -ckr]])
    Ge = np.linalg.inv(np.eye(2) - dt * M)
    return Ge @ Gd


@pytest.mark.parametrize("name", ["linear_weak", "linear_strong"])
def test_oracle_step_linear_response(name):
    pv, _ = _case(name)
    # radiative-diffusion mode: small dt resolves its rate
    dt_fast = 1e-6
    G, prob, info = _oracle_amplification(name, dt_fast)
    Gp = _predicted_amplification(prob, info, dt_fast)
    np.testing.assert_allclose(G, Gp, rtol=1e-5, atol=1e-8)
    g = np.sort(np.linalg.eigvals(G).real)
    rate_fast = -np.log(g[0]) / dt_fast
    radiative = -pv["roots"]["radiative_diffusion"][1]
    assert abs(rate_fast / radiative - 1) < 2e-3
    # thermal mode: a longer step, the radiative mode is then damped out
    dt_slow = 0.5
    G, prob, info = _oracle_amplification(name, dt_slow)
    Gp = _predicted_amplification(prob, info, dt_slow)
    np.testing.assert_allclose(G, Gp, rtol=1e-5, atol=1e-8)
    g = np.sort(np.linalg.eigvals(G).real)
    rate_slow = -np.log(g[1]) / dt_slow
    thermal = -pv["roots"]["thermal"][1]
    assert abs(rate_slow / thermal - 1) < 0.03
