"""Linear modes of a static, uniform radiating medium (Appendix B).

TEST INFRASTRUCTURE ONLY (pins for the oracle; never used by the product).

``octic_coefficients`` writes out the dispersion relation of Appendix B
(eq. dispersion_relation_simplified): the Alfven quadratic times the hexic
in omega, for k = (k, 0, 0).  Two readings make it reproduce Tables 2 and 3:
the last bracket of the omega^1 coefficient is taken with qdot_{T_r} (the
printed qdot_{T_g} there makes the slow mode grow), and the Alfven speeds
use v_A^2 = B^2 / (4 pi rho) for B in Gauss.

``static_rate_matrix`` is the same linearisation restricted to what the FLD
update itself contains (v = 0, rho_1 = 0, lambda = 1/3): gas pressure and
radiation energy perturbations coupled by the heating/cooling derivatives
(eqs. qdot_Tr, qdot_Tg) and damped by radiative diffusion c k^2 / (3 rho kappa).
"""
from __future__ import annotations

import numpy as np


def background(rho0, p0, mu, gamma, kappa, k_B, m_p, a_r, c):
    """Equilibrium temperature, E0 and the qdot derivatives (eqs. qdot_*)."""
    T0 = p0 * mu * m_p / (rho0 * k_B)
    E0 = a_r * T0 ** 4
    q_Tr = 4.0 * c * rho0 * kappa * a_r * T0 ** 3
    q_Tg = -4.0 * c * rho0 * kappa * a_r * T0 ** 3
    return dict(T0=T0, E0=E0, q_Tr=q_Tr, q_Tg=q_Tg)


def octic_coefficients(rho0, p0, B0, mu, gamma, kappa, k, k_B, m_p, a_r, c):
    """Coefficients (highest power first) of the octic in omega."""
    bg = background(rho0, p0, mu, gamma, kappa, k_B, m_p, a_r, c)
    T0, E0, qTr, qTg = bg["T0"], bg["E0"], bg["q_Tr"], bg["q_Tg"]
    g = gamma
    cg2 = g * p0 / rho0
    cr2 = 4.0 * E0 / (9.0 * rho0)
    vA2 = (B0[0] ** 2 + B0[1] ** 2 + B0[2] ** 2) / (4.0 * np.pi * rho0)
    vAx2 = B0[0] ** 2 / (4.0 * np.pi * rho0)
    Dk = c / (3.0 * rho0 * kappa)  # diffusion coefficient, lambda = 1/3
    k2, k4, k6 = k ** 2, k ** 4, k ** 6
    h = np.zeros(7, dtype=complex)  # hexic, omega^6 ... omega^0
    h[0] = 1.0
    h[1] = 1j * (Dk * k2 + qTr * T0 / (4.0 * E0) - (g - 1.0) * qTg * T0 / p0)
    h[2] = -k2 * (cr2 + cg2 + vA2 - (g - 1.0) * qTg * (T0 / p0) * Dk)
    h[3] = 1j * k2 * (-Dk * k2 * (cg2 + vA2)
                      + (g - 1.0) * qTg * (T0 / rho0)
                      * (4.0 / 3.0 + g * cr2 / cg2 + g * vA2 / cg2)
                      - qTr * (T0 / rho0)
                      * (cg2 / (9.0 * cr2) + (g - 1.0) / 3.0 + vA2 / (9.0 * cr2)))
    h[4] = k4 * ((g - 1.0) * (-qTg * (T0 / rho0) * Dk) * (1.0 + g * vA2 / cg2)
                 + vAx2 * (cr2 + cg2))
    h[5] = 1j * k4 * vAx2 * (k2 * cg2 * Dk
                             - qTg * (T0 / rho0) * (g - 1.0)
                             * (g * cr2 / cg2 + 4.0 / 3.0)
                             + qTr * (T0 / rho0)
                             * ((g - 1.0) / 3.0 + cg2 / (9.0 * cr2)))
    h[6] = k6 * (g - 1.0) * vAx2 * qTg * (T0 / rho0) * Dk
    alfven = np.array([1.0, 0.0, -k2 * vAx2], dtype=complex)
    return np.convolve(alfven, h)


def octic_roots(**kw):
    return np.roots(octic_coefficients(**kw))


def static_rate_matrix(rho0, p0, mu, gamma, kappa, k, k_B, m_p, a_r, c):
    """d/dt [p1, E1] = M [p1, E1] for v = 0, rho1 = 0, lambda = 1/3.

    From eqs. mhd_energy_lin and mhd_r_e_lin with T_g1 = T0 p1 / p0 and
    T_r1 = T0 E1 / (4 E0):
      dp1/dt = (gamma-1) (qdot_Tg T0/p0 p1 + qdot_Tr T0/(4E0) E1)
      dE1/dt = -(qdot_Tg T0/p0 p1 + qdot_Tr T0/(4E0) E1) - c k^2/(3 rho kappa) E1
    """
    bg = background(rho0, p0, mu, gamma, kappa, k_B, m_p, a_r, c)
    Qg = bg["q_Tg"] * bg["T0"] / p0
    Qr = bg["q_Tr"] * bg["T0"] / (4.0 * bg["E0"])
    Dk2 = c * k * k / (3.0 * rho0 * kappa)
    return np.array([[(gamma - 1.0) * Qg, (gamma - 1.0) * Qr],
                     [-Qg, -(Qr + Dk2)]])
