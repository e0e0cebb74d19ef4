"""FP64 CPU oracle of the explicit FLD source terms.

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path.
Shares no code with the HIP library.

Sect. 3 adds three terms explicitly around the implicit radiation update,
all built from the same five-point gradient of E, R and flux limiter as the
diffusion coefficient (eqs. fld_F, fld_lambda, fld_R):

* the radiation force density f_r = rho kappa F / c (eq. rad_force) with the
  flux of eq. fld_F, i.e. f_r = -lambda grad E;
* its work term v . f_r (the gas energy equation's source);
* photon tiring P : grad v, with the radiation pressure tensor P = f E
  (eq. fld_P), the Eddington tensor
  f_ij = (1 - f)/2 delta_ij + (3 f - 1)/2 n_i n_j (eq. fld_Eddington_tensor),
  n = grad E / |grad E|, and the Eddington factor f = lambda + lambda^2 R^2
  (eq. fld_f); grad v by the same five-point stencil (Sect. 3).

Readings: everything lives at cell centres, with the coefficient stage's
ghost cells (periodic wrap or Neumann mirror ghosts) for E and for every
velocity component; where grad E = 0, n is taken as 0 (there R = 0, so
f = 1/3 and the n n term has weight 0 anyway).  Only derivatives along the
grid's dimensions exist, so P : grad v = sum over i, j < ndim of
P_ij d_i v_j (a velocity component across the grid has no derivative, and
its n component is 0).
"""
from __future__ import annotations

import numpy as np

from . import fldref as F


def explicit_sources(E, rho, kappa, v, prob):
    """Returns (f_r, work, tiring, f): f_r a list of ndim arrays, work =
    v . f_r, tiring = P : grad v, f the Eddington factor.  v: a list of
    ndim velocity arrays (x, y, z order), each shaped like E."""
    nd = prob.ndim
    G = F.gradient(E, prob)
    gmag = np.sqrt(sum(g * g for g in G))
    R = gmag / (rho * kappa * E)
    lam = F.limiter(R, prob.limiter)
    fr = [-lam * g for g in G]
    work = sum(v[d] * fr[d] for d in range(nd))
    f = F.eddington_factor(lam, R)
    safe = np.where(gmag > 0.0, gmag, 1.0)
    n = [np.where(gmag > 0.0, g / safe, 0.0) for g in G]
    # dv[i][j] = d v_j / d x_i
    grads = [F.gradient(v[j], prob) for j in range(nd)]
    tiring = np.zeros_like(E)
    for i in range(nd):
        for j in range(nd):
            t_ij = 0.5 * (3.0 * f - 1.0) * n[i] * n[j]
            if i == j:
                t_ij = t_ij + 0.5 * (1.0 - f)
            tiring = tiring + t_ij * grads[j][i]
    tiring = E * tiring
    return fr, work, tiring, f


def eddington_tensor(f, n):
    """The 3x3 Eddington tensor of eq. fld_Eddington_tensor for a scalar
    factor f and a unit vector n (three components)."""
    n = np.asarray(n, dtype=np.float64)
    return 0.5 * (1.0 - f) * np.eye(3) + 0.5 * (3.0 * f - 1.0) * np.outer(n, n)
