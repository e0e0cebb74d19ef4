"""The FP64 oracle behind the library's three calls, on host arrays.

TEST INFRASTRUCTURE ONLY: tests drive the GPU library (fld_setup / fld_step
/ fld_exchange) and this module with the same parameters.  It shares no code
with the HIP path and does not import the library: parameters are a plain
mapping with the field names and codes of the library's parameter struct
(ndim, n, dx, bc_lo, bc_hi with 0 = periodic / 1 = Neumann, c, a_rad,
gamma, gas_const, limiter with 0 = Levermore-Pomraning / 1 = 1/3 /
2 = Minerbo,
face_mean with 0 = arithmetic / 1 = harmonic).

fldref_step returns the exact backward-Euler diffusion solve E* = A^-1 E^n
(eq. mhd_r_e with v = 0 and the exchange split off; D from E^n) and the
relative residual of what it returns; fldref_exchange the implicit
gas-radiation exchange (eqs. heating, qdot: one quartic per cell).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import fldref as F


@dataclasses.dataclass
class RefCtx:
    prob: F.Problem
    rtol: float


def fldref_setup(params):
    """params: mapping with the fields named in the module docstring."""
    p = dict(params)
    nd = int(p["ndim"])
    if nd not in (1, 2, 3):
        raise ValueError("ndim must be 1, 2 or 3")
    n = tuple(int(v) for v in p["n"])[:3]
    n = n + (1,) * (3 - len(n))
    dx = tuple(float(v) for v in p["dx"])[:3]
    dx = dx + (1.0,) * (3 - len(dx))
    lo = list(p.get("bc_lo", [0, 0, 0]))
    hi = list(p.get("bc_hi", lo))
    if lo[:nd] != hi[:nd]:
        raise ValueError("both sides of a dimension need the same condition")
    bc = tuple(F.PERIODIC if lo[d] == 0 else F.NEUMANN for d in range(nd))
    prob = F.Problem(
        ndim=nd, n=n, dx=dx, bc=bc, c=float(p.get("c", 1.0)),
        a_rad=float(p.get("a_rad", 1.0)), gamma=float(p.get("gamma", 5.0 / 3.0)),
        gas_const=float(p.get("gas_const", 1.0)),
        limiter=("lp", "diffusion", "minerbo")[int(p.get("limiter", 0))],
        face_mean="arith" if int(p.get("face_mean", 0)) == 0 else "harmonic")
    return RefCtx(prob=prob, rtol=float(p.get("rtol", 1e-13)))


def _field(ctx, a, name):
    a = np.asarray(a, dtype=np.float64)
    shape = ctx.prob.shape
    if a.size != int(np.prod(shape)):
        raise ValueError(f"{name} has {a.size} cells, the grid {int(np.prod(shape))}")
    return a.reshape(shape)


def fldref_step(ctx, dt, rho, kappa, E_in):
    """(E*, stats): the exact diffusion step and its relative residual."""
    if not (dt > 0.0):
        raise ValueError("dt must be positive")
    rho, kappa, E = (_field(ctx, a, k) for a, k in
                     ((rho, "rho"), (kappa, "kappa"), (E_in, "E_in")))
    alphas = F.face_coefficients(E, rho, kappa, dt, ctx.prob)
    x = F.solve(alphas, E, ctx.prob, rtol=min(ctx.rtol, 1e-13))
    res = F.relative_residual(x, E, alphas, ctx.prob)
    return x, {"rel_res_final": res,
               "rel_res_initial": F.relative_residual(E, E, alphas, ctx.prob)}


def fldref_exchange(ctx, dt, rho, kappa, E, e_int):
    """(E^{n+1}, e^{n+1}) of the implicit exchange."""
    rho, kappa, E, e = (_field(ctx, a, k) for a, k in
                        ((rho, "rho"), (kappa, "kappa"), (E, "E"),
                         (e_int, "e_int")))
    return F.exchange(E, e, rho, kappa, dt, ctx.prob)
