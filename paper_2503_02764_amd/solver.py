"""Convenience driver of whole split steps on device tensors.

``make_params`` fills an ``fld_params`` from plain grid/physics values and
``Stepper`` runs, per step and all through the C ABI: the opacity law (if
given), the diffusion solve ``fld_step`` and the exchange ``fld_exchange``.
"""
from __future__ import annotations

from . import fld

_BC = {"periodic": fld.FLD_BC_PERIODIC, "neumann": fld.FLD_BC_NEUMANN}
_LIM = {"lp": fld.FLD_LIMITER_LP, "diffusion": fld.FLD_LIMITER_DIFFUSION,
        "minerbo": fld.FLD_LIMITER_MINERBO}
_FACE = {"arith": fld.FLD_FACE_ARITH, "harmonic": fld.FLD_FACE_HARMONIC}
_PREC = {"fp64": fld.FLD_PREC_FP64, "fp32_ir": fld.FLD_PREC_FP32_IR}
_GUESS = {"prev": fld.FLD_GUESS_PREV, "zero": fld.FLD_GUESS_ZERO,
          "learned": fld.FLD_GUESS_LEARNED}
_POLICY = {"adaptive": fld.FLD_GUESS_ADAPTIVE,
           "every_step": fld.FLD_GUESS_EVERY_STEP}


def make_params(ndim, n, dx, bc, c=1.0, a_rad=1.0, gamma=5.0 / 3.0,
                gas_const=1.0, limiter="lp", face_mean="arith",
                precision="fp64", guess="prev", rtol=1e-8, max_cycles=50,
                pre_smooth=2, post_smooth=2, ir_inner=0, coarse_pre_smooth=0,
                coarse_post_smooth=0, guess_policy="adaptive", krylov=False,
                dirichlet=None, held_cells=False):
    """`bc`: "periodic" or "neumann" per dimension; `dirichlet`: optional
    {(d, side): E_w} (side 0 the lower wall of dimension d, 1 the upper)
    turning those walls of non-periodic dimensions into Dirichlet walls;
    `held_cells`: the context takes held cells (fld.fld_set_held)."""
    n = list(n) + [1] * (3 - len(n))
    dx = list(dx) + [1.0] * (3 - len(dx))
    codes = [_BC[b] for b in bc] + [fld.FLD_BC_PERIODIC] * (3 - len(bc))
    lo, hi = list(codes), list(codes)
    vlo, vhi = [0.0] * 3, [0.0] * 3
    for (d, side), v in (dirichlet or {}).items():
        (hi if side else lo)[d] = fld.FLD_BC_DIRICHLET
        (vhi if side else vlo)[d] = float(v)
    return fld.fld_params_default(
        ndim=ndim, n=n[:3], dx=dx[:3], bc_lo=lo, bc_hi=hi,
        bc_value_lo=vlo, bc_value_hi=vhi, c=c,
        a_rad=a_rad, gamma=gamma, gas_const=gas_const,
        limiter=_LIM[limiter], face_mean=_FACE[face_mean],
        precision=_PREC[precision], guess=_GUESS[guess], rtol=rtol,
        max_cycles=max_cycles, pre_smooth=pre_smooth,
        post_smooth=post_smooth, ir_inner=ir_inner,
        coarse_pre_smooth=coarse_pre_smooth,
        coarse_post_smooth=coarse_post_smooth,
        guess_policy=_POLICY[guess_policy], krylov=int(bool(krylov)),
        held_cells=int(bool(held_cells)))


class Stepper:
    """Split steps (opacity -> diffusion -> exchange) on device tensors."""

    def __init__(self, params, opacity=None, stream=None):
        self.ctx = fld.fld_setup(params, stream=stream)
        self.opacity = opacity

    def step(self, dt, rho, kappa, E, e, stats=True):
        """Advance (E, e) in place; kappa is overwritten if an opacity law
        is set.  Returns the fld_step statistics."""
        if self.opacity is not None:
            o = self.opacity
            fld.fld_opacity_powerlaw(self.ctx, rho, e, o["k0"], o["a"],
                                     o["b"], o["kmin"], o["kmax"], kappa)
        _, st = fld.fld_step(self.ctx, dt, rho, kappa, E, E, stats=stats)
        fld.fld_exchange(self.ctx, dt, rho, kappa, E, e)
        return st
