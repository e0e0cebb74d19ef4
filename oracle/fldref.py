"""FP64 CPU oracle of the implicit FLD radiation-energy update.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  Shares no code
with the HIP library.

What it computes (paper: Sect. 2, eqs. mhd_r_e, heating/qdot, fld_F,
fld_lambda, fld_R, ideal_gas_law, energy_density; Sect. 3, implicit
treatment of div F by multigrid and of qdot by a quartic):

1. ``face_coefficients``: the 4th-order five-point central gradient of E
   (Sect. 3), R = |grad E| / (rho kappa E) (eq. fld_R), the flux limiter
   (eq. fld_lambda, Levermore-Pomraning, or the diffusion value 1/3),
   D = c lambda / (rho kappa) (eq. fld_F) at cell centres, a face mean of D,
   and alpha_d = dt D_face / dx_d^2.
2. ``assemble`` / ``apply_operator``: the backward-Euler system of the
   diffusion part of eq. mhd_r_e with v = 0 and qdot split off,
   (A x)_i = x_i + sum over faces alpha_f (x_i - x_neighbour), b = E^n.
3. ``solve``: the exact solution E* = A^-1 b.  Multigrid in the paper is a
   fast way to this same vector; the oracle uses a direct factorisation
   (dense LU or sparse LU) or, for very large grids, conjugate gradients to
   a relative residual of 1e-13.
4. ``exchange``: the implicit heating/cooling update (eqs. heating, qdot)
   done for gas and radiation together, which conserves e + E per cell and
   leaves one quartic for e^{n+1}: a4 x^4 + (1 + beta) x - (e^n + beta S) = 0
   with beta = dt c kappa rho, S = E* + e^n, a4 = beta a_R ((gamma-1)/(rho R_g))^4
   (T from eqs. ideal_gas_law and energy_density).  The root is unique.
5. ``opacity_powerlaw``: kappa = k0 rho^a T^b clipped (a workload recipe,
   not the paper's constant opacity).

Readings where the paper is silent (all documented in the design notes):
limiter and D live at cell centres and faces take a mean of D; Neumann
("zero-gradient") boundaries use mirror ghosts for the gradient and zero
flux on the boundary face; D is lagged (computed from E^n); diffusion is
done before the exchange, one backward-Euler stage each.

A wall can instead hold E at a given value E_w (a Dirichlet wall: the
radiation temperature tied to the gas temperature on the boundary of the
magnetoconvection case, Sect. 4.5).  Readings: the gradient's ghosts are
the odd reflection about E_w (E_ghost = 2 E_w - E_mirror), and the wall
face, half a cell from the centre, carries the boundary cell's D:
(A x)_i gains alpha_w x_i and b_i gains alpha_w E_w, alpha_w = 2 dt D_i /
dx_d^2 (``dirichlet_terms``).

Cells can also be held at a prescribed new value (``held_step``, an
interior boundary: the linear-wave tests of Sect. 4.3 overwrite the first
wavelength of the domain).  Reading: their rows become x_i = E_hold_i and
free neighbours couple to them through the usual face coefficients.

Arrays are float64, C order, x fastest: shape (nx,), (ny, nx) or
(nz, ny, nx).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

PERIODIC = "periodic"
NEUMANN = "neumann"


@dataclasses.dataclass
class Problem:
    ndim: int
    n: tuple  # (nx, ny, nz)
    dx: tuple  # (dx, dy, dz)
    bc: tuple  # one of PERIODIC / NEUMANN per dimension
    c: float = 1.0
    a_rad: float = 1.0
    gamma: float = 5.0 / 3.0
    gas_const: float = 1.0  # R_g = k_B / (mu m_p)
    limiter: str = "lp"  # "lp", "diffusion" or "minerbo"
    face_mean: str = "arith"  # "arith" or "harmonic"
    # Dirichlet walls: {(d, side): E_w}, side 0 the lower wall of dimension
    # d and 1 the upper one; that dimension's bc must be NEUMANN
    dirichlet: dict = dataclasses.field(default_factory=dict)

    @property
    def shape(self):
        return tuple(reversed(self.n[: self.ndim]))

    def axis(self, d):
        """numpy axis of spatial dimension d (x = 0, y = 1, z = 2)."""
        return self.ndim - 1 - d


def problem_from_medium(m):
    return Problem(ndim=m.ndim, n=tuple(m.n), dx=tuple(m.dx), bc=tuple(m.bc),
                   c=m.c, a_rad=m.a_rad, gamma=m.gamma,
                   gas_const=m.gas_const, limiter=m.limiter,
                   face_mean=m.face_mean)


# ---------------------------------------------------------------------------
# Coefficient stage
# ---------------------------------------------------------------------------

def _with_ghosts(f, prob, width=2):
    """Pad every axis by ``width`` ghost cells.

    Periodic: wrap-around.  Neumann (zero gradient): mirror ghosts,
    f[-1] = f[0], f[-2] = f[1], and likewise at the upper end.
    """
    out = f
    for d in range(prob.ndim):
        ax = prob.axis(d)
        pad = [(0, 0)] * prob.ndim
        pad[ax] = (width, width)
        mode = "wrap" if prob.bc[d] == PERIODIC else "symmetric"
        out = np.pad(out, pad, mode=mode)
    return out


def gradient(E, prob):
    """Five-point 4th-order central gradient of E, one array per dimension.

    G_d = (E_{i-2} - 8 E_{i-1} + 8 E_{i+1} - E_{i+2}) / (12 dx_d)  (Sect. 3).
    A Dirichlet wall's ghosts are the odd reflection about its value,
    E_{-1} = 2 E_w - E_0, E_{-2} = 2 E_w - E_1 (mirror ghosts reflected).
    """
    Ep = _with_ghosts(E, prob, 2)
    for (d, side), Ew in prob.dirichlet.items():
        ax = prob.axis(d)
        for k in (0, 1):  # the two ghost layers of that wall
            sl = [slice(None)] * prob.ndim
            sl[ax] = k if side == 0 else Ep.shape[ax] - 1 - k
            Ep[tuple(sl)] = 2.0 * Ew - Ep[tuple(sl)]
    interior = [slice(2, -2)] * prob.ndim
    out = []
    for d in range(prob.ndim):
        ax = prob.axis(d)

        def shifted(s):
            sl = list(interior)
            n = E.shape[ax]
            sl[ax] = slice(2 + s, 2 + s + n)
            return Ep[tuple(sl)]

        G = (shifted(-2) - 8.0 * shifted(-1) + 8.0 * shifted(1)
             - shifted(2)) / (12.0 * prob.dx[d])
        out.append(G)
    return out


def limiter(R, kind="lp"):
    """Flux limiter lambda(R): eq. fld_lambda (LP), the diffusion value 1/3,
    or Minerbo's limiter, which Sect. 2 names after eq. fld_lambda without a
    formula; the published piecewise form is taken (Minerbo 1978):
    2 / (3 + sqrt(9 + 12 R^2)) up to R = 3/2, 1 / (1 + R + sqrt(1 + 2 R))
    beyond."""
    R = np.asarray(R, dtype=np.float64)
    if kind == "lp":
        return (2.0 + R) / (6.0 + 3.0 * R + R * R)
    if kind == "diffusion":
        return np.full_like(R, 1.0 / 3.0)
    if kind == "minerbo":
        low = 2.0 / (3.0 + np.sqrt(9.0 + 12.0 * R * R))
        high = 1.0 / (1.0 + R + np.sqrt(1.0 + 2.0 * R))
        return np.where(R <= 1.5, low, high)
    raise ValueError(kind)


def eddington_factor(lam, R):
    """Scalar Eddington factor f = lambda + lambda^2 R^2 (eq. fld_f)."""
    return lam + lam * lam * R * R


def diffusion_coefficient(E, rho, kappa, prob):
    """Cell-centred D = c lambda / (rho kappa) with R from eq. fld_R.

    Returns (D, R, lambda).
    """
    G = gradient(E, prob)
    gmag = np.sqrt(sum(g * g for g in G))
    R = gmag / (rho * kappa * E)
    lam = limiter(R, prob.limiter)
    D = prob.c * lam / (rho * kappa)
    return D, R, lam


def _face_mean(Dl, Dr, kind):
    if kind == "arith":
        return 0.5 * (Dl + Dr)
    if kind == "harmonic":
        return 2.0 * Dl * Dr / (Dl + Dr)
    raise ValueError(kind)


def face_coefficients(E, rho, kappa, dt, prob):
    """alpha_d[i] = dt * D_face / dx_d^2 on the face between cell i and i+e_d.

    The face of the last cell along a Neumann dimension is a wall: alpha = 0.
    Along a periodic dimension it couples the last cell to the first.
    """
    D, _, _ = diffusion_coefficient(E, rho, kappa, prob)
    alphas = []
    for d in range(prob.ndim):
        ax = prob.axis(d)
        Dr = np.roll(D, -1, axis=ax)
        a = dt * _face_mean(D, Dr, prob.face_mean) / (prob.dx[d] ** 2)
        if prob.bc[d] == NEUMANN:
            sl = [slice(None)] * prob.ndim
            sl[ax] = -1
            a[tuple(sl)] = 0.0
        alphas.append(a)
    return alphas


def dirichlet_terms(E, rho, kappa, dt, prob):
    """Diagonal and right-hand-side terms of the Dirichlet walls.

    For a cell on a Dirichlet wall along d the wall face lies half a cell
    away and carries the cell's D: the face flux is 2 D_i (E_i - E_w) /
    dx_d, so (A x)_i gains alpha_w x_i and b_i gains alpha_w E_w with
    alpha_w = 2 dt D_i / dx_d^2.  Returns (alpha_w summed per cell,
    alpha_w E_w summed per cell); zeros without Dirichlet walls.
    """
    diag = np.zeros(prob.shape)
    rhs = np.zeros(prob.shape)
    if not prob.dirichlet:
        return diag, rhs
    D, _, _ = diffusion_coefficient(E, rho, kappa, prob)
    for (d, side), Ew in prob.dirichlet.items():
        ax = prob.axis(d)
        sl = [slice(None)] * prob.ndim
        sl[ax] = 0 if side == 0 else -1
        sl = tuple(sl)
        aw = 2.0 * dt * D[sl] / (prob.dx[d] ** 2)
        diag[sl] += aw
        rhs[sl] += aw * Ew
    return diag, rhs


# ---------------------------------------------------------------------------
# Backward-Euler diffusion operator and its exact solution
# ---------------------------------------------------------------------------

def apply_operator(x, alphas, prob, diag=None):
    """(A x)_i = x_i + sum_faces alpha_f (x_i - x_neighbour) (+ the
    Dirichlet walls' diag_i x_i)."""
    Ax = x.copy()
    for d in range(prob.ndim):
        ax = prob.axis(d)
        flux = alphas[d] * (x - np.roll(x, -1, axis=ax))  # through face i+1/2
        Ax += flux
        Ax -= np.roll(flux, 1, axis=ax)  # face i-1/2 seen from cell i
    if diag is not None:
        Ax += diag * x
    return Ax


def assemble(alphas, prob, diag=None):
    """Sparse matrix of the operator in ``apply_operator`` (CSR, float64)."""
    shape = prob.shape
    N = int(np.prod(shape))
    idx = np.arange(N).reshape(shape)
    one = np.ones(N) if diag is None else 1.0 + diag.ravel()
    rows, cols, vals = [np.arange(N)], [np.arange(N)], [one]
    for d in range(prob.ndim):
        ax = prob.axis(d)
        nb = np.roll(idx, -1, axis=ax).ravel()
        a = alphas[d].ravel()
        i = idx.ravel()
        rows += [i, nb, i, nb]
        cols += [i, nb, nb, i]
        vals += [a, a, -a, -a]
    A = sp.coo_matrix((np.concatenate(vals),
                       (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return A.tocsr()


def solve(alphas, b, prob, rtol=1e-13, method=None, diag=None):
    """Exact solution of A x = b.

    Dense LU up to 4096 cells, sparse LU (SuperLU) up to ``SPLU_MAX`` cells,
    else Jacobi-preconditioned conjugate gradients (A is SPD) to ``rtol``.
    """
    A = assemble(alphas, prob, diag)
    N = A.shape[0]
    bf = b.ravel()
    if method is None:
        method = "dense" if N <= 4096 else ("splu" if N <= SPLU_MAX else "cg")
    if method == "dense":
        x = np.linalg.solve(A.toarray(), bf)
    elif method == "splu":
        x = spla.splu(A.tocsc()).solve(bf)
    elif method == "cg":
        dinv = 1.0 / A.diagonal()
        M = spla.LinearOperator(A.shape, matvec=lambda v: dinv * v)
        x, info = spla.cg(A, bf, x0=bf.copy(), rtol=rtol, atol=0.0, M=M,
                          maxiter=100000)
        if info != 0:
            raise RuntimeError(f"oracle CG did not converge (info={info})")
    else:
        raise ValueError(method)
    return x.reshape(b.shape)


SPLU_MAX = 1 << 18


def diffusion_step(E, rho, kappa, dt, prob, **kw):
    """E* = A^-1 b with A built from E^n (lagged D); b = E^n plus the
    Dirichlet walls' alpha_w E_w."""
    alphas = face_coefficients(E, rho, kappa, dt, prob)
    if not prob.dirichlet:
        return solve(alphas, E, prob, **kw)
    diag, rhs = dirichlet_terms(E, rho, kappa, dt, prob)
    return solve(alphas, E + rhs, prob, diag=diag, **kw)


def held_step(E, rho, kappa, dt, prob, held, E_hold, method=None):
    """Backward-Euler step with held cells: an interior boundary whose
    cells (``held`` true) take a prescribed new value ``E_hold`` (the
    linear-wave tests of Sect. 4.3 overwrite the first wavelength of the
    domain with a known solution).

    Reading: a held cell's row of the system becomes x_i = E_hold_i; every
    other row is the plain one (with the Dirichlet walls' terms), so a free
    cell next to a held one couples to the held value through the usual
    face coefficient: the held cells are interior Dirichlet data at cell
    centres.  D is still computed from E^n in every cell.  The system is no
    longer symmetric, so only the direct solves apply.
    """
    alphas = face_coefficients(E, rho, kappa, dt, prob)
    diag, rhs = dirichlet_terms(E, rho, kappa, dt, prob)
    A = assemble(alphas, prob, diag)
    h = np.asarray(held, dtype=bool).ravel()
    free_rows = sp.diags((~h).astype(np.float64))
    A = (free_rows @ A + sp.diags(h.astype(np.float64))).tocsr()
    b = np.where(held, E_hold, E + rhs).ravel()
    if method is None:
        method = "dense" if A.shape[0] <= 4096 else "splu"
    if method == "dense":
        x = np.linalg.solve(A.toarray(), b)
    elif method == "splu":
        x = spla.splu(A.tocsc()).solve(b)
    else:
        raise ValueError(f"held cells: direct solves only, not {method}")
    return x.reshape(E.shape)


def relative_residual(x, b, alphas, prob, diag=None):
    r = b - apply_operator(x, alphas, prob, diag)
    return float(np.linalg.norm(r.ravel()) / np.linalg.norm(b.ravel()))


# ---------------------------------------------------------------------------
# Gas-radiation energy exchange
# ---------------------------------------------------------------------------

def temperature(e, rho, prob):
    """Gas temperature from eqs. energy_density (v = B = 0) and ideal_gas_law."""
    return (prob.gamma - 1.0) * e / (rho * prob.gas_const)


def quartic_root(a4, a1, c0, max_iter=200):
    """Unique positive root of f(x) = a4 x^4 + a1 x - c0, a4 >= 0, a1, c0 > 0.

    f(0) < 0 and f is increasing and convex on x > 0, so Newton started at
    an upper bound decreases monotonically onto the root.  Upper bound:
    min(c0 / a1, (c0 / a4)^(1/4)); the root is at least half of it.  Each
    Newton iterate that leaves the bracket (rounding) is replaced by
    bisection.  Ends with one Newton correction evaluated in extended
    precision and rounded back to float64.
    """
    a4 = np.asarray(a4, dtype=np.float64)
    a1 = np.asarray(a1, dtype=np.float64)
    c0 = np.asarray(c0, dtype=np.float64)
    a4, a1, c0 = np.broadcast_arrays(a4, a1, c0)
    with np.errstate(divide="ignore"):
        u_quart = np.where(a4 > 0, (c0 / np.where(a4 > 0, a4, 1.0)) ** 0.25,
                           np.inf)
    hi = np.minimum(c0 / a1, u_quart)
    lo = 0.5 * hi
    x = hi.copy()
    for _ in range(max_iter):
        f = a4 * x ** 4 + a1 * x - c0
        hi = np.where(f > 0, x, hi)
        lo = np.where(f < 0, x, lo)
        fp = 4.0 * a4 * x ** 3 + a1
        xn = x - f / fp
        xn = np.where((xn >= lo) & (xn <= hi), xn, 0.5 * (lo + hi))
        moved = np.abs(xn - x) > 0.5 * np.spacing(x)
        x = xn
        if not np.any(moved):
            break
    # one Newton correction in extended precision
    X = x.astype(np.longdouble)
    A4 = a4.astype(np.longdouble)
    A1 = a1.astype(np.longdouble)
    C0 = c0.astype(np.longdouble)
    F = A4 * X ** 4 + A1 * X - C0
    FP = 4 * A4 * X ** 3 + A1
    return (X - F / FP).astype(np.float64)


def exchange(E_star, e, rho, kappa, dt, prob):
    """Implicit gas-radiation exchange; returns (E^{n+1}, e^{n+1}).

    Backward Euler on de/dt = qdot, dE/dt = -qdot with
    qdot = c kappa rho (E - a_R T^4) (eq. qdot).  Adding the two equations
    gives e^{n+1} + E^{n+1} = S = e^n + E*; substituting E^{n+1} = S - e^{n+1}
    into the gas equation leaves the quartic solved by ``quartic_root``.
    """
    beta = dt * prob.c * kappa * rho
    S = E_star + e
    a4 = beta * prob.a_rad * ((prob.gamma - 1.0) / (rho * prob.gas_const)) ** 4
    x = quartic_root(a4, 1.0 + beta, e + beta * S)
    return S - x, x


def opacity_powerlaw(rho, e, prob, k0, a, b, kmin, kmax):
    """kappa = clip(k0 rho^a T^b, kmin, kmax) with T the gas temperature."""
    T = temperature(e, rho, prob)
    return np.clip(k0 * rho ** a * T ** b, kmin, kmax)


# ---------------------------------------------------------------------------
# One split step
# ---------------------------------------------------------------------------

def step(E, e, rho, prob, dt, kappa=None, opacity=None, **solve_kw):
    """(E^n, e^n) -> diffusion -> exchange -> (E^{n+1}, e^{n+1}, E*).

    If ``opacity`` (a dict of power-law parameters) is given, kappa is
    evaluated once from the gas temperature at t^n and frozen for the step.
    """
    if opacity is not None:
        kappa = opacity_powerlaw(rho, e, prob, **opacity)
    E_star = diffusion_step(E, rho, kappa, dt, prob, **solve_kw)
    E_new, e_new = exchange(E_star, e, rho, kappa, dt, prob)
    return E_new, e_new, E_star
