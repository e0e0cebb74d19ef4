"""FP64 CPU oracle of the backward-Euler FLD diffusion step on a 2D
block-adaptive grid: a base grid and one level of refined blocks
(``amr_step``), or several nested levels (``hier_step``, at the end).

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path.
Shares no code with the HIP library.

Paper: Sect. 3 solves the parabolic term of eq. mhd_r_e by geometric
multigrid on MPI-AMRVAC's block-adaptive (quadtree / octree) grids (Sect. 3
and 4.1 use several AMR levels); the physics per cell is that of
``fldref`` (eqs. fld_F, fld_lambda, fld_R, Sect. 3 five-point gradient).
The paper does not give the discretisation at refinement boundaries; the
readings taken here:

- Grid: a base grid of nx x ny cells (spacing dx, dy), tiled by blocks of
  b x b base cells.  A refined block is covered by 2b x 2b fine cells of
  half the spacing.  The unknowns are the leaf cells: the base cells
  outside refined blocks and every fine cell.
- D on each level from that level's view of E: the fine view takes the
  fine values inside refined blocks and copies each base value to its four
  fine cells elsewhere; the base view takes the base values outside refined
  blocks and the mean of the four fine children inside them.  The limiter,
  the five-point gradient and the walls are those of a uniform grid of the
  level's spacing (``fldref.diffusion_coefficient``).
- Faces between two leaf cells of one level: as on a uniform grid of that
  level, alpha = dt D_face / h^2 with the face mean of the two cells' D.
- A face between a fine leaf cell f and a base leaf cell c across a block
  edge: the flux runs between the two centres, 3/2 fine spacings apart, so
  the fine row gains beta (x_f - x_c) with beta = (2/3) dt D_face / h_f^2,
  and the base row gains beta (V_f / V_c) (x_c - x_f) = beta / 4 (x_c - x_f)
  from each of the two fine cells along its face: the flux leaving one
  side enters the other (conservation), and the system is symmetric in the
  volume-weighted inner product.
- A covered base cell's output is the mean of its four fine children.

Arrays: base fields (ny, nx); fine fields (nblocks, 2b, 2b), block k
covering base block ``blocks[k] = (bx, by)`` (base cells bx*b .. bx*b+b-1
along x), row-major (y, x) inside the block.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fldref as F


@dataclasses.dataclass
class AmrGrid:
    nx: int
    ny: int
    dx: float
    dy: float
    b: int  # base cells per block side
    bc: tuple  # (x, y): fldref.PERIODIC or fldref.NEUMANN
    blocks: list  # refined base blocks, (bx, by) each
    c: float = 1.0
    limiter: str = "lp"
    face_mean: str = "arith"

    def base_problem(self):
        return F.Problem(ndim=2, n=(self.nx, self.ny, 1),
                         dx=(self.dx, self.dy, 1.0), bc=tuple(self.bc),
                         c=self.c, limiter=self.limiter,
                         face_mean=self.face_mean)

    def fine_problem(self):
        return F.Problem(ndim=2, n=(2 * self.nx, 2 * self.ny, 1),
                         dx=(self.dx / 2, self.dy / 2, 1.0),
                         bc=tuple(self.bc), c=self.c, limiter=self.limiter,
                         face_mean=self.face_mean)

    def refined(self):
        """Base-resolution mask of the cells covered by refined blocks."""
        m = np.zeros((self.ny, self.nx), dtype=bool)
        for bx, by in self.blocks:
            m[by * self.b:(by + 1) * self.b, bx * self.b:(bx + 1) * self.b] = True
        return m


def fine_to_full(grid, fine, fill):
    """Fine-resolution (2ny, 2nx) array: the blocks' values where refined,
    ``fill`` (a (2ny, 2nx) array) elsewhere."""
    out = np.array(fill, dtype=np.float64, copy=True)
    s = 2 * grid.b
    for k, (bx, by) in enumerate(grid.blocks):
        out[by * s:(by + 1) * s, bx * s:(bx + 1) * s] = fine[k]
    return out


def full_to_fine(grid, full):
    s = 2 * grid.b
    return np.stack([full[by * s:(by + 1) * s, bx * s:(bx + 1) * s]
                     for bx, by in grid.blocks]) if grid.blocks else \
        np.zeros((0, s, s))


def inject(base):
    """Each base value copied to its four fine cells."""
    return np.repeat(np.repeat(base, 2, axis=0), 2, axis=1)


def child_mean(full_fine):
    """Mean of the four fine children of every base cell."""
    f = full_fine
    return 0.25 * (f[0::2, 0::2] + f[1::2, 0::2] + f[0::2, 1::2] + f[1::2, 1::2])


def level_views(grid, base, fine):
    """(base view, fine view) of one field, as the readings define them."""
    ref = grid.refined()
    fine_full = fine_to_full(grid, fine, inject(base))
    base_view = np.where(ref, child_mean(fine_full), base)
    return base_view, fine_full


def coefficients(grid, Eb, rhob, kapb, Ef, rhof, kapf):
    """Cell-centred D on both levels: (D_base (ny, nx), D_fine (2ny, 2nx))."""
    views = [level_views(grid, bf, ff) for bf, ff in
             ((Eb, Ef), (rhob, rhof), (kapb, kapf))]
    Db, _, _ = F.diffusion_coefficient(views[0][0], views[1][0], views[2][0],
                                       grid.base_problem())
    Df, _, _ = F.diffusion_coefficient(views[0][1], views[1][1], views[2][1],
                                       grid.fine_problem())
    return Db, Df


def _mean(a, b, kind):
    return 0.5 * (a + b) if kind == "arith" else 2.0 * a * b / (a + b)


def leaf_numbering(grid):
    """Index of every leaf cell: base leaf cells first (row-major), then the
    fine cells block by block (row-major inside each block).  Returns
    (base index array (ny, nx), -1 where covered; fine index array
    (2ny, 2nx), -1 outside refined blocks; number of leaf cells)."""
    ref = grid.refined()
    bidx = np.full((grid.ny, grid.nx), -1, dtype=np.int64)
    nb = int(np.count_nonzero(~ref))
    bidx[~ref] = np.arange(nb)
    fidx = np.full((2 * grid.ny, 2 * grid.nx), -1, dtype=np.int64)
    s = 2 * grid.b
    k = nb
    for bx, by in grid.blocks:
        fidx[by * s:(by + 1) * s, bx * s:(bx + 1) * s] = \
            np.arange(k, k + s * s).reshape(s, s)
        k += s * s
    return bidx, fidx, k


def assemble(grid, Db, Df, dt):
    """Sparse composite operator (CSR) over the leaf cells, and their
    volumes."""
    bidx, fidx, N = leaf_numbering(grid)
    rows, cols, vals = [], [], []

    def couple(i, j, wi, wj):
        # row i gains wi (x_i - x_j), row j gains wj (x_j - x_i)
        rows.extend([i, i, j, j])
        cols.extend([i, j, j, i])
        vals.extend([wi, -wi, wj, -wj])

    per = [b == F.PERIODIC for b in grid.bc]
    h = [(grid.dx, grid.dy), (grid.dx / 2, grid.dy / 2)]
    # faces of the base level: between two base leaf cells
    for j in range(grid.ny):
        for i in range(grid.nx):
            if bidx[j, i] < 0:
                continue
            for d, (di, dj) in enumerate(((1, 0), (0, 1))):
                ii, jj = i + di, j + dj
                n = (grid.nx, grid.ny)[d]
                if (ii, jj)[d] == n:
                    if not per[d]:
                        continue
                    ii, jj = ii % grid.nx, jj % grid.ny
                if bidx[jj, ii] < 0:
                    continue  # a refined neighbour: its fine cells own the face
                a = dt * _mean(Db[j, i], Db[jj, ii], grid.face_mean) / h[0][d] ** 2
                couple(bidx[j, i], bidx[jj, ii], a, a)
    # faces of the fine level: to a fine neighbour (upper faces only) or to
    # a base leaf cell across a block edge (both sides)
    NX, NY = 2 * grid.nx, 2 * grid.ny
    for J in range(NY):
        for I in range(NX):
            if fidx[J, I] < 0:
                continue
            for d, (di, dj) in enumerate(((1, 0), (0, 1))):
                for sgn in (1, -1):
                    II, JJ = I + sgn * di, J + sgn * dj
                    n = (NX, NY)[d]
                    k = (II, JJ)[d]
                    if k < 0 or k >= n:
                        if not per[d]:
                            continue
                        II, JJ = II % NX, JJ % NY
                    if fidx[JJ, II] >= 0:
                        if sgn < 0:
                            continue  # counted from the lower cell
                        a = dt * _mean(Df[J, I], Df[JJ, II],
                                       grid.face_mean) / h[1][d] ** 2
                        couple(fidx[J, I], fidx[JJ, II], a, a)
                    else:
                        cb = (JJ // 2, II // 2)
                        beta = (2.0 / 3.0) * dt * _mean(
                            Df[J, I], Db[cb], grid.face_mean) / h[1][d] ** 2
                        couple(fidx[J, I], bidx[cb], beta, beta / 4.0)
    rows.extend(range(N))
    cols.extend(range(N))
    vals.extend([1.0] * N)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsr()
    vol = np.empty(N)
    vb = grid.dx * grid.dy
    nbase = int(np.count_nonzero(bidx >= 0))
    vol[:nbase] = vb
    vol[nbase:] = vb / 4.0
    return A, vol


def to_leaf(grid, base, fine):
    bidx, fidx, N = leaf_numbering(grid)
    v = np.empty(N)
    v[bidx[bidx >= 0]] = base[bidx >= 0]
    full = fine_to_full(grid, fine, np.zeros((2 * grid.ny, 2 * grid.nx)))
    v[fidx[fidx >= 0]] = full[fidx >= 0]
    return v


def from_leaf(grid, v):
    """(base (ny, nx), fine (nblocks, 2b, 2b)); covered base cells get the
    mean of their four fine children."""
    bidx, fidx, _ = leaf_numbering(grid)
    full = np.zeros((2 * grid.ny, 2 * grid.nx))
    full[fidx >= 0] = v[fidx[fidx >= 0]]
    base = np.where(bidx >= 0, v[np.maximum(bidx, 0)], child_mean(full))
    return base, full_to_fine(grid, full)


def amr_step(grid, Eb, rhob, kapb, Ef, rhof, kapf, dt, method="splu"):
    """E* = A^-1 E^n on the leaf cells, D lagged from E^n."""
    Db, Df = coefficients(grid, Eb, rhob, kapb, Ef, rhof, kapf)
    A, _ = assemble(grid, Db, Df, dt)
    b = to_leaf(grid, Eb, Ef)
    if method == "dense":
        x = np.linalg.solve(A.toarray(), b)
    else:
        x = spla.splu(A.tocsc()).solve(b)
    return from_leaf(grid, x)


# ---------------------------------------------------------------------------
# Deeper hierarchies: refined blocks inside refined blocks
# ---------------------------------------------------------------------------
#
# Readings (the same as one level, applied between each level and the next
# coarser one): level l has spacing dx / 2^l on a lattice of 2^l nx x 2^l ny
# cells; a block of level l >= 1 refines a b x b patch of level l-1 cells
# (its corner (bx, by) counted in units of b level-(l-1) cells) into 2b x 2b
# level-l cells, and that patch must lie inside a level-(l-1) block (the
# base for l = 1).  A leaf cell's face neighbour is a cell of its own level
# or, across the edge of its level's blocks, a leaf cell of the next coarser
# level (2:1 nesting; the step checks it).  Views: each level's cells under
# finer blocks take the mean of their four children (from the finest level
# down); a level's view outside its blocks is the next coarser level's view
# copied to the four cells under each of its cells.


def level_lattice(grid, l):
    return (grid.ny << l, grid.nx << l)


def level_present(grid, levels, l):
    """Cells of the level-l lattice inside level-l blocks (l = 0: all)."""
    shape = level_lattice(grid, l)
    if l == 0:
        return np.ones(shape, dtype=bool)
    m = np.zeros(shape, dtype=bool)
    s = 2 * grid.b
    for bx, by in levels[l - 1]:
        m[by * s:(by + 1) * s, bx * s:(bx + 1) * s] = True
    return m


def level_problem(grid, l):
    return F.Problem(ndim=2, n=(grid.nx << l, grid.ny << l, 1),
                     dx=(grid.dx / (1 << l), grid.dy / (1 << l), 1.0),
                     bc=tuple(grid.bc), c=grid.c, limiter=grid.limiter,
                     face_mean=grid.face_mean)


def blocks_to_full(grid, blocks, arr, fill):
    out = np.array(fill, dtype=np.float64, copy=True)
    s = 2 * grid.b
    for k, (bx, by) in enumerate(blocks):
        out[by * s:(by + 1) * s, bx * s:(bx + 1) * s] = arr[k]
    return out


def full_to_blocks(grid, blocks, full):
    s = 2 * grid.b
    if not blocks:
        return np.zeros((0, s, s))
    return np.stack([full[by * s:(by + 1) * s, bx * s:(bx + 1) * s]
                     for bx, by in blocks])


def hier_views(grid, levels, fields):
    """Full-lattice views of one field on every level; `fields` = [base
    (ny, nx), level-1 blocks, level-2 blocks, ...]."""
    L = len(levels)
    present = [level_present(grid, levels, l) for l in range(L + 1)]
    vals = [fields[0]] + [blocks_to_full(grid, levels[l - 1], fields[l],
                                         np.zeros(level_lattice(grid, l)))
                          for l in range(1, L + 1)]
    avg = [None] * (L + 1)
    avg[L] = vals[L]
    for l in range(L - 1, -1, -1):  # under finer blocks: child means
        avg[l] = np.where(present[l + 1][0::2, 0::2], child_mean(avg[l + 1]),
                          vals[l])
    view = [avg[0]]
    for l in range(1, L + 1):  # outside a level's blocks: the coarser view
        view.append(np.where(present[l], avg[l], inject(view[l - 1])))
    return view, present


def hier_numbering(grid, levels):
    """Leaf index per lattice cell of every level (-1: not a leaf)."""
    L = len(levels)
    present = [level_present(grid, levels, l) for l in range(L + 1)]
    idx, k = [], 0
    for l in range(L + 1):
        covered = present[l + 1][0::2, 0::2] if l < L else \
            np.zeros_like(present[l])
        leaf = present[l] & ~covered
        a = np.full(present[l].shape, -1, dtype=np.int64)
        if l == 0:
            n = int(np.count_nonzero(leaf))
            a[leaf] = np.arange(k, k + n)
            k += n
        else:
            s = 2 * grid.b
            for bx, by in levels[l - 1]:
                blk = leaf[by * s:(by + 1) * s, bx * s:(bx + 1) * s]
                sub = a[by * s:(by + 1) * s, bx * s:(bx + 1) * s]
                n = int(np.count_nonzero(blk))
                sub[blk] = np.arange(k, k + n)
                k += n
        idx.append(a)
    return idx, k


def hier_assemble(grid, levels, D, dt):
    """Composite operator over the leaf cells of every level, and their
    volumes; D: full-lattice D per level."""
    idx, N = hier_numbering(grid, levels)
    L = len(levels)
    per = [b == F.PERIODIC for b in grid.bc]
    rows, cols, vals = [], [], []

    def couple(i, j, wi, wj):
        rows.extend([i, i, j, j])
        cols.extend([i, j, j, i])
        vals.extend([wi, -wi, wj, -wj])

    for l in range(L + 1):
        NY, NX = idx[l].shape
        h = (grid.dx / (1 << l), grid.dy / (1 << l))
        present = level_present(grid, levels, l)
        for J in range(NY):
            for I in range(NX):
                me = idx[l][J, I]
                if me < 0:
                    continue
                for d, (di, dj) in enumerate(((1, 0), (0, 1))):
                    for sgn in (1, -1):
                        II, JJ = I + sgn * di, J + sgn * dj
                        if not (0 <= (II, JJ)[d] < (NX, NY)[d]):
                            if not per[d]:
                                continue
                            II, JJ = II % NX, JJ % NY
                        if present[JJ, II]:
                            nb = idx[l][JJ, II]
                            if nb < 0 or sgn < 0:
                                continue  # finer side, or counted below
                            a = dt * _mean(D[l][J, I], D[l][JJ, II],
                                           grid.face_mean) / h[d] ** 2
                            couple(me, nb, a, a)
                        else:
                            c = idx[l - 1][JJ // 2, II // 2]
                            if c < 0:
                                raise ValueError("levels not 2:1 nested")
                            beta = (2.0 / 3.0) * dt * _mean(
                                D[l][J, I], D[l - 1][JJ // 2, II // 2],
                                grid.face_mean) / h[d] ** 2
                            couple(me, c, beta, beta / 4.0)
    rows.extend(range(N))
    cols.extend(range(N))
    vals.extend([1.0] * N)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsr()
    vol = np.empty(N)
    for l in range(L + 1):
        m = idx[l] >= 0
        vol[idx[l][m]] = grid.dx * grid.dy / (4 ** l)
    return A, vol


def hier_to_leaf(grid, levels, fields):
    idx, N = hier_numbering(grid, levels)
    v = np.empty(N)
    for l, f in enumerate(fields):
        full = f if l == 0 else blocks_to_full(
            grid, levels[l - 1], f, np.zeros(level_lattice(grid, l)))
        m = idx[l] >= 0
        v[idx[l][m]] = full[m]
    return v


def hier_from_leaf(grid, levels, v):
    """Per-level arrays from a leaf vector; cells under finer blocks get the
    mean of their children (from the finest level down)."""
    idx, _ = hier_numbering(grid, levels)
    L = len(levels)
    full = []
    for l in range(L + 1):
        a = np.zeros(idx[l].shape)
        m = idx[l] >= 0
        a[m] = v[idx[l][m]]
        full.append(a)
    for l in range(L - 1, -1, -1):
        cov = level_present(grid, levels, l + 1)[0::2, 0::2]
        full[l] = np.where(cov, child_mean(full[l + 1]), full[l])
    return [full[0]] + [full_to_blocks(grid, levels[l - 1], full[l])
                        for l in range(1, L + 1)]


def hier_coefficients(grid, levels, E, rho, kappa):
    views = [hier_views(grid, levels, f)[0] for f in (E, rho, kappa)]
    return [F.diffusion_coefficient(views[0][l], views[1][l], views[2][l],
                                    level_problem(grid, l))[0]
            for l in range(len(levels) + 1)]


def hier_step(grid, levels, E, rho, kappa, dt, method="splu"):
    """E* on every leaf cell of a hierarchy; fields and result as lists
    [base, level-1 blocks, ...]."""
    D = hier_coefficients(grid, levels, E, rho, kappa)
    A, _ = hier_assemble(grid, levels, D, dt)
    b = hier_to_leaf(grid, levels, E)
    x = np.linalg.solve(A.toarray(), b) if method == "dense" else \
        spla.splu(A.tocsc()).solve(b)
    return hier_from_leaf(grid, levels, x)
