// Block-adaptive 2D step: geometry, physics and kernel launchers
// (fld_amr.hip), used by the host driver (fld_amr.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fld {

constexpr int kAmrMaxLevels = 4;  // refined levels above the base

// A base grid of nx x ny cells and L refined levels.  Level l >= 1 has
// spacing dx / 2^l on a lattice of (nx << l) x (ny << l) cells; each of its
// blocks refines a b x b patch of level-(l-1) cells (the patch's corner in
// units of b level-(l-1) cells) into S x S = 2b x 2b level-l cells.
// Vectors hold the base cells, then level 1's blocks, level 2's, ...
struct AmrGeom {
  int nx, ny, b, S, nbx, nby, L;
  int per[2];        // periodic along x, y (else zero-gradient walls)
  int64_t Nb, Nf;    // base cells, fine cells of all levels
  double dx, dy;     // base spacing
  double vb;         // base cell volume (area); level l: vb / 4^l
  // per refined level l = 1..L (index l - 1):
  int64_t off[kAmrMaxLevels + 1];  // level l holds fine cells
                                   // off[l - 1] .. off[l] - 1 (off[0] = 0,
                                   // off[L] = Nf)
  int nblk[kAmrMaxLevels];         // blocks of the level
  int units_x[kAmrMaxLevels];      // b-cell units per row of level l - 1
  const int* bmap[kAmrMaxLevels];  // block of each unit of level l - 1, or
                                   // -1 (device)
  const int* bxy[kAmrMaxLevels];   // (bx, by) of each block (device)
};

struct AmrPhys {
  double c;
  int limiter;    // 0 LP, 1 diffusion, 2 Minerbo
  int face_mean;  // 0 arithmetic, 1 harmonic
};

// up to three volume-weighted dot products in one pass
struct AmrDots {
  const double* u[3];
  const double* v[3];
  int n;
};

// Views (cells under finer blocks: the mean of their four children) of E,
// rho, kappa on every level; vf* arrays hold the fine levels.
hipError_t amr_views(const AmrGeom& G, const double* Eb, const double* rb,
                     const double* kb, const double* Ef, const double* rf,
                     const double* kf, double* Ev, double* rv, double* kv,
                     double* Evf, double* rvf, double* kvf, hipStream_t s);
// D on every level from the views, and the four faces of every fine cell.
hipError_t amr_coefficients(const AmrGeom& G, const AmrPhys& P, double dt,
                            const double* Ev, const double* rv,
                            const double* kv, const double* Evf,
                            const double* rvf, const double* kvf, double* Db,
                            double* Df, double* cf, int* bad, hipStream_t s);
// y = A x; with r and partials also the block sums of (r, x) and (x, y)
// (rows 0 and 1 of amr_dot_blocks entries each)
hipError_t amr_apply(const AmrGeom& G, const double* ax, const double* ay,
                     const double* cf, const double* x, double* y,
                     hipStream_t s, const double* r = nullptr,
                     double* partials = nullptr);
// The preconditioner's cycle through the levels.  amr_smooth_level: one
// colour of a red-black sweep over every cell of level l >= 1 for the
// level's own correction problem L_l e = g (the coarser level's e fixed
// outside the level's blocks); with ev0 and ev1 the launch records its
// start and end on them.  amr_resid_level: t = g - L_l e on level l.
// amr_coarse_rhs: g on level l (0: the base) after level l + 1's sweeps
// (cells under level-(l+1) blocks: the mean of their children's t; leaf
// cells next to level-(l+1) cells: plus the flux of those cells' e).
// amr_prolong_level: e of every cell of level l += bilinear from level
// l - 1's e.
hipError_t amr_smooth_level(const AmrGeom& G, int level, const double* cf,
                            const double* g, double* e, int colour,
                            hipStream_t s, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr);
hipError_t amr_resid_level(const AmrGeom& G, int level, const double* cf,
                           const double* g, const double* e, double* t,
                           hipStream_t s);
hipError_t amr_coarse_rhs(const AmrGeom& G, int level, const double* cf,
                          const double* e, const double* t, double* g,
                          hipStream_t s);
// Cells of level l >= 1 under finer blocks: the mean of their children.
hipError_t amr_restrict_level(const AmrGeom& G, int level, double* v,
                              hipStream_t s);
hipError_t amr_prolong_level(const AmrGeom& G, int level, double* e,
                             hipStream_t s);
// entries of cells under finer blocks (base and fine) back to 0
hipError_t amr_zero_covered(const AmrGeom& G, double* v, hipStream_t s);
hipError_t amr_pack(const AmrGeom& G, const double* vb, const double* vf,
                    double* v, hipStream_t s);
// (base, fine) arrays from a leaf vector (cells under finer blocks: the
// mean of their children); v's covered entries are filled on the way
hipError_t amr_unpack(const AmrGeom& G, double* v, double* vb, double* vf,
                      hipStream_t s);
hipError_t amr_axpy(int64_t n, double a, const double* p, const double* x,
                    double* y, hipStream_t s);
int amr_dot_blocks(const AmrGeom& G);
hipError_t amr_dots(const AmrGeom& G, const AmrDots& D, double* partials,
                    hipStream_t s);
// Krylov scalars kept on the device (sc[0..4]: (z, q_old), (p_old, q_old),
// (r, p), (p, q), (r, r)): a one-block sum of `npair` rows of partials into
// sc[slot ...] (copy: sc[1] = sc[3] first); p = z - sc[0] / sc[1] p_old
// (or z); x += a p, r -= a q with a = sc[2] / sc[3] and the block sums of
// (r, r).
hipError_t amr_reduce(const double* partials, int nb, int npair, double* sc,
                      int slot, int copy, hipStream_t s);
hipError_t amr_dir(int64_t n, const double* z, const double* p_old, double* p,
                   const double* sc, int first, hipStream_t s);
hipError_t amr_update(const AmrGeom& G, const double* p, const double* q,
                      double* x, double* r, const double* sc,
                      double* partials, hipStream_t s);

}  // namespace fld
