// Block-adaptive 2D step: geometry, physics and kernel launchers
// (fld_amr.hip), used by the host driver (fld_amr.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fld {

// A base grid of nx x ny cells tiled by b x b blocks (nbx x nby of them),
// nbf of which are refined into S x S = 2b x 2b fine cells.
struct AmrGeom {
  int nx, ny, b, S, nbx, nby, nbf;
  int per[2];        // periodic along x, y (else zero-gradient walls)
  int64_t Nb, Nf;    // base cells, fine cells
  double dx, dy;     // base spacing
  double vb, vf;     // base and fine cell volumes (areas)
  const int* bmap;   // refined block of each base block, or -1 (device)
  const int* bxy;    // (bx, by) of each refined block (device)
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

hipError_t amr_views(const AmrGeom& G, const double* Eb, const double* rb,
                     const double* kb, const double* Ef, const double* rf,
                     const double* kf, double* Ev, double* rv, double* kv,
                     hipStream_t s);
hipError_t amr_coefficients(const AmrGeom& G, const AmrPhys& P, double dt,
                            const double* Ev, const double* rv,
                            const double* kv, const double* Ef,
                            const double* rf, const double* kf, double* Db,
                            double* Df, double* cf, int* bad, hipStream_t s);
// y = A x; with r and partials also the block sums of (r, x) and (x, y)
// (rows 0 and 1 of amr_dot_blocks entries each)
hipError_t amr_apply(const AmrGeom& G, const double* ax, const double* ay,
                     const double* cf, const double* x, double* y,
                     hipStream_t s, const double* r = nullptr,
                     double* partials = nullptr);
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
// with ev0 and ev1 the launch records its start and end on them
hipError_t amr_smooth(const AmrGeom& G, const double* cf, const double* r,
                      double* z, int colour, hipStream_t s,
                      hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t amr_base_rhs(const AmrGeom& G, const double* cf, const double* r,
                        const double* z, double* rhs, hipStream_t s);
hipError_t amr_prolong(const AmrGeom& G, double* z, hipStream_t s);
hipError_t amr_zero_covered(const AmrGeom& G, double* v, hipStream_t s);
hipError_t amr_pack(const AmrGeom& G, const double* vb, const double* vf,
                    double* v, hipStream_t s);
hipError_t amr_unpack(const AmrGeom& G, const double* v, double* vb,
                      double* vf, hipStream_t s);
hipError_t amr_axpy(int64_t n, double a, const double* p, const double* x,
                    double* y, hipStream_t s);
int amr_dot_blocks(const AmrGeom& G);
hipError_t amr_dots(const AmrGeom& G, const AmrDots& D, double* partials,
                    hipStream_t s);

}  // namespace fld
