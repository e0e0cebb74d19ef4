// Arguments and launchers of the LDS-tiled 2D multigrid kernels
// (fld_tile2d.hip).
#pragma once

#include "fld_internal.h"

namespace fld {

template <typename T>
struct Tile2DArgs {
  Geom g;             // this level
  const T* x;         // iterate read (unless zero_init), halo included
  T* xo;              // iterate written (tile interiors); never x: blocks
                      // read their halo from x while neighbours write
  const T* b;         // right-hand side
  const T* ax;        // face coefficients along x and y
  const T* ay;
  Geom gc;            // coarse level (restriction target / correction source)
  T* cb;              // down: coarse right-hand side (mean of 2x2 residuals)
  const T* ce;        // up: coarse correction to interpolate and add
  double* partials;   // down on the finest level: per-tile sum of r^2
  int zero_init;      // x starts at zero and is not read
  int tiles_x, tiles_y;  // set by the launcher
  int vec;            // x, xo, b, ax, ay 16-byte aligned and n[0] even
                      // (tile2d_vec_ok; set by the launcher)
  int spec;           // load the operands before testing the stop flag
  // down on level 1, FP64: the finest down pass's partial sums of r^2, to be
  // reduced here for its stop test (instead of a separate finalize launch);
  // fin_cycle is the index of the V-cycle within the solve, fin_ctrl the
  // control block block 0 updates
  const double* fin_partials;
  int fin_count;
  int fin_cycle;
  Control* fin_ctrl;
  const Control* ctrl;
};

// Tile shapes available to the launchers (see fld_tile2d.hip); the batched
// launcher takes the same shapes.
constexpr int kTileVariants = 7;
constexpr int kTileVariantsBatch = 7;
const char* tile2d_variant_name(int variant);

// Launch the down (pre-smoothing + residual + restriction) or up
// (prolongation + post-smoothing) kernel with nu red-black sweeps
// (nu in 1..3) and tile shape `variant`.  *nblocks receives the number of
// tiles (one partial sum each on the finest down pass).  Given ev0 and ev1,
// the launch records them around the kernel's own execution.
template <typename T>
hipError_t launch_tile2d(const Tile2DArgs<T>& a, int nu, bool down,
                         int variant, hipStream_t s, int* nblocks,
                         hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// 1 when the 16-byte load path may be used for these arguments.
template <typename T>
int tile2d_vec_ok(const Tile2DArgs<T>& a);

// Number of tiles (blocks) the launcher will use.
int tile2d_blocks(const Geom& g, int nu, bool down, int variant);
// Same, also returning the tile grid (for the batched form's argument table).
int tile2d_grid(const Geom& g, int nu, bool down, int variant, int* tiles_x,
                int* tiles_y);

// Batched form: tab[g] (device memory, tiles_x/tiles_y filled in) are the
// arguments of grid g, whose tiles are blocks start[g] .. start[g+1]-1 of a
// launch of nblocks blocks.  With ev0/ev1 the launch records them itself.
template <typename T>
hipError_t launch_tile2d_batch(const Tile2DArgs<T>* tab, const int* start,
                               int ng, int nblocks, int nu, bool down,
                               int variant, hipStream_t s,
                               hipEvent_t ev0 = nullptr,
                               hipEvent_t ev1 = nullptr);

}  // namespace fld
