// Arguments and launchers of the LDS-tiled 2D multigrid kernels
// (fld_tile2d.hip).
#pragma once

#include "fld_internal.h"

namespace fld {

template <typename T>
struct Tile2DArgs {
  Geom g;             // this level
  T* x;               // iterate, read (unless zero_init) and written
  const T* b;         // right-hand side
  const T* ax;        // face coefficients along x and y
  const T* ay;
  Geom gc;            // coarse level (restriction target / correction source)
  T* cb;              // down: coarse right-hand side (mean of 2x2 residuals)
  const T* ce;        // up: coarse correction to interpolate and add
  double* partials;   // down on the finest level: per-tile sum of r^2
  int zero_init;      // x starts at zero and is not read
  int tiles_x, tiles_y;  // set by the launcher
  const Control* ctrl;
};

// Launch the down (pre-smoothing + residual + restriction) or up
// (prolongation + post-smoothing) kernel with nu red-black sweeps
// (nu in 1..3).  *nblocks receives the number of tiles.
template <typename T>
hipError_t launch_tile2d(const Tile2DArgs<T>& a, int nu, bool down,
                         hipStream_t s, int* nblocks);

// Number of tiles (blocks) the launcher will use.
int tile2d_blocks(const Geom& g, int nu, bool down);

}  // namespace fld
