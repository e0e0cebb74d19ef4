// Red-black Gauss-Seidel update of one 3D cell from staged neighbour
// values (fused sweep kernels: fld_sweep3d.hip, fld_tile3d.hip).
//
// x = (b + sum alpha x_nb) / (1 + sum alpha), faces in the order -x, +x,
// -y, +y, -z, +z: the operations of the colour-pass kernel (relax_value),
// so the fused sweeps give its bits.
#pragma once

#include "fld_internal.h"

namespace fld {
namespace {

// Coordinate v in [-2, n + 1] mapped into the level: wrapped along a
// periodic dimension, clamped otherwise (a clamped neighbour is the cell
// itself, which is what the colour pass reads at a wall, where its face
// coefficient is 0).
__device__ __forceinline__ int sw_map(int v, int n, int per) {
  if (v < 0) return per ? v + n : 0;
  if (v >= n) return per ? v - n : n - 1;
  return v;
}

__device__ __forceinline__ bool sw_inside(int v, int n, int per) {
  return per || (v >= 0 && v < n);
}

// rhs and the six face coefficients of cell (X, Y, Z) (in the level), with
// the wall and periodic rules of lower_nb / upper_nb.
template <typename T>
struct SwCoef {
  T b, al[3], au[3];
  int wall;  // bit d: the lower face along d is a wall (coefficient 0)
};

template <typename T>
__device__ __forceinline__ SwCoef<T> sw_coef(const LevelView<T>& L, int X,
                                             int Y, int Z) {
  // branch-free: every load is issued, from an address inside the level; a
  // wall's lower face is zeroed where the update uses it
  const Geom& g = L.g;
  const int64_t st[3] = {1, g.n[0], (int64_t)g.n[0] * g.n[1]};
  const int c[3] = {X, Y, Z};
  const int64_t idx = Z * st[2] + Y * st[1] + X;
  SwCoef<T> r;
  r.b = L.b[idx];
  r.wall = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    r.au[d] = L.a[d][idx];
    const int64_t lo = c[d] > 0 ? idx - st[d] : idx + (int64_t)(g.n[d] - 1) * st[d];
    r.al[d] = L.a[d][lo];
    if (c[d] == 0 && !g.per[d]) r.wall |= 1 << d;
  }
  return r;
}

// Block barrier that waits for this wave's LDS operations only: the global
// loads of the next step's operands stay in flight across it (a
// __syncthreads fence would wait for them too).  The memory clobber keeps
// the compiler from moving LDS accesses across.
__device__ __forceinline__ void sw_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// The update of relax_value, faces in the order -x, +x, -y, +y, -z, +z.
// The face pair is one explicit FMA over the upper face's product, which is
// how the compiler contracts relax_value's loop: left to itself it may
// contract the other product in one kernel and not in another (one ulp).
template <typename T>
__device__ __forceinline__ T sw_relax(const SwCoef<T>& k, const T xl[3],
                                      const T xu[3]) {
  T num = k.b, den = T(1);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const T al = (k.wall >> d) & 1 ? T(0) : k.al[d];
    num += fma(al, xl[d], k.au[d] * xu[d]);
    den += al + k.au[d];
  }
  return num / den;
}

}  // namespace
}  // namespace fld
