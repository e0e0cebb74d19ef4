// One red-black Gauss-Seidel sweep of a mid-sized 3D multigrid level in one
// launch, by tiles (gfx950).
//
// The smoother of the backward-Euler diffusion multigrid (Sect. 3).  On
// levels too small for the z-marching sweep (fld_sweep3d.hip: one block
// marches a chunk of planes, a latency-bound chain of plane steps) but too
// large for one workgroup, a sweep used to take two colour-pass launches.
// Here a block owns a 32 x 8 x 4 tile and does the whole sweep at once:
//   1. it stages the iterate of the tile and a two-cell ring in LDS and
//      loads the operands of the red cells of the tile and its one-cell
//      ring and of the tile's black cells, all before the first use;
//   2. it updates every red cell of tile + ring in LDS from the old black
//      values (the ring's red cells belong to neighbouring tiles and are
//      computed again here from the same operands and old values);
//   3. it updates the tile's black cells from the new red values and
//      writes both colours of the tile to the output array.
// Out of place (x -> xo), so no block sees a neighbour's new values, and
// every cell gets exactly the update of a red pass followed by a black
// pass, with the operations of the colour-pass kernel: the same bits.
//
// A block's 512 threads each own an x pair of the tile (the black update)
// and up to two x pairs of the tile + ring box (the red update: each x
// pair of that box holds one red cell).  Tiles are numbered x fastest, then
// y, then z, and handed to the 8 XCDs in contiguous runs, so the halo
// lines that neighbouring tiles share meet in one XCD's L2.
#include <hip/hip_ext.h>

#include "fld_internal.h"
#include "fld_device.h"
#include "fld_relax3d.h"

namespace fld {

namespace {

constexpr int kTlX = 32, kTlY = 8, kTlZ = 4;      // tile
constexpr int kTlT = kTlX / 2 * kTlY * kTlZ;      // threads: one x pair each
// staged box: tile + two-cell ring
constexpr int kTlSX = kTlX + 4, kTlSY = kTlY + 4, kTlSZ = kTlZ + 4;
constexpr int kTlStaged = kTlSX * kTlSY * kTlSZ;
constexpr int kTlLoads = (kTlStaged + kTlT - 1) / kTlT;
// red box: tile + one-cell ring, as x pairs (one red cell each)
constexpr int kTlPX = (kTlX + 2) / 2, kTlPY = kTlY + 2, kTlPZ = kTlZ + 2;
constexpr int kTlPairs = kTlPX * kTlPY * kTlPZ;
static_assert(kTlPairs <= 2 * kTlT, "two red cells per thread at most");

__device__ __forceinline__ int tl_at(int rx, int ry, int rz) {
  return (rz * kTlSY + ry) * kTlSX + rx;
}

template <typename T>
__global__ void __launch_bounds__(kTlT)
    k_gs_tile_3d(LevelView<T> L, T* __restrict__ xo, int group,
                 const Control* __restrict__ ctrl) {
  __shared__ T S[kTlStaged];
  if (ctrl->done != kRunning) return;
  const Geom& g = L.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int t = threadIdx.x;
  const int gx = nx / kTlX, gy = ny / kTlY;
  const int nb = gridDim.x, b = blockIdx.x;
  const int tile = group ? (b % 8) * (nb / 8) + b / 8 : b;
  const int x0 = (tile % gx) * kTlX, y0 = ((tile / gx) % gy) * kTlY;
  const int z0 = (tile / (gx * gy)) * kTlZ;

  // ---- loads: staged iterate, red operands, black operands ----
  T xv[kTlLoads];
#pragma unroll
  for (int j = 0; j < kTlLoads; ++j) {
    const int i = min(t + j * kTlT, kTlStaged - 1);  // past the end: unused
    const int rx = i % kTlSX, ry = (i / kTlSX) % kTlSY, rz = i / (kTlSX * kTlSY);
    const int X = sw_map(x0 - 2 + rx, nx, g.per[0]);
    const int Y = sw_map(y0 - 2 + ry, ny, g.per[1]);
    const int Z = sw_map(z0 - 2 + rz, nz, g.per[2]);
    xv[j] = L.x[((int64_t)Z * ny + Y) * nx + X];
  }
  SwCoef<T> rc[2];
  bool rok[2];
  int rat[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int j = min(t + e * kTlT, kTlPairs - 1);
    const int bx = j % kTlPX, by = (j / kTlPX) % kTlPY, bz = j / (kTlPX * kTlPY);
    const int y = y0 - 1 + by, z = z0 - 1 + bz;
    const int x = x0 - 1 + 2 * bx + ((x0 - 1 + y + z) & 1);  // the red one
    rok[e] = t + e * kTlT < kTlPairs && sw_inside(x, nx, g.per[0]) &&
             sw_inside(y, ny, g.per[1]) && sw_inside(z, nz, g.per[2]);
    rat[e] = tl_at(x - x0 + 2, by + 1, bz + 1);
    rc[e] = sw_coef(L, sw_map(x, nx, g.per[0]), sw_map(y, ny, g.per[1]),
                    sw_map(z, nz, g.per[2]));
  }
  const int pk = t % (kTlX / 2), pr = (t / (kTlX / 2)) % kTlY,
            ps = t / (kTlX / 2 * kTlY);
  const int px = x0 + 2 * pk, py = y0 + pr, pz = z0 + ps;
  const int eb = ((px + py + pz) & 1) ? 0 : 1;  // the pair's black cell
  const SwCoef<T> bc = sw_coef(L, px + eb, py, pz);
#pragma unroll
  for (int j = 0; j < kTlLoads; ++j) {
    const int i = t + j * kTlT;
    if (i < kTlStaged) S[i] = xv[j];
  }
  __syncthreads();

  // ---- red cells of tile + ring, in place (they read black cells only) --
#pragma unroll
  for (int e = 0; e < 2; ++e)
    if (rok[e]) {
      const int a = rat[e];
      const T xl[3] = {S[a - 1], S[a - kTlSX], S[a - kTlSX * kTlSY]};
      const T xu[3] = {S[a + 1], S[a + kTlSX], S[a + kTlSX * kTlSY]};
      S[a] = sw_relax(rc[e], xl, xu);
    }
  __syncthreads();

  // ---- black cells of the tile; both colours out ----
  const int a = tl_at(2 * pk + 2 + eb, pr + 2, ps + 2);
  const T xl[3] = {S[a - 1], S[a - kTlSX], S[a - kTlSX * kTlSY]};
  const T xu[3] = {S[a + 1], S[a + kTlSX], S[a + kTlSX * kTlSY]};
  const T vb = sw_relax(bc, xl, xu);
  const T vr = S[eb ? a - 1 : a + 1];
  T* dst = xo + ((int64_t)pz * ny + py) * nx + px;
  dst[0] = eb ? vr : vb;
  dst[1] = eb ? vb : vr;
}

}  // namespace

bool gs_tile3d_ok(const Geom& g) {
  return g.ndim == 3 && g.n[0] % kTlX == 0 && g.n[1] % kTlY == 0 &&
         g.n[2] % kTlZ == 0 && gs_colors(g) == 2 &&
         (int64_t)g.n[0] * g.n[1] * g.n[2] == g.N;
}

template <typename T>
hipError_t launch_gs_tile3d(const LevelView<T>& L, T* xo, const Control* ctrl,
                            hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (!gs_tile3d_ok(L.g)) return hipErrorInvalidValue;
  const int nb = (L.g.n[0] / kTlX) * (L.g.n[1] / kTlY) * (L.g.n[2] / kTlZ);
  const int group = nb % 8 == 0;
  if (ev0 && ev1)
    hipExtLaunchKernelGGL(k_gs_tile_3d<T>, dim3(nb), dim3(kTlT), 0, s, ev0,
                          ev1, 0, L, xo, group, ctrl);
  else
    hipLaunchKernelGGL(k_gs_tile_3d<T>, dim3(nb), dim3(kTlT), 0, s, L, xo,
                       group, ctrl);
  return hipGetLastError();
}

template hipError_t launch_gs_tile3d<double>(const LevelView<double>&, double*,
                                             const Control*, hipStream_t,
                                             hipEvent_t, hipEvent_t);
template hipError_t launch_gs_tile3d<float>(const LevelView<float>&, float*,
                                            const Control*, hipStream_t,
                                            hipEvent_t, hipEvent_t);

}  // namespace fld
