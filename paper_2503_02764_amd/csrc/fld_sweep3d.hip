// Fused red-black Gauss-Seidel sweep of a 3D multigrid level (gfx950).
//
// The smoother of the backward-Euler diffusion multigrid (Sect. 3): a sweep
// updates every red cell ((x + y + z) even) from the old black values, then
// every black cell from the new red ones, each by
// x = (b + sum alpha x_nb) / (1 + sum alpha).  The colour-pass kernels do
// this in two launches, each streaming the iterate and all four operand
// arrays; here one launch does the whole sweep, out of place (x -> xo), so
// each array is read about once per sweep instead of twice.
//
// A block owns a kSwX x kSwY tile of (x, y) and a chunk of z planes and
// marches up through them, with the iterate of six planes staged in LDS
// over the tile and a two-cell ring.  At plane p it updates the red cells of
// plane p over the tile and a one-cell ring and the black cells of plane
// p - 2 over the tile, and writes both colours of plane p - 2 to xo.  The
// red values of the ring, and of the planes just outside the chunk, are the
// neighbouring blocks' cells, computed again here from the same old values:
// every cell gets exactly the update of a red pass followed by a black pass,
// with the operations of the colour-pass kernel, and no block depends on
// another's progress (the old values stay in x until the launch ends).
//
// The black update lags the red one by two planes, so both run between the
// same pair of barriers, and every operand is loaded a full step before its
// use (the staged plane two steps before).
#include <hip/hip_ext.h>

#include <algorithm>

#include "fld_internal.h"
#include "fld_device.h"
#include "fld_relax3d.h"

namespace fld {

namespace {

constexpr int kSwX = 64, kSwY = 16;            // output tile of a block
constexpr int kSwT = kSwX * kSwY / 2;          // threads: one x pair each
constexpr int kSwRX = kSwX + 4, kSwRY = kSwY + 4;  // staged: tile + 2-cell ring
constexpr int kSwPlane = kSwRX * kSwRY;
constexpr int kSwSlots = 6;                    // planes p - 3 .. p + 2
constexpr int kSwRing = 2 * (kSwX / 2 + 1) + kSwY;  // red cells of the 1-cell ring
constexpr int kSwLoads = (kSwPlane + kSwT - 1) / kSwT;
constexpr int kSwBlocks = 256;                 // z chunking aims at one per CU
static_assert(kSwRing <= kSwT, "one extra ring cell per thread at most");

// The red cell a thread updates on plane p: e == 0 its pair's, e == 1 its
// cell of the one-cell ring (threads below kSwRing).  Tile-relative
// coordinates (rx, ry) of the staged plane; false if it has none.
__device__ __forceinline__ bool sw_red_cell(int e, int t, int x0, int y0,
                                            int p, int& rx, int& ry) {
  if (e == 0) {
    const int k = t % (kSwX / 2), r = t / (kSwX / 2);
    const int x = x0 + 2 * k, y = y0 + r;
    rx = 2 * k + 2 + ((x + y + p) & 1);
    ry = r + 2;
    return true;
  }
  if (t >= kSwRing) return false;
  if (t < 2 * (kSwX / 2 + 1)) {  // the rows below and above the tile
    const int half = t / (kSwX / 2 + 1), k = t % (kSwX / 2 + 1);
    const int y = half ? y0 + kSwY : y0 - 1;
    rx = 1 + 2 * k + (((x0 - 1) + y + p) & 1);
    ry = y - y0 + 2;
    return true;
  }
  const int y = y0 + (t - 2 * (kSwX / 2 + 1));  // the columns left and right
  rx = (((x0 - 1) + y + p) & 1) ? kSwX + 2 : 1;
  ry = y - y0 + 2;
  return true;
}

template <typename T>
__global__ void __launch_bounds__(kSwT)
    k_gs_sweep_3d(LevelView<T> L, T* __restrict__ xo, int zc, int group,
                  const Control* __restrict__ ctrl) {
  __shared__ T S[kSwSlots][kSwPlane];
  if (ctrl->done != kRunning) return;
  const Geom& g = L.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int64_t sz = (int64_t)nx * ny;
  const int t = threadIdx.x;
  // Blocks go to the 8 XCDs in turn; with `group`, block b takes tile
  // (b % 8) * (blocks / 8) + b / 8 of the x-fastest tile order, so each XCD
  // holds a contiguous run of tiles whose shared halo lines meet in its L2.
  const int gx = nx / kSwX, gy = ny / kSwY;
  const int nb = gridDim.x, b = blockIdx.x;
  const int tile = group ? (b % 8) * (nb / 8) + b / 8 : b;
  const int x0 = (tile % gx) * kSwX, y0 = ((tile / gx) % gy) * kSwY;
  const int z0 = (tile / (gx * gy)) * zc, z1 = min(z0 + zc, nz);
  const int base = z0 - 2;  // plane staged in slot 0 first
  auto slot = [&](int p) { return (p - base) % kSwSlots; };
  auto at = [](int rx, int ry) { return ry * kSwRX + rx; };

  // staged-plane loads: element i of the ring-2 region of plane p
  auto load_plane = [&](int p, T (&xv)[kSwLoads]) {
    const int64_t zo = (int64_t)sw_map(p, nz, g.per[2]) * sz;
#pragma unroll
    for (int j = 0; j < kSwLoads; ++j) {
      const int i = min(t + j * kSwT, kSwPlane - 1);  // past the end: unused
      const int X = sw_map(x0 - 2 + i % kSwRX, nx, g.per[0]);
      const int Y = sw_map(y0 - 2 + i / kSwRX, ny, g.per[1]);
      xv[j] = L.x[zo + (int64_t)Y * nx + X];
    }
  };
  auto store_plane = [&](int p, const T (&xv)[kSwLoads]) {
    T* s = S[slot(p)];
#pragma unroll
    for (int j = 0; j < kSwLoads; ++j) {
      const int i = t + j * kSwT;
      if (i < kSwPlane) s[i] = xv[j];
    }
  };

  // red operands of plane p: the pair's red cell and the ring cell
  struct Red {
    SwCoef<T> c[2];
    bool ok[2];
    int rx[2], ry[2];
  };
  // (loads issued for every thread and step, from addresses inside the
  // level; ok says whether the cell is updated)
  auto load_red = [&](int p, Red& R) {
    const bool pin = p <= z1 && sw_inside(p, nz, g.per[2]);
    const int Z = sw_map(min(p, z1 + 1), nz, g.per[2]);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      R.ok[e] = sw_red_cell(e, t, x0, y0, p, R.rx[e], R.ry[e]);
      if (!R.ok[e]) R.rx[e] = R.ry[e] = 2;  // a cell of the tile
      const int x = x0 - 2 + R.rx[e], y = y0 - 2 + R.ry[e];
      R.ok[e] = R.ok[e] && pin && sw_inside(x, nx, g.per[0]) &&
                sw_inside(y, ny, g.per[1]);
      R.c[e] = sw_coef(L, sw_map(x, nx, g.per[0]), sw_map(y, ny, g.per[1]), Z);
    }
  };

  // the thread's pair: cells x0 + 2k, x0 + 2k + 1 of row y0 + r; its black
  // cell on plane q sits at staged column brx(q)
  const int pk = t % (kSwX / 2), pr = t / (kSwX / 2);
  const int px = x0 + 2 * pk, py = y0 + pr;
  auto brx_of = [&](int q) { return 2 * pk + 2 + ((px + py + q + 1) & 1); };
  auto load_black = [&](int q, SwCoef<T>& c) {
    q = min(max(q, z0), z1 - 1);
    c = sw_coef(L, px + brx_of(q) - 2 - 2 * pk, py, q);
  };

  // Black lags red by two planes: at step p the red cells of plane p read
  // the black cells of planes p - 1 .. p + 1, not yet updated, and the black
  // cells of plane p - 2 read red cells of planes p - 3 .. p - 1, updated at
  // earlier steps; neither reads what the other writes, so one barrier per
  // step suffices.  Six slots: planes p - 3 .. p + 1 in use, p + 2 staged.
  Red rA, rB;
  SwCoef<T> bA, bB;
  T xA[kSwLoads], xB[kSwLoads];
  load_plane(base, xA);
  store_plane(base, xA);
  load_plane(base + 1, xA);
  store_plane(base + 1, xA);
  load_plane(base + 2, xA);
  store_plane(base + 2, xA);
  load_plane(base + 3, xA);
  load_red(z0 - 1, rA);
  __syncthreads();

  // One step; the operands of the next step go to the other register set
  // (the steps alternate between the two, so nothing is copied and the
  // loads stay in flight across the barrier).
  //
  // The black cells' operands of plane p are loaded at step p, into the set
  // the black update of plane p - 2 has just used (the sets alternate with
  // the steps), one step after the red cells' of the same plane: the two
  // colours share cache lines, which are then still in L2.
  auto step = [&](int p, const Red& rc, Red& rn, SwCoef<T>& bc,
                  const T (&xv)[kSwLoads], T (&xn)[kSwLoads]) {
    const int q = p - 2;  // plane of this step's black update
    load_plane(min(p + 3, z1 + 1), xn);
    load_red(p + 1, rn);
    // red cells of plane p
    if (p <= z1) {
      T* sp = S[slot(p)];
      const T* sm = S[slot(p - 1)];
      const T* sq = S[slot(p + 1)];
#pragma unroll
      for (int e = 0; e < 2; ++e)
        if (rc.ok[e]) {
          const int rx = rc.rx[e], ry = rc.ry[e];
          const T xl[3] = {sp[at(rx - 1, ry)], sp[at(rx, ry - 1)], sm[at(rx, ry)]};
          const T xu[3] = {sp[at(rx + 1, ry)], sp[at(rx, ry + 1)], sq[at(rx, ry)]};
          sp[at(rx, ry)] = sw_relax(rc.c[e], xl, xu);
        }
    }
    // black cells of plane q, and plane q of both colours out
    if (q >= z0 && q < z1) {
      T* sb = S[slot(q)];
      const T* sm = S[slot(q - 1)];
      const T* sq = S[slot(q + 1)];
      const int bx = brx_of(q), ry = pr + 2;
      const T xl[3] = {sb[at(bx - 1, ry)], sb[at(bx, ry - 1)], sm[at(bx, ry)]};
      const T xu[3] = {sb[at(bx + 1, ry)], sb[at(bx, ry + 1)], sq[at(bx, ry)]};
      const T vb = sw_relax(bc, xl, xu);
      sb[at(bx, ry)] = vb;
      const T vr = sb[at(bx ^ 1, ry)];  // the pair's red cell
      const bool red_first = ((px + py + q) & 1) == 0;
      T* dst = xo + (int64_t)q * sz + (int64_t)py * nx + px;
      dst[0] = red_first ? vr : vb;
      dst[1] = red_first ? vb : vr;
    }
    load_black(p, bc);
    if (p + 2 <= z1 + 1) store_plane(p + 2, xv);
    sw_barrier();
  };
  // steps z0 - 1 .. z1 + 1, two per trip (a last step past z1 + 1 does
  // nothing but load, inside the level)
  for (int p = z0 - 1; p <= z1 + 1; p += 2) {
    step(p, rA, rB, bA, xA, xB);
    step(p + 1, rB, rA, bB, xB, xA);
  }
}

// z planes per block: the blocks of one launch fill the chip once, one per
// CU (on 256^3, 64 planes: FP64 206 us per sweep against 226 with 32, FP32
// 134 against 140; a second wave of blocks costs more than the two extra
// planes a block redoes at each end of its chunk).
template <typename T>
int sw_zchunk(const Geom& g) {
  const int tiles = (g.n[0] / kSwX) * (g.n[1] / kSwY);
  const int chunks = std::max(1, std::min(g.n[2], kSwBlocks / std::max(tiles, 1)));
  return std::max(8, (g.n[2] + chunks - 1) / chunks);
}

}  // namespace

bool gs_sweep3d_ok(const Geom& g) {
  return g.ndim == 3 && g.n[0] % kSwX == 0 && g.n[1] % kSwY == 0 &&
         gs_colors(g) == 2 && (int64_t)g.n[0] * g.n[1] * g.n[2] == g.N;
}

template <typename T>
hipError_t launch_gs_sweep3d(const LevelView<T>& L, T* xo, int zc,
                             const Control* ctrl, hipStream_t s,
                             hipEvent_t ev0, hipEvent_t ev1) {
  if (!gs_sweep3d_ok(L.g)) return hipErrorInvalidValue;
  if (zc <= 0) zc = sw_zchunk<T>(L.g);
  const int nb = (L.g.n[0] / kSwX) * (L.g.n[1] / kSwY) *
                 ((L.g.n[2] + zc - 1) / zc);
  // XCD-grouped tile order (FP64 sweep on 256^3: 250 -> 205 us, FP32 155 ->
  // 140 us against the plain order)
  const int group = nb % 8 == 0;
  if (ev0 && ev1)
    hipExtLaunchKernelGGL(k_gs_sweep_3d<T>, dim3(nb), dim3(kSwT), 0, s, ev0,
                          ev1, 0, L, xo, zc, group, ctrl);
  else
    hipLaunchKernelGGL(k_gs_sweep_3d<T>, dim3(nb), dim3(kSwT), 0, s, L, xo, zc,
                       group, ctrl);
  return hipGetLastError();
}

template hipError_t launch_gs_sweep3d<double>(const LevelView<double>&,
                                              double*, int, const Control*,
                                              hipStream_t, hipEvent_t,
                                              hipEvent_t);
template hipError_t launch_gs_sweep3d<float>(const LevelView<float>&, float*,
                                             int, const Control*, hipStream_t,
                                             hipEvent_t, hipEvent_t);

}  // namespace fld
