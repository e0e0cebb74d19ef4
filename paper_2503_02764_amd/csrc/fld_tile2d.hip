// Temporally blocked multigrid kernels for 2D levels (gfx950).
//
// One workgroup owns a region of RX x RY cells: an output tile plus a halo
// of H cells on every side.  Each thread keeps its cells' iterate and
// Gauss-Seidel weights in registers:
//   x_new = b/d + (a_l x_l + a_r x_r + a_d x_d + a_u x_u)/d,  d = 1 + sum a,
// and the workgroup runs NU red-black sweeps (2*NU colour passes) on chip.
// Each colour pass invalidates one more ring of the region, so after 2*NU
// passes the cells at depth >= 2*NU are exactly what a global red-black
// Gauss-Seidel sweep would produce; the tile interior is written back.
//
//   down kernel (H = 2*NU + 2): pre-smoothing, then the residual of the
//     tile (needs one more valid ring), its restriction to the coarse level
//     (mean of the 2x2 children, computed in registers) and, on the finest
//     level, the block sum of r^2 for the convergence test.
//   up kernel (H = 2*NU): x += P e_coarse (cell-centred bilinear
//     interpolation, weights 9/16, 3/16, 3/16, 1/16), then post-smoothing.
//
// Thread layout: RX/2 x NPY threads; thread (px, py) owns the cell pair
// (2px, 2px+1) in the K consecutive rows py*K .. py*K+K-1.  With the region
// origin, H and K all even, the cell of colour c in row k of the pair is
// (c + k) & 1 for every thread, so colour passes have no divergence and all
// register arrays are indexed by compile-time constants; the 2x2 children
// of a coarse cell sit in one thread's registers.
//
// Neighbours: along x, a cell's other neighbour than the thread's own cell
// belongs to the adjacent lane (a thread-row lies within one wave) and is
// read with a DPP lane shift; along y, rows inside the thread's K rows are
// registers, and only the first and last row of every thread-row go
// through LDS (two writes, two reads and one barrier per colour pass).
// Lane shifts that cross the region's x edge (or into another thread-row)
// return some other finite cell value or zero; they may only feed the
// weights of ring-0 cells, which are invalid after the first pass anyway.
// Starting values are exact on every ring (the up kernel's edge lanes load
// their outer coarse neighbours), since a wrong starting value at ring 0
// would cost one more ring per pass.  Tiles whose
// region lies inside the domain load with 16-byte accesses and take the
// left and lower face coefficients from the neighbouring cell's right and
// upper ones; tiles at the domain edge map every cell (periodic wrap,
// Neumann walls) as the one-pass kernels do.
//
// The iterate is double-buffered: a block reads its region (halo included)
// from x and writes its tile interior to xo, so no block can see a
// neighbour's already-updated cells, whatever the dispatch order.
//
// Blocks are dispatched round-robin over the 8 XCDs; tiles are renumbered
// so that each XCD sweeps one contiguous band of tiles and the halos that
// neighbouring tiles share stay in that XCD's L2.
#include <hip/hip_ext.h>

#include "fld_internal.h"
#include "fld_device.h"
#include "fld_tile2d.h"

namespace fld {

namespace {

__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int q = nb >> 3, r = nb & 7;
  return xcd * q + (xcd < r ? xcd : r) + idx;
}

// Map a (possibly out-of-range) coordinate onto the domain; -1 when it lies
// beyond a Neumann wall.
__device__ __forceinline__ int map_coord(int g, int n, int per) {
  if (g >= 0 && g < n) return g;
  if (!per) return -1;
  g %= n;
  return g < 0 ? g + n : g;
}

template <typename T>
__device__ __forceinline__ T block_sum_t(T v, T* sh, int nt) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T r = T(0);
  if (threadIdx.x == 0)
    for (int q = 0; q < (nt + 63) / 64; ++q) r += sh[q];
  return r;
}

// DPP lane shifts over the whole wave: lane i receives lane i-1's value
// (wave_shr:1) or lane i+1's (wave_shl:1); the lane without a source gets 0.
constexpr int kDppWaveShr1 = 0x138, kDppWaveShl1 = 0x130;

template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi =
      __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <typename T>
__device__ __forceinline__ T lane_prev(T v) { return lane_shift<kDppWaveShr1>(v); }
template <typename T>
__device__ __forceinline__ T lane_next(T v) { return lane_shift<kDppWaveShl1>(v); }

template <typename T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };

// One red-black update, with the rounding pinned by explicit FMAs (every
// kernel shape evaluates exactly this).
template <typename T>
__device__ __forceinline__ T gs_value(T bp, T wl, T xl, T wr, T xr, T wd,
                                      T xd, T wu, T xu) {
  return fma(wu, xu, fma(wd, xd, fma(wr, xr, fma(wl, xl, bp))));
}

// Bilinear prolongation weights of the four nearest coarse cells.
template <typename T>
__device__ __forceinline__ T bilinear4(T e0, T e1, T e2, T e3) {
  return fma(T(0.0625), e3, fma(T(0.1875), e2, fma(T(0.1875), e1, T(0.5625) * e0)));
}

}  // namespace

template <typename T, int RX, int NPY, int K, int NU, bool DOWN>
__device__ __forceinline__ void tile2d_body(const Tile2DArgs<T>& A,
                                            const int tile) {
  constexpr int PX = RX / 2;  // threads per thread-row
  constexpr int NT = PX * NPY;
  constexpr int RY = NPY * K;
  constexpr int H = DOWN ? 2 * NU + 2 : 2 * NU;
  constexpr int TX = RX - 2 * H, TY = RY - 2 * H;
  static_assert(K % 2 == 0 && RX % 2 == 0 && TX > 0 && TY > 0, "tile shape");
  static_assert(64 % PX == 0, "a thread-row must lie within one wave");
  using T2 = typename Pair<T>::type;
  // First (slot 0) and last (slot 1) row of every thread-row, by column
  // parity; thread-row py sits at index py + 1, between two zero rows.
  __shared__ T xb[2][NPY + 2][2][PX];
  __shared__ double red[NT / 64 + 1];
  __shared__ int stop_now;
  // With A.spec the operands are loaded before the stop flag is tested, so
  // that the flag's memory round trip overlaps theirs (used on the finest
  // down pass, which rarely runs after convergence: the stop test follows
  // it; a launch past the stop then reads its operands for nothing).
  const int done = A.ctrl->done;
  if (!A.spec && done != kRunning) return;
  if constexpr (DOWN) {
    if (A.fin_count > 0) {
      // stop test of the finest down pass, taken by every block of this
      // launch from the same partial sums in the same order (so all reach
      // the same decision); block 0 records it in the control block
      double v = 0.0;
      for (int i = threadIdx.x; i < A.fin_count; i += NT) v += A.fin_partials[i];
      const double s = block_sum_t<double>(v, red, NT);
      if (threadIdx.x == 0) {
        const Control* C = A.ctrl;
        const double r = sqrt(s / C->bnorm2);
        stop_now = r <= C->rtol || A.fin_cycle + 1 >= C->max_cycles;
        if (blockIdx.x == 0) {
          finalize_update(kFinCycle, s, A.fin_ctrl);
          if (A.fin_ctrl->mirror) *A.fin_ctrl->mirror = *A.fin_ctrl;
        }
      }
      __syncthreads();
      if (stop_now) return;
    }
  }

  const int tyi = tile / A.tiles_x, txi = tile - tyi * A.tiles_x;
  const int gx0 = txi * TX - H, gy0 = tyi * TY - H;  // region origin (even)
  const int px = threadIdx.x % PX, py = threadIdx.x / PX;
  const int nx = A.g.n[0], ny = A.g.n[1];
  const int perx = A.g.per[0], pery = A.g.per[1];

  for (int i = threadIdx.x; i < 8 * PX; i += NT) {
    const int slot = i / (4 * PX), row = (i / (2 * PX)) & 1 ? NPY + 1 : 0;
    (&xb[slot][row][0][0])[i % (2 * PX)] = T(0);
  }

  T x[K][2], bp[K][2], wl[K][2], wr[K][2], wd[K][2], wu[K][2];
  T dn[DOWN ? K : 1][2];
  (void)dn;
  {
    T xv[K][2], bv[K][2], al[K][2], ar[K][2], ad[K][2], au[K][2];
    T cr[DOWN ? 1 : K][2];  // prolongated coarse correction (up)
    bool vv[K][2];
    (void)cr;
    const bool fast = A.vec && gx0 >= 2 && gx0 + RX + 2 <= nx && gy0 >= 2 &&
                      gy0 + RY + 2 <= ny;
    if (fast) {
      // region and its coarse neighbours inside the domain: no mapping
      const int gx = gx0 + 2 * px;
      T ce0[DOWN ? 1 : K], ce2[DOWN ? 1 : K];
      (void)ce0;
      (void)ce2;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int gy = gy0 + py * K + k;
        const int64_t gi = (int64_t)gy * nx + gx;
        if (A.zero_init) {
          xv[k][0] = xv[k][1] = T(0);
        } else {
          const T2 v = *reinterpret_cast<const T2*>(A.x + gi);
          xv[k][0] = v.x;
          xv[k][1] = v.y;
        }
        const T2 b2 = *reinterpret_cast<const T2*>(A.b + gi);
        const T2 r2 = *reinterpret_cast<const T2*>(A.ax + gi);
        const T2 u2 = *reinterpret_cast<const T2*>(A.ay + gi);
        bv[k][0] = b2.x;
        bv[k][1] = b2.y;
        ar[k][0] = r2.x;
        ar[k][1] = r2.y;
        au[k][0] = u2.x;
        au[k][1] = u2.y;
        if (k == 0) {
          const T2 d2 = *reinterpret_cast<const T2*>(A.ay + gi - nx);
          ad[0][0] = d2.x;
          ad[0][1] = d2.y;
        }
        if constexpr (!DOWN) {
          const int ncx = A.gc.n[0];
          const int I = gx >> 1, J = gy >> 1;
          const int J2 = (gy & 1) ? J + 1 : J - 1;
          ce0[k] = A.ce[(int64_t)J * ncx + I];
          ce2[k] = A.ce[(int64_t)J2 * ncx + I];
        }
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        al[k][0] = lane_prev(ar[k][1]);
        al[k][1] = ar[k][0];
        if (k > 0) {
          ad[k][0] = au[k - 1][0];
          ad[k][1] = au[k - 1][1];
        }
        vv[k][0] = vv[k][1] = true;
        if constexpr (!DOWN) {
          // the even cell's second coarse column is I - 1 (lane px - 1),
          // the odd cell's I + 1 (lane px + 1).  The first and last lane of
          // a thread-row load theirs: the starting values of ring 0 must be
          // exact, or one more ring would be lost per colour pass.
          T p0 = lane_prev(ce0[k]), p2 = lane_prev(ce2[k]);
          T n0 = lane_next(ce0[k]), n2 = lane_next(ce2[k]);
          if (px == 0 || px == PX - 1) {
            const int ncx = A.gc.n[0];
            const int gy = gy0 + py * K + k;
            const int I = (gx0 + 2 * px) >> 1, J = gy >> 1;
            const int J2 = (gy & 1) ? J + 1 : J - 1;
            const int Ie = px == 0 ? I - 1 : I + 1;
            const T e0 = A.ce[(int64_t)J * ncx + Ie];
            const T e2 = A.ce[(int64_t)J2 * ncx + Ie];
            if (px == 0) {
              p0 = e0;
              p2 = e2;
            } else {
              n0 = e0;
              n2 = e2;
            }
          }
          cr[k][0] = bilinear4(ce0[k], p0, ce2[k], p2);
          cr[k][1] = bilinear4(ce0[k], n0, ce2[k], n2);
        }
      }
    } else {
      const int mx0 = map_coord(gx0 + 2 * px, nx, perx);
      const int mx1 = map_coord(gx0 + 2 * px + 1, nx, perx);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int my = map_coord(gy0 + py * K + k, ny, pery);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int mx = q ? mx1 : mx0;
          const bool v = mx >= 0 && my >= 0;
          const int cx = v ? mx : 0, cy = v ? my : 0;
          const bool vl = v && (cx > 0 || perx);
          const bool vd = v && (cy > 0 || pery);
          const int64_t gi = (int64_t)cy * nx + cx;
          const int64_t gl = cx > 0 ? gi - 1 : gi + nx - 1;
          const int64_t gd = cy > 0 ? gi - nx : gi + (int64_t)(ny - 1) * nx;
          // loads issued unconditionally (indices clamped into the domain),
          // values masked afterwards
          const T lx = A.zero_init ? T(0) : A.x[gi];
          const T lb = A.b[gi], lr = A.ax[gi], lu = A.ay[gi];
          const T ll = A.ax[gl], ld = A.ay[gd];
          vv[k][q] = v;
          xv[k][q] = v ? lx : T(0);
          bv[k][q] = v ? lb : T(0);
          ar[k][q] = v ? lr : T(0);
          au[k][q] = v ? lu : T(0);
          al[k][q] = vl ? ll : T(0);
          ad[k][q] = vd ? ld : T(0);
          if constexpr (!DOWN) {
            const int ncx = A.gc.n[0], ncy = A.gc.n[1];
            const int I = cx >> 1, J = cy >> 1;
            int I2 = (cx & 1) ? I + 1 : I - 1;
            int J2 = (cy & 1) ? J + 1 : J - 1;
            if (I2 < 0) I2 = perx ? ncx - 1 : 0;
            if (I2 >= ncx) I2 = perx ? 0 : ncx - 1;
            if (J2 < 0) J2 = pery ? ncy - 1 : 0;
            if (J2 >= ncy) J2 = pery ? 0 : ncy - 1;
            cr[k][q] = bilinear4(A.ce[(int64_t)J * ncx + I],
                                     A.ce[(int64_t)J * ncx + I2],
                                     A.ce[(int64_t)J2 * ncx + I],
                                     A.ce[(int64_t)J2 * ncx + I2]);
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        T xq = xv[k][q];
        if constexpr (!DOWN) {
          if (vv[k][q]) xq += cr[k][q];
        }
        const T d = T(1) + al[k][q] + ar[k][q] + ad[k][q] + au[k][q];
        const T inv = T(1) / d;
        x[k][q] = xq;
        bp[k][q] = bv[k][q] * inv;
        wl[k][q] = al[k][q] * inv;
        wr[k][q] = ar[k][q] * inv;
        wd[k][q] = ad[k][q] * inv;
        wu[k][q] = au[k][q] * inv;
        if constexpr (DOWN) dn[k][q] = d;
      }
  }
  if (done != kRunning) return;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    xb[0][py + 1][q][px] = x[0][q];
    xb[1][py + 1][q][px] = x[K - 1][q];
  }
  __syncthreads();

#pragma unroll
  for (int pass = 0; pass < 2 * NU; ++pass) {
    const int c = pass & 1;
    // neighbours of the other colour: first and last rows from the
    // thread-rows below and above, the rest from this thread's rows
    const T below = xb[1][py][c][px];
    const T above = xb[0][py + 2][c ^ 1][px];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int q = (c + k) & 1;
      const T xl = q ? x[k][0] : lane_prev(x[k][1]);
      const T xr = q ? lane_next(x[k][0]) : x[k][1];
      const T xd = k > 0 ? x[k - 1][q] : below;
      const T xu = k < K - 1 ? x[k + 1][q] : above;
      x[k][q] = gs_value(bp[k][q], wl[k][q], xl, wr[k][q], xr, wd[k][q], xd,
                         wu[k][q], xu);
    }
    // publish the updated cells of the first and last row (colour c sits
    // in column c of the first row and column c ^ 1 of the last, K even)
    xb[0][py + 1][c][px] = x[0][c];
    xb[1][py + 1][c ^ 1][px] = x[K - 1][c ^ 1];
    __syncthreads();
  }

  const bool vec_out = A.vec != 0;
  // write the tile interior (cells of this tile inside the domain); a cell
  // pair is inside or outside as a whole (H, TX and nx even)
  {
    const int lx = 2 * px;
    const int gx = gx0 + lx;
    const bool colok = lx >= H && lx < H + TX && gx < nx;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int ly = py * K + k;
      const int gy = gy0 + ly;
      if (!colok || ly < H || ly >= H + TY || gy >= ny) continue;
      T* dst = A.xo + (int64_t)gy * nx + gx;
      if (vec_out) {
        T2 v;
        v.x = x[k][0];
        v.y = x[k][1];
        *reinterpret_cast<T2*>(dst) = v;
      } else {
        dst[0] = x[k][0];
        if (gx + 1 < nx) dst[1] = x[k][1];
      }
    }
  }

  if constexpr (DOWN) {
    // both colours of the neighbouring thread-rows' boundary rows
    T bl[2], ab[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      bl[q] = xb[1][py][q][px];
      ab[q] = xb[0][py + 2][q][px];
    }
    T pl[K], nr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      pl[k] = lane_prev(x[k][1]);
      nr[k] = lane_next(x[k][0]);
    }
    double r2 = 0.0;
    const int ncx = A.gc.n[0];
    const int lx = 2 * px;
    const int gx = gx0 + lx;
    const bool colok = lx >= H && lx < H + TX && gx < nx;
#pragma unroll
    for (int k = 0; k < K; k += 2) {
      const int ly = py * K + k;
      const int gy = gy0 + ly;
      if (!colok || ly < H || ly >= H + TY || gy >= ny) continue;
      T r[2][2];
#pragma unroll
      for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int j = k + kk;
          const T xl = q ? x[j][0] : pl[j];
          const T xr = q ? nr[j] : x[j][1];
          const T xd = j > 0 ? x[j - 1][q] : bl[q];
          const T xu = j < K - 1 ? x[j + 1][q] : ab[q];
          r[kk][q] = dn[j][q] * (gs_value(bp[j][q], wl[j][q], xl, wr[j][q], xr,
                                          wd[j][q], xd, wu[j][q], xu) -
                                 x[j][q]);
        }
      const T s = (r[0][0] + r[0][1]) + (r[1][0] + r[1][1]);
      A.cb[(int64_t)(gy >> 1) * ncx + (gx >> 1)] = T(0.25) * s;
      r2 += (double)r[0][0] * r[0][0] + (double)r[0][1] * r[0][1] +
            (double)r[1][0] * r[1][0] + (double)r[1][1] * r[1][1];
    }
    if (A.partials) {
      const double t = block_sum_t<double>(r2, red, NT);
      if (threadIdx.x == 0) A.partials[tile] = t;
    }
  }
}

template <typename T, int RX, int NPY, int K, int NU, bool DOWN>
__global__ void __launch_bounds__(RX / 2 * NPY) k_tile2d(Tile2DArgs<T> A) {
  tile2d_body<T, RX, NPY, K, NU, DOWN>(A, xcd_tile(blockIdx.x, gridDim.x));
}

// Batched form: the tiles of many independent grids in one launch.  Block
// b (after the XCD renumbering) belongs to the grid g with
// start[g] <= b < start[g + 1]; its arguments are tab[g] (device memory).
template <typename T, int RX, int NPY, int K, int NU, bool DOWN>
__global__ void __launch_bounds__(RX / 2 * NPY)
    k_tile2d_batch(const Tile2DArgs<T>* __restrict__ tab,
                   const int* __restrict__ start, int ng) {
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  int lo = 0, hi = ng - 1;
  while (lo < hi) {  // last g with start[g] <= b
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  tile2d_body<T, RX, NPY, K, NU, DOWN>(tab[lo], b - start[lo]);
}

// Tile shapes (region RX x NPY*K cells, RX/2 * NPY threads); the
// autotuner picks one per level and direction.
//   0: 64 x 48, 256 threads (6 rows per thread)
//   1: 64 x 64, 512 threads (4 rows)
//   2: 64 x 64, 1024 threads (2 rows)
//   3: 32 x 32, 256 threads (2 rows)  -- small levels: more, lighter blocks
//   4: 128 x 48, 512 threads (6 rows)
//   5: 32 x 64, 256 threads (4 rows)
//   6: 64 x 32, 512 threads (2 rows)
#define FLD_TILE_SHAPES(X)                                                  \
  X(0, 64, 8, 6) X(1, 64, 16, 4) X(2, 64, 32, 2) X(3, 32, 16, 2) X(4, 128, 8, 6) \
  X(5, 32, 16, 4) X(6, 64, 16, 2)

namespace {
struct Shape {
  int rx, npy, k;
};
constexpr Shape kShapes[kTileVariants] = {
#define FLD_SHAPE_ROW(v, rx, npy, k) {rx, npy, k},
    FLD_TILE_SHAPES(FLD_SHAPE_ROW)
#undef FLD_SHAPE_ROW
};

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }
}  // namespace

const char* tile2d_variant_name(int v) {
  switch (v) {
    case 0: return "64x48/256";
    case 1: return "64x64/512";
    case 2: return "64x64/1024";
    case 3: return "32x32/256";
    case 4: return "128x48/512";
    case 5: return "32x64/256";
    case 6: return "64x32/512";
    default: return "?";
  }
}

template <typename T>
int tile2d_vec_ok(const Tile2DArgs<T>& a) {
  return (a.g.n[0] % 2 == 0) && (a.zero_init || aligned16(a.x)) &&
         aligned16(a.xo) && aligned16(a.b) && aligned16(a.ax) &&
         aligned16(a.ay);
}

template <typename T, int RX, int NPY, int K, int NU, bool DOWN>
static hipError_t launch_batch_one(const Tile2DArgs<T>* tab, const int* start,
                                   int ng, int nblocks, hipStream_t s,
                                   hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0 && ev1)
    hipExtLaunchKernelGGL((k_tile2d_batch<T, RX, NPY, K, NU, DOWN>),
                          dim3(nblocks), dim3(RX / 2 * NPY), 0, s, ev0, ev1, 0,
                          tab, start, ng);
  else
    hipLaunchKernelGGL((k_tile2d_batch<T, RX, NPY, K, NU, DOWN>), dim3(nblocks),
                       dim3(RX / 2 * NPY), 0, s, tab, start, ng);
  return hipGetLastError();
}

template <typename T, int RX, int NPY, int K>
static hipError_t batch_shape(const Tile2DArgs<T>* tab, const int* start,
                              int ng, int nblocks, int nu, bool down,
                              hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (down) {
    switch (nu) {
      case 1: return launch_batch_one<T, RX, NPY, K, 1, true>(tab, start, ng, nblocks, s, ev0, ev1);
      case 2: return launch_batch_one<T, RX, NPY, K, 2, true>(tab, start, ng, nblocks, s, ev0, ev1);
      case 3: return launch_batch_one<T, RX, NPY, K, 3, true>(tab, start, ng, nblocks, s, ev0, ev1);
      default: return hipErrorInvalidValue;
    }
  }
  switch (nu) {
    case 1: return launch_batch_one<T, RX, NPY, K, 1, false>(tab, start, ng, nblocks, s, ev0, ev1);
    case 2: return launch_batch_one<T, RX, NPY, K, 2, false>(tab, start, ng, nblocks, s, ev0, ev1);
    case 3: return launch_batch_one<T, RX, NPY, K, 3, false>(tab, start, ng, nblocks, s, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_tile2d_batch(const Tile2DArgs<T>* tab, const int* start,
                               int ng, int nblocks, int nu, bool down,
                               int variant, hipStream_t s, hipEvent_t ev0,
                               hipEvent_t ev1) {
  if (nblocks == 0) return hipSuccess;
  if (variant < 0 || variant >= kTileVariantsBatch) return hipErrorInvalidValue;
  switch (variant) {
#define FLD_SHAPE_CASE(v, rx, npy, k) \
  case v: return batch_shape<T, rx, npy, k>(tab, start, ng, nblocks, nu, down, s, ev0, ev1);
    FLD_TILE_SHAPES(FLD_SHAPE_CASE)
#undef FLD_SHAPE_CASE
    default: return hipErrorInvalidValue;
  }
}

// With ev0/ev1 given, the launch itself records them (hipExtLaunchKernelGGL):
// their interval is the kernel's own execution, with no marker packets
// between them.
template <typename T, int RX, int NPY, int K, int NU, bool DOWN>
static hipError_t launch_one(const Tile2DArgs<T>& a0, hipStream_t s,
                             int* nblocks, hipEvent_t ev0, hipEvent_t ev1) {
  constexpr int RY = NPY * K;
  constexpr int H = DOWN ? 2 * NU + 2 : 2 * NU;
  constexpr int TX = RX - 2 * H, TY = RY - 2 * H;
  Tile2DArgs<T> a = a0;
  a.tiles_x = (a.g.n[0] + TX - 1) / TX;
  a.tiles_y = (a.g.n[1] + TY - 1) / TY;
  a.vec = tile2d_vec_ok(a);
  const int nb = a.tiles_x * a.tiles_y;
  if (nblocks) *nblocks = nb;
  if (ev0 && ev1)
    hipExtLaunchKernelGGL((k_tile2d<T, RX, NPY, K, NU, DOWN>), dim3(nb),
                          dim3(RX / 2 * NPY), 0, s, ev0, ev1, 0, a);
  else
    hipLaunchKernelGGL((k_tile2d<T, RX, NPY, K, NU, DOWN>), dim3(nb),
                       dim3(RX / 2 * NPY), 0, s, a);
  return hipGetLastError();
}

template <typename T, int RX, int NPY, int K>
static hipError_t single_shape(const Tile2DArgs<T>& a, int nu, bool down,
                               hipStream_t s, int* nb, hipEvent_t e0,
                               hipEvent_t e1) {
  if (down) {
    switch (nu) {
      case 1: return launch_one<T, RX, NPY, K, 1, true>(a, s, nb, e0, e1);
      case 2: return launch_one<T, RX, NPY, K, 2, true>(a, s, nb, e0, e1);
      case 3: return launch_one<T, RX, NPY, K, 3, true>(a, s, nb, e0, e1);
      default: return hipErrorInvalidValue;
    }
  }
  switch (nu) {
    case 1: return launch_one<T, RX, NPY, K, 1, false>(a, s, nb, e0, e1);
    case 2: return launch_one<T, RX, NPY, K, 2, false>(a, s, nb, e0, e1);
    case 3: return launch_one<T, RX, NPY, K, 3, false>(a, s, nb, e0, e1);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_tile2d(const Tile2DArgs<T>& a, int nu, bool down,
                         int variant, hipStream_t s, int* nblocks,
                         hipEvent_t ev0, hipEvent_t ev1) {
  switch (variant) {
#define FLD_SHAPE_CASE(v, rx, npy, k) \
  case v: return single_shape<T, rx, npy, k>(a, nu, down, s, nblocks, ev0, ev1);
    FLD_TILE_SHAPES(FLD_SHAPE_CASE)
#undef FLD_SHAPE_CASE
    default: return hipErrorInvalidValue;
  }
}

int tile2d_blocks(const Geom& g, int nu, bool down, int variant) {
  int tx, ty;
  return tile2d_grid(g, nu, down, variant, &tx, &ty);
}

int tile2d_grid(const Geom& g, int nu, bool down, int variant, int* tiles_x,
                int* tiles_y) {
  const Shape sh = kShapes[variant];
  const int H = down ? 2 * nu + 2 : 2 * nu;
  const int TX = sh.rx - 2 * H, TY = sh.npy * sh.k - 2 * H;
  *tiles_x = (g.n[0] + TX - 1) / TX;
  *tiles_y = (g.n[1] + TY - 1) / TY;
  return *tiles_x * *tiles_y;
}

template int tile2d_vec_ok<double>(const Tile2DArgs<double>&);
template int tile2d_vec_ok<float>(const Tile2DArgs<float>&);
template hipError_t launch_tile2d<double>(const Tile2DArgs<double>&, int, bool,
                                          int, hipStream_t, int*, hipEvent_t,
                                          hipEvent_t);
template hipError_t launch_tile2d<float>(const Tile2DArgs<float>&, int, bool,
                                         int, hipStream_t, int*, hipEvent_t,
                                         hipEvent_t);
template hipError_t launch_tile2d_batch<double>(const Tile2DArgs<double>*,
                                                const int*, int, int, int,
                                                bool, int, hipStream_t,
                                                hipEvent_t, hipEvent_t);
template hipError_t launch_tile2d_batch<float>(const Tile2DArgs<float>*,
                                               const int*, int, int, int, bool,
                                               int, hipStream_t, hipEvent_t,
                                               hipEvent_t);

}  // namespace fld
