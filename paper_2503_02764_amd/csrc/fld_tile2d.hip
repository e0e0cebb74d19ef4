// LDS-tiled, temporally blocked multigrid kernels for 2D levels (gfx950).
//
// One workgroup owns a region of RX x RY cells: an output tile plus a halo
// of H cells on every side.  It loads x once into LDS and keeps, per cell,
// the Gauss-Seidel weights in registers:
//   x_new = b/d + (a_l x_l + a_r x_r + a_d x_d + a_u x_u)/d,  d = 1 + sum a.
// It then runs NU red-black sweeps (2*NU colour passes) entirely on chip.
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
// The iterate is double-buffered: a block reads its region (halo included)
// from x and writes its tile interior to xo, so no block can see a
// neighbour's already-updated cells, whatever the dispatch order.
//
// Blocks are dispatched round-robin over the 8 XCDs; tiles are renumbered
// so that each XCD sweeps one contiguous band of tiles and the halos that
// neighbouring tiles share stay in that XCD's L2.
#include "fld_internal.h"
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
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T r = T(0);
  if (threadIdx.x == 0)
    for (int q = 0; q < (nt + 63) / 64; ++q) r += sh[q];
  return r;
}

}  // namespace

template <typename T, int RX, int NPY, int K, int NU, bool DOWN>
__device__ __forceinline__ void tile2d_body(const Tile2DArgs<T>& A,
                                            const int tile) {
  constexpr int NT = RX / 2 * NPY;
  constexpr int RY = NPY * K;
  constexpr int H = DOWN ? 2 * NU + 2 : 2 * NU;
  constexpr int TX = RX - 2 * H, TY = RY - 2 * H;
  constexpr int LX = RX + 2, LY = RY + 2;  // LDS copy with a zero border
  static_assert(K % 2 == 0 && RX % 2 == 0 && TX > 0 && TY > 0, "tile shape");
  __shared__ T xs[LY * LX];
  __shared__ double red[NT / 64 + 1];
  if (A.ctrl->done != kRunning) return;

  const int tyi = tile / A.tiles_x, txi = tile - tyi * A.tiles_x;
  const int gx0 = txi * TX - H, gy0 = tyi * TY - H;  // region origin (even)
  const int px = threadIdx.x % (RX / 2), py = threadIdx.x / (RX / 2);
  const int nx = A.g.n[0], ny = A.g.n[1];
  const int perx = A.g.per[0], pery = A.g.per[1];

  // zero border of the LDS copy
  for (int i = threadIdx.x; i < 2 * LX + 2 * RY; i += NT) {
    int o;
    if (i < LX) o = i;
    else if (i < 2 * LX) o = (LY - 1) * LX + (i - LX);
    else if (i < 2 * LX + RY) o = (1 + i - 2 * LX) * LX;
    else o = (1 + i - 2 * LX - RY) * LX + LX - 1;
    xs[o] = T(0);
  }

  T bp[K][2], wl[K][2], wr[K][2], wd[K][2], wu[K][2];
  T dn[DOWN ? K : 1][2];
  (void)dn;
  const int mx0 = map_coord(gx0 + 2 * px, nx, perx);
  const int mx1 = map_coord(gx0 + 2 * px + 1, nx, perx);
  // Loads are issued branch-free (indices clamped into the domain, values
  // masked afterwards) for all rows of the thread at once, so that they are
  // all in flight before the first use.
  constexpr int KG = DOWN ? K : K / 2;  // rows per load group
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += KG) {
    T lx[KG][2], lb[KG][2], lal[KG][2], lar[KG][2], lad[KG][2], lau[KG][2];
    T le[DOWN ? 1 : KG][2][4];
    (void)le;
    bool vv[KG][2], vl[KG][2], vd[KG][2];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
      const int my = map_coord(gy0 + py * K + k0 + kk, ny, pery);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int mx = q ? mx1 : mx0;
        const bool v = mx >= 0 && my >= 0;
        const int cx = v ? mx : 0, cy = v ? my : 0;
        vv[kk][q] = v;
        vl[kk][q] = v && (cx > 0 || perx);
        vd[kk][q] = v && (cy > 0 || pery);
        const int64_t gi = (int64_t)cy * nx + cx;
        const int64_t gl = cx > 0 ? gi - 1 : gi + nx - 1;
        const int64_t gd = cy > 0 ? gi - nx : gi + (int64_t)(ny - 1) * nx;
        lx[kk][q] = A.zero_init ? T(0) : A.x[gi];
        lb[kk][q] = A.b[gi];
        lar[kk][q] = A.ax[gi];
        lau[kk][q] = A.ay[gi];
        lal[kk][q] = A.ax[gl];
        lad[kk][q] = A.ay[gd];
        if constexpr (!DOWN) {
          // bilinear prolongation of the coarse correction
          const int ncx = A.gc.n[0], ncy = A.gc.n[1];
          const int I = cx >> 1, J = cy >> 1;
          int I2 = (cx & 1) ? I + 1 : I - 1;
          int J2 = (cy & 1) ? J + 1 : J - 1;
          if (I2 < 0) I2 = perx ? ncx - 1 : 0;
          if (I2 >= ncx) I2 = perx ? 0 : ncx - 1;
          if (J2 < 0) J2 = pery ? ncy - 1 : 0;
          if (J2 >= ncy) J2 = pery ? 0 : ncy - 1;
          le[kk][q][0] = A.ce[(int64_t)J * ncx + I];
          le[kk][q][1] = A.ce[(int64_t)J * ncx + I2];
          le[kk][q][2] = A.ce[(int64_t)J2 * ncx + I];
          le[kk][q][3] = A.ce[(int64_t)J2 * ncx + I2];
        }
      }
    }
#pragma unroll
    for (int kk = 0; kk < KG; ++kk)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = k0 + kk;
        const bool v = vv[kk][q];
        T xv = v ? lx[kk][q] : T(0);
        const T bv = v ? lb[kk][q] : T(0);
        const T ar = v ? lar[kk][q] : T(0);
        const T au = v ? lau[kk][q] : T(0);
        const T al = vl[kk][q] ? lal[kk][q] : T(0);
        const T ad = vd[kk][q] ? lad[kk][q] : T(0);
        if constexpr (!DOWN) {
          if (v)
            xv += T(0.5625) * le[kk][q][0] + T(0.1875) * le[kk][q][1] +
                  T(0.1875) * le[kk][q][2] + T(0.0625) * le[kk][q][3];
        }
        const T d = T(1) + al + ar + ad + au;
        const T inv = T(1) / d;
        bp[k][q] = bv * inv;
        wl[k][q] = al * inv;
        wr[k][q] = ar * inv;
        wd[k][q] = ad * inv;
        wu[k][q] = au * inv;
        if constexpr (DOWN) dn[k][q] = d;
        xs[(py * K + k + 1) * LX + 2 * px + q + 1] = xv;
      }
  }
  __syncthreads();

#pragma unroll
  for (int pass = 0; pass < 2 * NU; ++pass) {
    const int c = pass & 1;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int q = (c + k) & 1;
      const int ly = py * K + k;
      const int o = (ly + 1) * LX + 2 * px + q + 1;
      const T xn = bp[k][q] + wl[k][q] * xs[o - 1] + wr[k][q] * xs[o + 1] +
                   wd[k][q] * xs[o - LX] + wu[k][q] * xs[o + LX];
      xs[o] = xn;
    }
    __syncthreads();
  }

  // write the tile interior (cells of this tile inside the domain)
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int ly = py * K + k;
    const int gy = gy0 + ly;
    if (ly < H || ly >= H + TY || gy >= ny) continue;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int lx = 2 * px + q;
      const int gx = gx0 + lx;
      if (lx < H || lx >= H + TX || gx >= nx) continue;
      A.xo[(int64_t)gy * nx + gx] = xs[(ly + 1) * LX + lx + 1];
    }
  }

  if constexpr (DOWN) {
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
          const int o = (ly + kk + 1) * LX + lx + q + 1;
          const T xc = xs[o];
          r[kk][q] = dn[k + kk][q] *
                     (bp[k + kk][q] + wl[k + kk][q] * xs[o - 1] +
                      wr[k + kk][q] * xs[o + 1] + wd[k + kk][q] * xs[o - LX] +
                      wu[k + kk][q] * xs[o + LX] - xc);
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

// ---------------------------------------------------------------------------
// Pipelined form: each block walks a contiguous range of tiles and issues the
// global loads of its next tile before running the colour passes of the
// current one (loads stay in flight across the LDS barriers), so HBM traffic
// overlaps the on-chip work instead of alternating with it.  Same arithmetic
// per cell as tile2d_body; two rows per thread (K = 2).
// ---------------------------------------------------------------------------

template <typename T, bool DOWN>
struct TileRaw {  // one thread's loaded operands of one tile (2 rows x 2 cells)
  T x[2][2], b[2][2], al[2][2], ar[2][2], ad[2][2], au[2][2];
  T e[DOWN ? 1 : 2][2][4];
  bool vv[2][2], vl[2][2], vd[2][2];
};

template <typename T, int RX, int NPY, bool DOWN>
__device__ __forceinline__ void tile_issue(const Tile2DArgs<T>& A, int tile,
                                           int H, int TX, int TY,
                                           TileRaw<T, DOWN>& R) {
  constexpr int K = 2;
  const int tyi = tile / A.tiles_x, txi = tile - tyi * A.tiles_x;
  const int gx0 = txi * TX - H, gy0 = tyi * TY - H;
  const int px = threadIdx.x % (RX / 2), py = threadIdx.x / (RX / 2);
  const int nx = A.g.n[0], ny = A.g.n[1];
  const int perx = A.g.per[0], pery = A.g.per[1];
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
      R.vv[k][q] = v;
      R.vl[k][q] = v && (cx > 0 || perx);
      R.vd[k][q] = v && (cy > 0 || pery);
      const int64_t gi = (int64_t)cy * nx + cx;
      const int64_t gl = cx > 0 ? gi - 1 : gi + nx - 1;
      const int64_t gd = cy > 0 ? gi - nx : gi + (int64_t)(ny - 1) * nx;
      R.x[k][q] = A.zero_init ? T(0) : A.x[gi];
      R.b[k][q] = A.b[gi];
      R.ar[k][q] = A.ax[gi];
      R.au[k][q] = A.ay[gi];
      R.al[k][q] = A.ax[gl];
      R.ad[k][q] = A.ay[gd];
      if constexpr (!DOWN) {
        const int ncx = A.gc.n[0], ncy = A.gc.n[1];
        const int I = cx >> 1, J = cy >> 1;
        int I2 = (cx & 1) ? I + 1 : I - 1;
        int J2 = (cy & 1) ? J + 1 : J - 1;
        if (I2 < 0) I2 = perx ? ncx - 1 : 0;
        if (I2 >= ncx) I2 = perx ? 0 : ncx - 1;
        if (J2 < 0) J2 = pery ? ncy - 1 : 0;
        if (J2 >= ncy) J2 = pery ? 0 : ncy - 1;
        R.e[k][q][0] = A.ce[(int64_t)J * ncx + I];
        R.e[k][q][1] = A.ce[(int64_t)J * ncx + I2];
        R.e[k][q][2] = A.ce[(int64_t)J2 * ncx + I];
        R.e[k][q][3] = A.ce[(int64_t)J2 * ncx + I2];
      }
    }
  }
}

template <typename T, int RX, int NPY, int NU, bool DOWN>
__device__ __forceinline__ void tile2d_pipe_body(const Tile2DArgs<T>& A,
                                                 int t0, int t1) {
  constexpr int K = 2;
  constexpr int NT = RX / 2 * NPY;
  constexpr int RY = NPY * K;
  constexpr int H = DOWN ? 2 * NU + 2 : 2 * NU;
  constexpr int TX = RX - 2 * H, TY = RY - 2 * H;
  constexpr int LX = RX + 2, LY = RY + 2;
  static_assert(RX % 2 == 0 && TX > 0 && TY > 0, "tile shape");
  __shared__ T xs[LY * LX];
  __shared__ double red[NT / 64 + 1];
  if (A.ctrl->done != kRunning || t0 >= t1) return;
  const int px = threadIdx.x % (RX / 2), py = threadIdx.x / (RX / 2);
  const int nx = A.g.n[0], ny = A.g.n[1];
  for (int i = threadIdx.x; i < 2 * LX + 2 * RY; i += NT) {
    int o;
    if (i < LX) o = i;
    else if (i < 2 * LX) o = (LY - 1) * LX + (i - LX);
    else if (i < 2 * LX + RY) o = (1 + i - 2 * LX) * LX;
    else o = (1 + i - 2 * LX - RY) * LX + LX - 1;
    xs[o] = T(0);
  }
  TileRaw<T, DOWN> R;
  tile_issue<T, RX, NPY, DOWN>(A, t0, H, TX, TY, R);
  for (int tile = t0; tile < t1; ++tile) {
    const int tyi = tile / A.tiles_x, txi = tile - tyi * A.tiles_x;
    const int gx0 = txi * TX - H, gy0 = tyi * TY - H;
    T bp[K][2], wl[K][2], wr[K][2], wd[K][2], wu[K][2];
    T dn[DOWN ? K : 1][2];
    (void)dn;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const bool v = R.vv[k][q];
        T xv = v ? R.x[k][q] : T(0);
        const T bv = v ? R.b[k][q] : T(0);
        const T ar = v ? R.ar[k][q] : T(0);
        const T au = v ? R.au[k][q] : T(0);
        const T al = R.vl[k][q] ? R.al[k][q] : T(0);
        const T ad = R.vd[k][q] ? R.ad[k][q] : T(0);
        if constexpr (!DOWN) {
          if (v)
            xv += T(0.5625) * R.e[k][q][0] + T(0.1875) * R.e[k][q][1] +
                  T(0.1875) * R.e[k][q][2] + T(0.0625) * R.e[k][q][3];
        }
        const T d = T(1) + al + ar + ad + au;
        const T inv = T(1) / d;
        bp[k][q] = bv * inv;
        wl[k][q] = al * inv;
        wr[k][q] = ar * inv;
        wd[k][q] = ad * inv;
        wu[k][q] = au * inv;
        if constexpr (DOWN) dn[k][q] = d;
        xs[(py * K + k + 1) * LX + 2 * px + q + 1] = xv;
      }
    __syncthreads();
    // the next tile's operands travel while this one is smoothed
    if (tile + 1 < t1) tile_issue<T, RX, NPY, DOWN>(A, tile + 1, H, TX, TY, R);
#pragma unroll
    for (int pass = 0; pass < 2 * NU; ++pass) {
      const int c = pass & 1;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int q = (c + k) & 1;
        const int o = (py * K + k + 1) * LX + 2 * px + q + 1;
        xs[o] = bp[k][q] + wl[k][q] * xs[o - 1] + wr[k][q] * xs[o + 1] +
                wd[k][q] * xs[o - LX] + wu[k][q] * xs[o + LX];
      }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int ly = py * K + k;
      const int gy = gy0 + ly;
      if (ly < H || ly >= H + TY || gy >= ny) continue;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int lx = 2 * px + q;
        const int gx = gx0 + lx;
        if (lx < H || lx >= H + TX || gx >= nx) continue;
        A.xo[(int64_t)gy * nx + gx] = xs[(ly + 1) * LX + lx + 1];
      }
    }
    if constexpr (DOWN) {
      double r2 = 0.0;
      const int ncx = A.gc.n[0];
      const int lx = 2 * px;
      const int gx = gx0 + lx;
      const int ly = py * K;
      const int gy = gy0 + ly;
      if (lx >= H && lx < H + TX && gx < nx && ly >= H && ly < H + TY &&
          gy < ny) {
        T r[2][2];
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int o = (ly + kk + 1) * LX + lx + q + 1;
            const T xc = xs[o];
            r[kk][q] = dn[kk][q] *
                       (bp[kk][q] + wl[kk][q] * xs[o - 1] + wr[kk][q] * xs[o + 1] +
                        wd[kk][q] * xs[o - LX] + wu[kk][q] * xs[o + LX] - xc);
          }
        const T s = (r[0][0] + r[0][1]) + (r[1][0] + r[1][1]);
        A.cb[(int64_t)(gy >> 1) * ncx + (gx >> 1)] = T(0.25) * s;
        r2 = (double)r[0][0] * r[0][0] + (double)r[0][1] * r[0][1] +
             (double)r[1][0] * r[1][0] + (double)r[1][1] * r[1][1];
      }
      if (A.partials) {
        const double t = block_sum_t<double>(r2, red, NT);
        if (threadIdx.x == 0) A.partials[tile] = t;
      }
    }
    __syncthreads();  // the LDS copy is rewritten for the next tile
  }
}

template <typename T, int RX, int NPY, int NU, bool DOWN>
__global__ void __launch_bounds__(RX / 2 * NPY) k_tile2d_pipe(Tile2DArgs<T> A,
                                                             int per_block) {
  // contiguous tile ranges; block -> XCD round-robin as in k_tile2d
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int nt = A.tiles_x * A.tiles_y;
  const int t0 = b * per_block;
  const int t1 = t0 + per_block < nt ? t0 + per_block : nt;
  tile2d_pipe_body<T, RX, NPY, NU, DOWN>(A, t0, t1);
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
// Pipelined (k_tile2d_pipe; single grids only), blocks per CU:
//   7: 64 x 32, 512 threads, 2      8: 32 x 32, 256 threads, 4
//   9: 64 x 32, 512 threads, 1
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
    {64, 16, 2}, {32, 16, 2}, {64, 16, 2}};
constexpr int kPipeBlocksPerCU[3] = {2, 4, 1};

int cu_count() {
  static const int n = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) !=
            hipSuccess || v < 1)
      v = 256;
    return v;
  }();
  return n;
}
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
    case 7: return "64x32/512 pipelined x2";
    case 8: return "32x32/256 pipelined x4";
    case 9: return "64x32/512 pipelined x1";
    default: return "?";
  }
}

template <typename T, int RX, int NPY, int K, int NU, bool DOWN>
static hipError_t launch_batch_one(const Tile2DArgs<T>* tab, const int* start,
                                   int ng, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_tile2d_batch<T, RX, NPY, K, NU, DOWN>), dim3(nblocks),
                     dim3(RX / 2 * NPY), 0, s, tab, start, ng);
  return hipGetLastError();
}

template <typename T, int RX, int NPY, int K>
static hipError_t batch_shape(const Tile2DArgs<T>* tab, const int* start,
                              int ng, int nblocks, int nu, bool down,
                              hipStream_t s) {
  if (down) {
    switch (nu) {
      case 1: return launch_batch_one<T, RX, NPY, K, 1, true>(tab, start, ng, nblocks, s);
      case 2: return launch_batch_one<T, RX, NPY, K, 2, true>(tab, start, ng, nblocks, s);
      case 3: return launch_batch_one<T, RX, NPY, K, 3, true>(tab, start, ng, nblocks, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (nu) {
    case 1: return launch_batch_one<T, RX, NPY, K, 1, false>(tab, start, ng, nblocks, s);
    case 2: return launch_batch_one<T, RX, NPY, K, 2, false>(tab, start, ng, nblocks, s);
    case 3: return launch_batch_one<T, RX, NPY, K, 3, false>(tab, start, ng, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_tile2d_batch(const Tile2DArgs<T>* tab, const int* start,
                               int ng, int nblocks, int nu, bool down,
                               int variant, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  if (variant >= kTileVariantsBatch) return hipErrorInvalidValue;
  switch (variant) {
#define FLD_SHAPE_CASE(v, rx, npy, k) \
  case v: return batch_shape<T, rx, npy, k>(tab, start, ng, nblocks, nu, down, s);
    FLD_TILE_SHAPES(FLD_SHAPE_CASE)
#undef FLD_SHAPE_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int RX, int NPY, int K, int NU, bool DOWN>
static hipError_t launch_one(const Tile2DArgs<T>& a0, hipStream_t s,
                             int* nblocks) {
  constexpr int RY = NPY * K;
  constexpr int H = DOWN ? 2 * NU + 2 : 2 * NU;
  constexpr int TX = RX - 2 * H, TY = RY - 2 * H;
  Tile2DArgs<T> a = a0;
  a.tiles_x = (a.g.n[0] + TX - 1) / TX;
  a.tiles_y = (a.g.n[1] + TY - 1) / TY;
  const int nb = a.tiles_x * a.tiles_y;
  if (nblocks) *nblocks = nb;
  hipLaunchKernelGGL((k_tile2d<T, RX, NPY, K, NU, DOWN>), dim3(nb),
                     dim3(RX / 2 * NPY), 0, s, a);
  return hipGetLastError();
}

template <typename T, int RX, int NPY, int K>
static hipError_t single_shape(const Tile2DArgs<T>& a, int nu, bool down,
                               hipStream_t s, int* nblocks) {
  if (down) {
    switch (nu) {
      case 1: return launch_one<T, RX, NPY, K, 1, true>(a, s, nblocks);
      case 2: return launch_one<T, RX, NPY, K, 2, true>(a, s, nblocks);
      case 3: return launch_one<T, RX, NPY, K, 3, true>(a, s, nblocks);
      default: return hipErrorInvalidValue;
    }
  }
  switch (nu) {
    case 1: return launch_one<T, RX, NPY, K, 1, false>(a, s, nblocks);
    case 2: return launch_one<T, RX, NPY, K, 2, false>(a, s, nblocks);
    case 3: return launch_one<T, RX, NPY, K, 3, false>(a, s, nblocks);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int RX, int NPY, int NU, bool DOWN>
static hipError_t launch_pipe_one(const Tile2DArgs<T>& a0, int per_cu,
                                  hipStream_t s, int* ntiles) {
  constexpr int RY = NPY * 2;
  constexpr int H = DOWN ? 2 * NU + 2 : 2 * NU;
  constexpr int TX = RX - 2 * H, TY = RY - 2 * H;
  Tile2DArgs<T> a = a0;
  a.tiles_x = (a.g.n[0] + TX - 1) / TX;
  a.tiles_y = (a.g.n[1] + TY - 1) / TY;
  const int nt = a.tiles_x * a.tiles_y;
  if (ntiles) *ntiles = nt;
  const int target = cu_count() * per_cu;
  const int per_block = (nt + target - 1) / target;
  const int nb = (nt + per_block - 1) / per_block;
  hipLaunchKernelGGL((k_tile2d_pipe<T, RX, NPY, NU, DOWN>), dim3(nb),
                     dim3(RX / 2 * NPY), 0, s, a, per_block);
  return hipGetLastError();
}

template <typename T, int RX, int NPY>
static hipError_t pipe_shape(const Tile2DArgs<T>& a, int nu, bool down,
                             int per_cu, hipStream_t s, int* ntiles) {
  if (down) {
    switch (nu) {
      case 1: return launch_pipe_one<T, RX, NPY, 1, true>(a, per_cu, s, ntiles);
      case 2: return launch_pipe_one<T, RX, NPY, 2, true>(a, per_cu, s, ntiles);
      case 3: return launch_pipe_one<T, RX, NPY, 3, true>(a, per_cu, s, ntiles);
      default: return hipErrorInvalidValue;
    }
  }
  switch (nu) {
    case 1: return launch_pipe_one<T, RX, NPY, 1, false>(a, per_cu, s, ntiles);
    case 2: return launch_pipe_one<T, RX, NPY, 2, false>(a, per_cu, s, ntiles);
    case 3: return launch_pipe_one<T, RX, NPY, 3, false>(a, per_cu, s, ntiles);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_tile2d(const Tile2DArgs<T>& a, int nu, bool down,
                         int variant, hipStream_t s, int* nblocks) {
  switch (variant) {
    case 7: return pipe_shape<T, 64, 16>(a, nu, down, kPipeBlocksPerCU[0], s, nblocks);
    case 8: return pipe_shape<T, 32, 16>(a, nu, down, kPipeBlocksPerCU[1], s, nblocks);
    case 9: return pipe_shape<T, 64, 16>(a, nu, down, kPipeBlocksPerCU[2], s, nblocks);
    default: break;
  }
  switch (variant) {
#define FLD_SHAPE_CASE(v, rx, npy, k) \
  case v: return single_shape<T, rx, npy, k>(a, nu, down, s, nblocks);
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

template hipError_t launch_tile2d<double>(const Tile2DArgs<double>&, int, bool,
                                          int, hipStream_t, int*);
template hipError_t launch_tile2d<float>(const Tile2DArgs<float>&, int, bool,
                                         int, hipStream_t, int*);
template hipError_t launch_tile2d_batch<double>(const Tile2DArgs<double>*,
                                                const int*, int, int, int,
                                                bool, int, hipStream_t);
template hipError_t launch_tile2d_batch<float>(const Tile2DArgs<float>*,
                                               const int*, int, int, int, bool,
                                               int, hipStream_t);

}  // namespace fld
