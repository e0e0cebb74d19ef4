// Coarse-level face coefficients of a 2D hierarchy, several levels per launch
// (gfx950).
//
// The rule is that of k_coarsen (multigrid of Sect. 3): the coarse face
// between coarse cells c and c+1 along d is a quarter of the mean, over the
// two fine rows crossing it, of the series conductance of the three fine
// faces on each row (half of the face inside cell c, the face on the coarse
// face, half of the face inside cell c+1), 2 / (0.5/a0 + 1/a1 + 0.5/a2), or 0
// when one of them is 0; a coarse face on a Neumann wall stays 0.  The
// operations per value are those of k_coarsen, so the coefficients are the
// same bits.  The difference is the launch structure: on a 1024^2 grid the
// eight coarsening launches (most of them a single block of latency) become
// three.
//
//   k_coarsen2d_pair: levels l+1 and l+2 from level l.  A block owns a PT x PT
//     tile of level l+2; it computes the level-(l+1) faces that tile needs
//     (its own 2PT x 2PT plus one more face along the face direction) into
//     LDS, writes its own 2PT x 2PT of them, then the level-(l+2) tile from
//     LDS.
//   k_coarsen2d_whole: every remaining level from level l in one block of
//     1024 threads, whole levels in LDS (level l+1 of at most 1024 cells).
#include "fld_internal.h"
#include "fld_device.h"

namespace fld {

namespace {

// level-(l+2) tile of the pair kernel: 8 x 8, so that a 1024^2 grid's
// first pair runs 1024 blocks of about one round of loads each (16 x 16:
// 256 blocks, one per CU, each thread four dependent rounds)
constexpr int PT = 8;
constexpr int PR = 2 * PT;       // level-(l+1) cells of the tile per side
constexpr int PNT = 256;         // pair kernel threads
constexpr int WNT = 1024;        // whole-levels kernel threads
constexpr int WMAX = 1024;       // cells of the first level of a whole stage

template <typename T>
struct Coarsen2DArgs {
  int n[kMaxLevels], m[kMaxLevels];  // cells along x and y per stage level
  int perx, pery;
  int levels;                        // output levels (pair: 2)
  const T* fa[2];                    // faces of the stage's input level
  T* ca[kMaxLevels][2];              // faces of output level j (1-based)
  int tiles_x;                       // pair kernel: tiles along x
};

// mean of the two series paths of a 2D coarse face, k_coarsen's rounding
template <typename T>
__device__ __forceinline__ T mean_of_paths(T p0, T p1) {
  T s = T(0);
  s += p0;
  s += p1;
  return T(0.25) * s / T(2);
}

// Coarse face along d (0: x, 1: y) of coarse cell (X, Y) of an n x m level,
// from the fine level held by src(d, xf, yf) (2n x 2m cells, indices already
// in range).
template <typename T, typename Src>
__device__ __forceinline__ T coarse_face(int d, int X, int Y, int n, int m,
                                         int per, Src src) {
  if (d == 0) {
    if (X == n - 1 && !per) return T(0);
    const int nf = 2 * n;
    const int x0 = 2 * X, x1 = (2 * X + 1) % nf, x2 = (2 * X + 2) % nf;
    const T p0 = series_path(src(0, x0, 2 * Y), src(0, x1, 2 * Y),
                             src(0, x2, 2 * Y));
    const T p1 = series_path(src(0, x0, 2 * Y + 1), src(0, x1, 2 * Y + 1),
                             src(0, x2, 2 * Y + 1));
    return mean_of_paths(p0, p1);
  }
  if (Y == m - 1 && !per) return T(0);
  const int mf = 2 * m;
  const int y0 = 2 * Y, y1 = (2 * Y + 1) % mf, y2 = (2 * Y + 2) % mf;
  const T p0 =
      series_path(src(1, 2 * X, y0), src(1, 2 * X, y1), src(1, 2 * X, y2));
  const T p1 = series_path(src(1, 2 * X + 1, y0), src(1, 2 * X + 1, y1),
                           src(1, 2 * X + 1, y2));
  return mean_of_paths(p0, p1);
}

}  // namespace

template <typename T>
__global__ void __launch_bounds__(PNT) k_coarsen2d_pair(Coarsen2DArgs<T> A) {
  // level-(l+1) faces of the tile: x faces over (PR + 1) x PR cells, y faces
  // over PR x (PR + 1), origin (2 ox2, 2 oy2), wrapped into the level
  __shared__ T fx[PR][PR + 1];
  __shared__ T fy[PR + 1][PR];
  const int by = blockIdx.x / A.tiles_x, bx = blockIdx.x - by * A.tiles_x;
  const int ox2 = bx * PT, oy2 = by * PT;
  const int ox1 = 2 * ox2, oy1 = 2 * oy2;
  const int n0 = A.n[0], n1 = A.n[1], m1 = A.m[1], n2 = A.n[2], m2 = A.m[2];
  auto g0 = [&](int d, int x, int y) {
    return A.fa[d][(int64_t)y * n0 + x];
  };
  for (int k = threadIdx.x; k < PR * (PR + 1); k += PNT) {
    {  // x face (lx, ly), lx < PR + 1
      const int ly = k / (PR + 1), lx = k - ly * (PR + 1);
      const int X = (ox1 + lx) % n1, Y = (oy1 + ly) % m1;
      const T v = coarse_face<T>(0, X, Y, n1, m1, A.perx, g0);
      fx[ly][lx] = v;
      if (lx < PR && ox1 + lx < n1 && oy1 + ly < m1)
        A.ca[1][0][(int64_t)(oy1 + ly) * n1 + ox1 + lx] = v;
    }
    {  // y face (lx, ly), ly < PR + 1
      const int ly = k / PR, lx = k - ly * PR;
      const int X = (ox1 + lx) % n1, Y = (oy1 + ly) % m1;
      const T v = coarse_face<T>(1, X, Y, n1, m1, A.pery, g0);
      fy[ly][lx] = v;
      if (ly < PR && ox1 + lx < n1 && oy1 + ly < m1)
        A.ca[1][1][(int64_t)(oy1 + ly) * n1 + ox1 + lx] = v;
    }
  }
  __syncthreads();
  // level l+2: the tile's own faces, level-(l+1) values from LDS (local
  // index = 2 x local coarse index + offset, the same cells as the wrapped
  // global indices of coarse_face)
  const int i = threadIdx.x % PT, j = threadIdx.x / PT;
  const int X = ox2 + i, Y = oy2 + j;
  if (j < PT && X < n2 && Y < m2) {
    auto lx_ = [&](int d, int x, int y) {
      // x, y are level-(l+1) indices relative to the tile origin
      return d == 0 ? fx[y][x] : fy[y][x];
    };
    T ax, ay;
    if (X == n2 - 1 && !A.perx) {
      ax = T(0);
    } else {
      const T p0 = series_path(lx_(0, 2 * i, 2 * j), lx_(0, 2 * i + 1, 2 * j),
                               lx_(0, 2 * i + 2, 2 * j));
      const T p1 =
          series_path(lx_(0, 2 * i, 2 * j + 1), lx_(0, 2 * i + 1, 2 * j + 1),
                      lx_(0, 2 * i + 2, 2 * j + 1));
      ax = mean_of_paths(p0, p1);
    }
    if (Y == m2 - 1 && !A.pery) {
      ay = T(0);
    } else {
      const T p0 = series_path(lx_(1, 2 * i, 2 * j), lx_(1, 2 * i, 2 * j + 1),
                               lx_(1, 2 * i, 2 * j + 2));
      const T p1 =
          series_path(lx_(1, 2 * i + 1, 2 * j), lx_(1, 2 * i + 1, 2 * j + 1),
                      lx_(1, 2 * i + 1, 2 * j + 2));
      ay = mean_of_paths(p0, p1);
    }
    A.ca[2][0][(int64_t)Y * n2 + X] = ax;
    A.ca[2][1][(int64_t)Y * n2 + X] = ay;
  }
}

template <typename T>
__global__ void __launch_bounds__(WNT) k_coarsen2d_whole(Coarsen2DArgs<T> A) {
  __shared__ T buf[2][2][WMAX];  // ping-pong: [level parity][x|y][cell]
  for (int j = 1; j <= A.levels; ++j) {
    const int n = A.n[j], m = A.m[j], nf = A.n[j - 1];
    T(*dst)[WMAX] = buf[j & 1];
    T(*src)[WMAX] = buf[(j - 1) & 1];
    for (int k = threadIdx.x; k < n * m; k += WNT) {
      const int Y = k / n, X = k - Y * n;
      T ax, ay;
      if (j == 1) {
        auto g = [&](int d, int x, int y) {
          return A.fa[d][(int64_t)y * nf + x];
        };
        ax = coarse_face<T>(0, X, Y, n, m, A.perx, g);
        ay = coarse_face<T>(1, X, Y, n, m, A.pery, g);
      } else {
        auto g = [&](int d, int x, int y) { return src[d][y * nf + x]; };
        ax = coarse_face<T>(0, X, Y, n, m, A.perx, g);
        ay = coarse_face<T>(1, X, Y, n, m, A.pery, g);
      }
      dst[0][k] = ax;
      dst[1][k] = ay;
      A.ca[j][0][k] = ax;
      A.ca[j][1][k] = ay;
    }
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_coarsen2d(const Geom* g, int L, T* const (*a)[3],
                            hipStream_t s) {
  // a[l][d]: faces along d of level l; levels 1 .. L-1 are written
  int l = 0;
  while (l + 1 < L) {
    Coarsen2DArgs<T> A;
    A.perx = g[l].per[0];
    A.pery = g[l].per[1];
    A.fa[0] = a[l][0];
    A.fa[1] = a[l][1];
    const int left = L - 1 - l;
    if (g[l + 1].N <= WMAX) {
      A.levels = left;
      for (int j = 0; j <= left; ++j) {
        A.n[j] = g[l + j].n[0];
        A.m[j] = g[l + j].n[1];
        if (j > 0) {
          A.ca[j][0] = a[l + j][0];
          A.ca[j][1] = a[l + j][1];
        }
      }
      hipLaunchKernelGGL(k_coarsen2d_whole<T>, dim3(1), dim3(WNT), 0, s, A);
      l += left;
    } else if (left >= 2) {
      A.levels = 2;
      for (int j = 0; j <= 2; ++j) {
        A.n[j] = g[l + j].n[0];
        A.m[j] = g[l + j].n[1];
        if (j > 0) {
          A.ca[j][0] = a[l + j][0];
          A.ca[j][1] = a[l + j][1];
        }
      }
      A.tiles_x = (A.n[2] + PT - 1) / PT;
      const int tiles_y = (A.m[2] + PT - 1) / PT;
      hipLaunchKernelGGL(k_coarsen2d_pair<T>, dim3(A.tiles_x * tiles_y),
                         dim3(PNT), 0, s, A);
      l += 2;
    } else {
      const T* fa[3] = {a[l][0], a[l][1], nullptr};
      T* ca[3] = {a[l + 1][0], a[l + 1][1], nullptr};
      const hipError_t e = launch_coarsen<T>(g[l], g[l + 1], fa, ca, s);
      if (e != hipSuccess) return e;
      l += 1;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_coarsen2d<double>(const Geom*, int,
                                             double* const (*)[3], hipStream_t);
template hipError_t launch_coarsen2d<float>(const Geom*, int,
                                            float* const (*)[3], hipStream_t);

}  // namespace fld
