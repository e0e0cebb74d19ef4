// Explicit FLD source terms around the implicit radiation update (Sect. 3
// adds them explicitly): the radiation force density f_r = -lambda grad E
// (eq. rad_force with the flux of eq. fld_F), its work v . f_r, and photon
// tiring P : grad v with P = f E (eq. fld_P), the Eddington tensor of
// eq. fld_Eddington_tensor and the Eddington factor f = lambda + lambda^2 R^2
// (eq. fld_f).  grad E and grad v by the five-point fourth-order stencil of
// the coefficient stage, with its ghost mapping (periodic wrap, Neumann
// mirror ghosts) for E and every velocity component; R and lambda as there.
//
// One pass: E and the velocity components are read with their stencil
// neighbours, rho and kappa once, and each requested output written once.
// 1D/2D: one thread per cell, coordinates from the launch grid (no index
// divisions); 3D: blocks march through z (k_explicit_3d).  Expanding
//   P : grad v = E [ (1 - f)/2 div v + (3 f - 1)/2 n . (grad v) . n ]
// keeps the Eddington tensor implicit: no 3 x 3 array per thread.
#include <algorithm>

#include "fld_internal.h"
#include "fld_device.h"

namespace fld {

__device__ __forceinline__ double grad5(const double* __restrict__ f,
                                        const Geom& g, const int c[3],
                                        int64_t idx, int d, double scale) {
  const int64_t st = stride_of(g, d);
  const int64_t base = idx - (int64_t)c[d] * st;
  const int n = g.n[d], p = g.per[d];
  const double m2 = f[base + (int64_t)ghost(c[d] - 2, n, p) * st];
  const double m1 = f[base + (int64_t)ghost(c[d] - 1, n, p) * st];
  const double p1 = f[base + (int64_t)ghost(c[d] + 1, n, p) * st];
  const double p2 = f[base + (int64_t)ghost(c[d] + 2, n, p) * st];
  return (m2 - 8.0 * m1 + 8.0 * p1 - p2) * scale;
}

// Launch grid: 64-cell x-runs by 4 rows per 256-thread block, one plane per
// blockIdx.z (no index divisions; a row's stencil neighbours along x share
// cache lines, those along y and z the block's and its neighbours' rows).
constexpr int kEX = 64, kEY = 4;

__global__ void __launch_bounds__(kEX * kEY) k_explicit(ExplicitArgs A) {
  const int x = blockIdx.x * kEX + threadIdx.x % kEX;
  const int y = blockIdx.y * kEY + threadIdx.x / kEX;
  const int z = blockIdx.z;
  if (x >= A.g.n[0] || y >= A.g.n[1]) return;
  const int c[3] = {x, y, z};
  const int64_t idx = ((int64_t)z * A.g.n[1] + y) * A.g.n[0] + x;
  const int nd = A.g.ndim;
  double G[3] = {0.0, 0.0, 0.0};
  double g2 = 0.0;
  for (int d = 0; d < nd; ++d) {
    G[d] = grad5(A.E, A.g, c, idx, d, A.gscale[d]);
    g2 += G[d] * G[d];
  }
  const double E0 = A.E[idx];
  const double gm = sqrt(g2);
  const double R = gm / (A.rho[idx] * A.kappa[idx] * E0);
  const double lam = flux_limiter(A.limiter, R);
  const double f = lam + lam * lam * R * R;
  double w = 0.0;
  for (int d = 0; d < nd; ++d) {
    const double fr = -lam * G[d];
    if (A.fr[d]) A.fr[d][idx] = fr;
    if (A.work) w += A.v[d][idx] * fr;
  }
  if (A.work) A.work[idx] = w;
  if (A.fedd) A.fedd[idx] = f;
  if (A.tiring) {
    const double inv = gm > 0.0 ? 1.0 / gm : 0.0;
    double div = 0.0, nn = 0.0;
    for (int j = 0; j < nd; ++j) {
      const double nj = G[j] * inv;
      for (int i = 0; i < nd; ++i) {
        const double dv = grad5(A.v[j], A.g, c, idx, i, A.gscale[i]);
        if (i == j) div += dv;
        nn += G[i] * inv * nj * dv;
      }
    }
    A.tiring[idx] = E0 * (0.5 * (1.0 - f) * div + 0.5 * (3.0 * f - 1.0) * nn);
  }
}

// 3D: a block owns a kEX x kEY column tile and marches up through a chunk
// of (at least 8) z planes, keeping the five planes k - 2 .. k + 2 of E and of each
// velocity component of its own column in registers: the z derivatives come
// from there, the x and y ones from loads of plane k (the tile's own rows,
// and its neighbours' rows, which the blocks of the same XCD march through
// at the same time: the tiles of one XCD are contiguous).  The planes of a
// chunk are then read from HBM about once (plus the four planes around it),
// instead of once per plane of the five-point reach.  Same operations, in
// the same order, as k_explicit.
template <bool HAS_V>
__global__ void __launch_bounds__(kEX * kEY)
    k_explicit_3d(ExplicitArgs A, int zc, int group) {
  const Geom& g = A.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int gx = (nx + kEX - 1) / kEX, gy = (ny + kEY - 1) / kEY;
  const int nb = gridDim.x, b = blockIdx.x;
  const int tile = group ? (b % 8) * (nb / 8) + b / 8 : b;
  const int x = (tile % gx) * kEX + threadIdx.x % kEX;
  const int y = ((tile / gx) % gy) * kEY + threadIdx.x / kEX;
  const int z0 = (tile / (gx * gy)) * zc, z1 = min(z0 + zc, nz);
  if (x >= nx || y >= ny || z0 >= nz) return;
  const int64_t sz = (int64_t)nx * ny;
  const int64_t col = (int64_t)y * nx + x;
  const int NF = HAS_V ? 4 : 1;  // E, then v_0 .. v_2
  const double* F[4] = {A.E, A.v[0], A.v[1], A.v[2]};
  // x and y neighbours (ghost mapped) of this column
  int64_t xo[4], yo[4];
  const int dd[4] = {-2, -1, 1, 2};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    xo[j] = (int64_t)y * nx + ghost(x + dd[j], nx, g.per[0]);
    yo[j] = (int64_t)ghost(y + dd[j], ny, g.per[1]) * nx + x;
  }
  auto zoff = [&](int k) { return (int64_t)ghost(k, nz, g.per[2]) * sz; };
  double w[4][5];  // w[f][j]: field f at plane k - 2 + j
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int j = 0; j < 4; ++j) w[f][j] = F[f][zoff(z0 - 2 + j) + col];
  for (int k = z0; k < z1; ++k) {
    const int64_t pk = (int64_t)k * sz, idx = pk + col;
    const int64_t p2 = zoff(k + 2) + col;
#pragma unroll
    for (int f = 0; f < NF; ++f) w[f][4] = F[f][p2];
    // grad of field f along d at this cell
    auto grad = [&](int f, int d) {
      if (d == 2)
        return (w[f][0] - 8.0 * w[f][1] + 8.0 * w[f][3] - w[f][4]) *
               A.gscale[2];
      const int64_t* o = d == 0 ? xo : yo;
      const double* Ff = F[f];
      return (Ff[pk + o[0]] - 8.0 * Ff[pk + o[1]] + 8.0 * Ff[pk + o[2]] -
              Ff[pk + o[3]]) * A.gscale[d];
    };
    double G[3];
    double g2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      G[d] = grad(0, d);
      g2 += G[d] * G[d];
    }
    const double E0 = w[0][2];
    const double gm = sqrt(g2);
    const double R = gm / (A.rho[idx] * A.kappa[idx] * E0);
    const double lam = flux_limiter(A.limiter, R);
    const double fe = lam + lam * lam * R * R;
    double wk = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double fr = -lam * G[d];
      if (A.fr[d]) A.fr[d][idx] = fr;
      if (HAS_V && A.work) wk += w[1 + d][2] * fr;
    }
    if (HAS_V && A.work) A.work[idx] = wk;
    if (A.fedd) A.fedd[idx] = fe;
    if (HAS_V && A.tiring) {
      const double inv = gm > 0.0 ? 1.0 / gm : 0.0;
      double div = 0.0, nn = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double nj = G[j] * inv;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const double dv = grad(1 + j, i);
          if (i == j) div += dv;
          nn += G[i] * inv * nj * dv;
        }
      }
      A.tiring[idx] = E0 * (0.5 * (1.0 - fe) * div + 0.5 * (3.0 * fe - 1.0) * nn);
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int j = 0; j < 4; ++j) w[f][j] = w[f][j + 1];
  }
}

hipError_t launch_explicit(const ExplicitArgs& a, hipStream_t s) {
  if (a.g.N == 0) return hipSuccess;
  if (a.g.ndim == 3) {
    // about 8192 blocks (z chunks of at least 8 planes).  On 256^3 with every
    // output: 751 us against 786 with 4096 blocks, 823 with 2048, 993 with
    // 1024 (158 VGPRs: 12 waves per CU, so the march needs many blocks to
    // hide the latency of its ~38 loads per cell), and 880 us for the
    // one-thread-per-cell kernel, which fetches 2.9x its inputs
    const int tiles = ((a.g.n[0] + kEX - 1) / kEX) * ((a.g.n[1] + kEY - 1) / kEY);
    const int chunks = std::max(1, std::min(a.g.n[2], 8192 / std::max(tiles, 1)));
    const int zc = std::max(std::min(8, a.g.n[2]), (a.g.n[2] + chunks - 1) / chunks);
    const int nb = tiles * ((a.g.n[2] + zc - 1) / zc);
    const int group = nb % 8 == 0;
    if (a.v[0])
      hipLaunchKernelGGL(k_explicit_3d<true>, dim3(nb), dim3(kEX * kEY), 0, s,
                         a, zc, group);
    else
      hipLaunchKernelGGL(k_explicit_3d<false>, dim3(nb), dim3(kEX * kEY), 0,
                         s, a, zc, group);
    return hipGetLastError();
  }
  const dim3 grid((a.g.n[0] + kEX - 1) / kEX, (a.g.n[1] + kEY - 1) / kEY,
                  a.g.n[2]);
  hipLaunchKernelGGL(k_explicit, grid, dim3(kEX * kEY), 0, s, a);
  return hipGetLastError();
}

}  // namespace fld
