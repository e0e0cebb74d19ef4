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

// 3D: a block owns a kEX x kLY column tile and marches up through a chunk
// of z planes.  The five planes k - 2 .. k + 2 of E and of each velocity
// component of its own column stay in registers (the z derivatives), and
// plane k of the tile with a two-cell ring (ghost mapped) is staged in LDS
// for the x and y derivatives: per cell and plane a few coalesced loads
// instead of the four neighbours of each field.  The tiles of one XCD are
// contiguous, so the ring rows shared with neighbouring tiles meet in its
// L2.  Same operations, in the same order, as k_explicit.
constexpr int kLY = 8, kLT = kEX * kLY;          // tile rows, threads
constexpr int kLRX = kEX + 4, kLRY = kLY + 4;    // staged: tile + ring
constexpr int kLSlots = kLRX * kLRY;

template <bool HAS_V>
__global__ void __launch_bounds__(kLT)
    k_explicit_3d(ExplicitArgs A, int zc, int group) {
  constexpr int NF = HAS_V ? 4 : 1;  // E, then v_0 .. v_2
  __shared__ double S[NF][kLSlots];
  const Geom& g = A.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int gx = (nx + kEX - 1) / kEX, gy = (ny + kLY - 1) / kLY;
  const int nb = gridDim.x, b = blockIdx.x;
  const int tile = group ? (b % 8) * (nb / 8) + b / 8 : b;
  const int tx = threadIdx.x % kEX, ty = threadIdx.x / kEX;
  const int x0 = (tile % gx) * kEX, y0 = ((tile / gx) % gy) * kLY;
  const int x = x0 + tx, y = y0 + ty;
  const int z0 = (tile / (gx * gy)) * zc, z1 = min(z0 + zc, nz);
  if (z0 >= nz) return;  // whole block
  const bool in = x < nx && y < ny;
  const int64_t sz = (int64_t)nx * ny;
  const int64_t col = (int64_t)min(y, ny - 1) * nx + min(x, nx - 1);
  const double* F[4] = {A.E, A.v[0], A.v[1], A.v[2]};
  // staged slots of this thread (ghost-mapped in-plane offsets).  A slot
  // more than two cells past the level's edge (a ragged tile) is read by no
  // cell inside: its coordinate is clamped into the ghost range first, so
  // its load stays inside the level.
  constexpr int kPer = (kLSlots + kLT - 1) / kLT;
  int64_t so[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int i = min((int)threadIdx.x + j * kLT, kLSlots - 1);
    const int sx = min(x0 - 2 + i % kLRX, nx + 1);
    const int sy = min(y0 - 2 + i / kLRX, ny + 1);
    so[j] = (int64_t)ghost(sy, ny, g.per[1]) * nx + ghost(sx, nx, g.per[0]);
  }
  auto zoff = [&](int k) { return (int64_t)ghost(k, nz, g.per[2]) * sz; };
  double w[NF][5];  // w[f][j]: field f at plane k - 2 + j, own column
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int j = 0; j < 4; ++j) w[f][j] = F[f][zoff(z0 - 2 + j) + col];
  const int me = (ty + 2) * kLRX + tx + 2;
  for (int k = z0; k < z1; ++k) {
    const int64_t pk = (int64_t)k * sz;
    const int64_t p2 = zoff(k + 2) + col;
#pragma unroll
    for (int f = 0; f < NF; ++f) w[f][4] = F[f][p2];
    // stage plane k of the tile and its ring
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int i = threadIdx.x + j * kLT;
      if (i < kLSlots)
#pragma unroll
        for (int f = 0; f < NF; ++f) S[f][i] = F[f][pk + so[j]];
    }
    __syncthreads();
    if (in) {
      const int64_t idx = pk + col;
      // grad of field f along d at this cell (five-point stencil)
      auto grad = [&](int f, int d) {
        if (d == 2)
          return (w[f][0] - 8.0 * w[f][1] + 8.0 * w[f][3] - w[f][4]) *
                 A.gscale[2];
        const int st = d == 0 ? 1 : kLRX;
        const double* s = S[f];
        return (s[me - 2 * st] - 8.0 * s[me - st] + 8.0 * s[me + st] -
                s[me + 2 * st]) * A.gscale[d];
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
        A.tiring[idx] =
            E0 * (0.5 * (1.0 - fe) * div + 0.5 * (3.0 * fe - 1.0) * nn);
      }
    }
    __syncthreads();  // the staged plane is read; the next one overwrites it
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int j = 0; j < 4; ++j) w[f][j] = w[f][j + 1];
  }
}

hipError_t launch_explicit(const ExplicitArgs& a, hipStream_t s) {
  if (a.g.N == 0) return hipSuccess;
  if (a.g.ndim == 3) {
    // about 2048 blocks (z chunks of at least 8 planes; on 256^3 with every
    // output 453 us whether 1024, 2048, 4096 or 8192 blocks: 1.6 GB
    // algorithmic, 2.3 GB measured, 0.44 of 8 TB/s; the register-window
    // kernel without the staged plane took 748 us, one thread per cell 880)
    const int tiles = ((a.g.n[0] + kEX - 1) / kEX) * ((a.g.n[1] + kLY - 1) / kLY);
    const int chunks = std::max(1, std::min(a.g.n[2], 2048 / std::max(tiles, 1)));
    const int zc = std::max(std::min(8, a.g.n[2]), (a.g.n[2] + chunks - 1) / chunks);
    const int nb = tiles * ((a.g.n[2] + zc - 1) / zc);
    const int group = nb % 8 == 0;
    if (a.v[0])
      hipLaunchKernelGGL(k_explicit_3d<true>, dim3(nb), dim3(kLT), 0, s, a, zc,
                         group);
    else
      hipLaunchKernelGGL(k_explicit_3d<false>, dim3(nb), dim3(kLT), 0, s, a,
                         zc, group);
    return hipGetLastError();
  }
  const dim3 grid((a.g.n[0] + kEX - 1) / kEX, (a.g.n[1] + kEY - 1) / kEY,
                  a.g.n[2]);
  hipLaunchKernelGGL(k_explicit, grid, dim3(kEX * kEY), 0, s, a);
  return hipGetLastError();
}

}  // namespace fld
