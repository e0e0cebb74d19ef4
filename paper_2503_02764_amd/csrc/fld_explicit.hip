// Explicit FLD source terms around the implicit radiation update (Sect. 3
// adds them explicitly): the radiation force density f_r = -lambda grad E
// (eq. rad_force with the flux of eq. fld_F), its work v . f_r, and photon
// tiring P : grad v with P = f E (eq. fld_P), the Eddington tensor of
// eq. fld_Eddington_tensor and the Eddington factor f = lambda + lambda^2 R^2
// (eq. fld_f).  grad E and grad v by the five-point fourth-order stencil of
// the coefficient stage, with its ghost mapping (periodic wrap, Neumann
// mirror ghosts) for E and every velocity component; R and lambda as there.
//
// One thread per cell, one pass: E and the velocity components are read
// with their stencil neighbours (cache hits after the first touch), rho and
// kappa once, and each requested output written once.  The cell's
// coordinates come from the launch grid, not from index divisions.  Expanding
//   P : grad v = E [ (1 - f)/2 div v + (3 f - 1)/2 n . (grad v) . n ]
// keeps the Eddington tensor implicit: no 3 x 3 array per thread.
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

hipError_t launch_explicit(const ExplicitArgs& a, hipStream_t s) {
  if (a.g.N == 0) return hipSuccess;
  const dim3 grid((a.g.n[0] + kEX - 1) / kEX, (a.g.n[1] + kEY - 1) / kEY,
                  a.g.n[2]);
  hipLaunchKernelGGL(k_explicit, grid, dim3(kEX * kEY), 0, s, a);
  return hipGetLastError();
}

}  // namespace fld
