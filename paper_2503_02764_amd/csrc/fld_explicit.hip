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
// kappa once, and each requested output written once.  Expanding
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

__global__ void __launch_bounds__(kBlock) k_explicit(ExplicitArgs A) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= A.g.N) return;
  int c[3];
  coords(A.g, idx, c);
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
  hipLaunchKernelGGL(k_explicit, dim3(blocks_for(a.g.N)), dim3(kBlock), 0, s,
                     a);
  return hipGetLastError();
}

}  // namespace fld
