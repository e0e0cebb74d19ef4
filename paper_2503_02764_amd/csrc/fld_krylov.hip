// Flexible conjugate gradients (FCG with one direction kept, Notay 2000)
// around the multigrid V-cycle: the Krylov form of the solve of
// (I + dt L) E* = E^n (eq. mhd_r_e's diffusion part; Sect. 3 solves it by
// multigrid).
//
// With a V-cycle M as preconditioner, each iteration k does
//   z   = M(r)                                  (V-cycle(s) from zero)
//   beta = -(z, q_old) / (p_old, q_old)         (k > 0; 0 at k = 0)
//   p   = z + beta p_old,  q = A p
//   alpha = (p, r) / (p, q)
//   x  += alpha p,  r -= alpha q,  stop when |r| / |b| <= rtol.
// The V-cycle alone overshoots where the face coefficients span many
// decades (the coarse operators are rediscretised, not Galerkin products),
// and a fixed-point iteration on it can then diverge; as a preconditioner
// of CG it cannot: the direction is re-weighted by the exact A every
// iteration.  The "flexible" beta tolerates a preconditioner that is not
// exactly symmetric or constant (red-black smoothing in the same colour
// order on both sides; FP32 V-cycles).
//
// Kernels walk rows (x fastest), each block a fixed contiguous run of them
// (row_range), so every block sums its cells in a fixed order and the dot
// products are deterministic; each writes one partial per block (two for
// the (p, q), (p, r) pair), which a single-block kernel reduces.
#include "fld_internal.h"
#include "fld_device.h"

namespace fld {

namespace {

constexpr int kKBlock = 256;

// Rows [r0, r1) of block b: every block takes a contiguous run of rows, and
// consecutive runs go to blocks that the hardware places on the same XCD
// (blocks are dealt round-robin over the 8 XCDs), so the rows above and
// below a run (stencil neighbours along y and z) mostly sit in the same
// XCD's L2.
__device__ __forceinline__ void row_range(int64_t rows, int64_t& r0,
                                          int64_t& r1) {
  const int nb = gridDim.x, b = blockIdx.x;
  const int c = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int64_t per = (rows + nb - 1) / nb;
  r0 = (int64_t)c * per;
  r1 = r0 + per < rows ? r0 + per : rows;
}

__device__ __forceinline__ double load_z(const double* z, int64_t i) {
  return z[i];
}
__device__ __forceinline__ double load_z(const float* z, int64_t i) {
  return (double)z[i];
}

// (A v)_i for v = z + beta p_old computed at the cell and its neighbours
// (p_old null: v = z, the first direction)
template <typename TZ>
__device__ __forceinline__ double apply_dir(const KrylovArgs& K, const TZ* z,
                                            const double* po, double beta,
                                            const int c[3], int64_t idx,
                                            double& vi) {
  const Geom& g = K.g;
  vi = po ? load_z(z, idx) + beta * po[idx] : load_z(z, idx);
  double av = vi;
  for (int d = 0; d < g.ndim; ++d) {
    const int64_t st = stride_of(g, d);
    int64_t nl, nu;
    double al, au;
    lower_nb(g, K.a[d], d, c[d], idx, st, nl, al);
    upper_nb(g, K.a[d], d, c[d], idx, st, nu, au);
    const double vl = po ? load_z(z, nl) + beta * po[nl] : load_z(z, nl);
    const double vu = po ? load_z(z, nu) + beta * po[nu] : load_z(z, nu);
    av += al * (vi - vl) + au * (vi - vu);
  }
  return av;
}

}  // namespace

// r = b - A x (and its FP32 copy), partials of |r|^2
__global__ void __launch_bounds__(kKBlock)
    k_fcg_init(KrylovArgs K, const double* __restrict__ x,
               const double* __restrict__ b) {
  __shared__ double sh[kKBlock / 64];
  if (K.ctrl->done != kRunning) return;
  const Geom& g = K.g;
  const int64_t rows = (int64_t)g.n[1] * g.n[2];
  double s = 0.0;
  int64_t rb, re;
  row_range(rows, rb, re);
  for (int64_t row = rb; row < re; ++row) {
    const int y = (int)(row % g.n[1]), zc = (int)(row / g.n[1]);
    for (int xc = threadIdx.x; xc < g.n[0]; xc += kKBlock) {
      const int c[3] = {xc, y, zc};
      const int64_t idx = row * g.n[0] + xc;
      const double xi = x[idx];
      double ax = xi;
      for (int d = 0; d < g.ndim; ++d) {
        const int64_t st = stride_of(g, d);
        int64_t nl, nu;
        double al, au;
        lower_nb(g, K.a[d], d, c[d], idx, st, nl, al);
        upper_nb(g, K.a[d], d, c[d], idx, st, nu, au);
        ax += al * (xi - x[nl]) + au * (xi - x[nu]);
      }
      const double r = b[idx] - ax;
      K.r[idx] = r;
      if (K.r32) K.r32[idx] = (float)r;
      s += r * r;
    }
  }
  const double t = block_sum<kKBlock>(s, sh);
  if (threadIdx.x == 0) K.partials[blockIdx.x] = t;
}

// partials of (z, q_old)
template <typename TZ>
__global__ void __launch_bounds__(kKBlock)
    k_fcg_zq(KrylovArgs K, const TZ* __restrict__ z) {
  __shared__ double sh[kKBlock / 64];
  if (K.ctrl->done != kRunning) return;
  const Geom& g = K.g;
  const int64_t rows = (int64_t)g.n[1] * g.n[2];
  double s = 0.0;
  int64_t rb, re;
  row_range(rows, rb, re);
  for (int64_t row = rb; row < re; ++row)
    for (int xc = threadIdx.x; xc < g.n[0]; xc += kKBlock) {
      const int64_t idx = row * g.n[0] + xc;
      s += load_z(z, idx) * K.q[idx];
    }
  const double t = block_sum<kKBlock>(s, sh);
  if (threadIdx.x == 0) K.partials[blockIdx.x] = t;
}

// p = z + beta p_old, q = A p; partials of (p, q) and (p, r)
template <typename TZ>
__global__ void __launch_bounds__(kKBlock)
    k_fcg_dir(KrylovArgs K, const TZ* __restrict__ z, int first) {
  __shared__ double sh[kKBlock / 64];
  if (K.ctrl->done != kRunning) return;
  const double beta = first ? 0.0 : K.ctrl->fcg_beta;
  const double* po = first ? nullptr : K.p_old;
  const Geom& g = K.g;
  const int64_t rows = (int64_t)g.n[1] * g.n[2];
  double spq = 0.0, spr = 0.0;
  int64_t rb, re;
  row_range(rows, rb, re);
  for (int64_t row = rb; row < re; ++row) {
    const int y = (int)(row % g.n[1]), zc = (int)(row / g.n[1]);
    for (int xc = threadIdx.x; xc < g.n[0]; xc += kKBlock) {
      const int c[3] = {xc, y, zc};
      const int64_t idx = row * g.n[0] + xc;
      double pi;
      const double qi = apply_dir(K, z, po, beta, c, idx, pi);
      K.p_new[idx] = pi;
      K.q[idx] = qi;
      spq += pi * qi;
      spr += pi * K.r[idx];
    }
  }
  const double t1 = block_sum<kKBlock>(spq, sh);
  __syncthreads();
  const double t2 = block_sum<kKBlock>(spr, sh);
  if (threadIdx.x == 0) {
    K.partials[blockIdx.x] = t1;
    K.partials[gridDim.x + blockIdx.x] = t2;
  }
}

// x += alpha p, r -= alpha q (and its FP32 copy); partials of |r|^2
__global__ void __launch_bounds__(kKBlock)
    k_fcg_update(KrylovArgs K, double* __restrict__ x) {
  __shared__ double sh[kKBlock / 64];
  if (K.ctrl->done != kRunning) return;
  const double alpha = K.ctrl->fcg_alpha;
  const Geom& g = K.g;
  const int64_t rows = (int64_t)g.n[1] * g.n[2];
  double s = 0.0;
  int64_t rb, re;
  row_range(rows, rb, re);
  for (int64_t row = rb; row < re; ++row)
    for (int xc = threadIdx.x; xc < g.n[0]; xc += kKBlock) {
      const int64_t idx = row * g.n[0] + xc;
      x[idx] += alpha * K.p_new[idx];
      const double r = K.r[idx] - alpha * K.q[idx];
      K.r[idx] = r;
      if (K.r32) K.r32[idx] = (float)r;
      s += r * r;
    }
  const double t = block_sum<kKBlock>(s, sh);
  if (threadIdx.x == 0) K.partials[blockIdx.x] = t;
}

// Single-block scalars: mode 0 beta = -(z, q_old) / (p_old, q_old);
// mode 1 alpha = (p, r) / (p, q), keeping (p, q) for the next beta.  A
// direction with (p, q) <= 0 or a non-finite scalar stops the solve
// (reported as the cycle cap: the last iterate is returned).
__global__ void __launch_bounds__(kReduceBlock)
    k_fcg_scalar(int mode, const double* __restrict__ partials, int count,
                 Control* ctrl) {
  __shared__ double sh[kReduceBlock / 64];
  if (ctrl->done != kRunning) return;
  double v1 = 0.0, v2 = 0.0;
  for (int i = threadIdx.x; i < count; i += kReduceBlock) {
    v1 += partials[i];
    if (mode == 1) v2 += partials[count + i];
  }
  const double s1 = block_sum<kReduceBlock>(v1, sh);
  __syncthreads();
  const double s2 = mode == 1 ? block_sum<kReduceBlock>(v2, sh) : 0.0;
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    const double beta = -s1 / ctrl->fcg_pq;
    if (isfinite(beta)) {
      ctrl->fcg_beta = beta;
    } else {
      ctrl->done = kCapped;
    }
  } else {
    const double alpha = s2 / s1;
    if (s1 > 0.0 && isfinite(alpha)) {
      ctrl->fcg_alpha = alpha;
      ctrl->fcg_pq = s1;
    } else {
      ctrl->done = kCapped;
    }
  }
  if (ctrl->done != kRunning && ctrl->mirror) *ctrl->mirror = *ctrl;
}

int krylov_blocks(const Geom& g) {
  const int64_t rows = (int64_t)g.n[1] * g.n[2];
  return (int)std::min<int64_t>(rows, kKrylovBlocks);
}

hipError_t launch_fcg_init(const KrylovArgs& K, const double* x,
                           const double* b, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_init, dim3(krylov_blocks(K.g)), dim3(kKBlock), 0, s,
                     K, x, b);
  return hipGetLastError();
}

template <typename TZ>
hipError_t launch_fcg_zq(const KrylovArgs& K, const TZ* z, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_zq<TZ>, dim3(krylov_blocks(K.g)), dim3(kKBlock), 0,
                     s, K, z);
  return hipGetLastError();
}

template <typename TZ>
hipError_t launch_fcg_dir(const KrylovArgs& K, const TZ* z, int first,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_dir<TZ>, dim3(krylov_blocks(K.g)), dim3(kKBlock), 0,
                     s, K, z, first);
  return hipGetLastError();
}

hipError_t launch_fcg_update(const KrylovArgs& K, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_update, dim3(krylov_blocks(K.g)), dim3(kKBlock), 0,
                     s, K, x);
  return hipGetLastError();
}

hipError_t launch_fcg_scalar(int mode, const KrylovArgs& K, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_scalar, dim3(1), dim3(kReduceBlock), 0, s, mode,
                     (const double*)K.partials, krylov_blocks(K.g), K.ctrl);
  return hipGetLastError();
}

template hipError_t launch_fcg_zq<double>(const KrylovArgs&, const double*,
                                          hipStream_t);
template hipError_t launch_fcg_zq<float>(const KrylovArgs&, const float*,
                                         hipStream_t);
template hipError_t launch_fcg_dir<double>(const KrylovArgs&, const double*,
                                           int, hipStream_t);
template hipError_t launch_fcg_dir<float>(const KrylovArgs&, const float*, int,
                                          hipStream_t);

}  // namespace fld
