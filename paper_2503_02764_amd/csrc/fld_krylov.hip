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
// the (p, q), (p, r) pair), which a single-block kernel reduces.  The
// stencil passes (r = b - A x, q = A p) are specialised on the dimension
// count and take the neighbour indices of a cell before any load, without
// branches, and handle two rows per iteration: all loads of both cells then
// issue together instead of one dimension's round trip after another.
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

// The cell of row `row` (rows run over y, then z), column xc, with its
// neighbours.
template <int ND>
__device__ __forceinline__ Nbrs<ND> row_cell(const Geom& g, int64_t row,
                                             int xc) {
  int c[3] = {xc, 0, 0};
  if (ND == 2) c[1] = (int)row;
  if (ND == 3) {
    const uint32_t r = (uint32_t)row, n1 = (uint32_t)g.n[1];
    c[1] = (int)(r % n1);
    c[2] = (int)(r / n1);
  }
  return neighbours<ND>(g, c, row * g.n[0] + xc);
}

// (A v)_i with v = z + beta p_old (FIRST: v = z) at the cell and its
// neighbours; returns A v, sets vi.  Same operation order as the V-cycle's
// residual.
template <int ND, bool FIRST, typename TZ>
__device__ __forceinline__ double apply_dir(const KrylovArgs& K,
                                            const TZ* __restrict__ z,
                                            const double* __restrict__ po,
                                            double beta, const Nbrs<ND>& n,
                                            double& vi) {
  double zl[ND], zu[ND], pl[ND], pu[ND], al[ND], au[ND];
  const double zc = load_z(z, n.idx);
  const double pc = FIRST ? 0.0 : po[n.idx];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    zl[d] = load_z(z, n.lo[d]);
    zu[d] = load_z(z, n.up[d]);
    if (!FIRST) {
      pl[d] = po[n.lo[d]];
      pu[d] = po[n.up[d]];
    }
    al[d] = K.a[d][n.lo[d]];
    au[d] = K.a[d][n.idx];
  }
  vi = FIRST ? zc : zc + beta * pc;
  double av = vi;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const double vl = FIRST ? zl[d] : zl[d] + beta * pl[d];
    const double vu = FIRST ? zu[d] : zu[d] + beta * pu[d];
    const double a_l = n.lo_face[d] ? al[d] : 0.0;
    av += a_l * (vi - vl) + au[d] * (vi - vu);
  }
  return av;
}

}  // namespace

// r = b - A x (and its FP32 copy), partials of |r|^2
template <int ND>
__global__ void __launch_bounds__(kKBlock)
    k_fcg_init(KrylovArgs K, const double* __restrict__ x,
               const double* __restrict__ b) {
  __shared__ double sh[kKBlock / 64];
  if (K.ctrl->done != kRunning) return;
  const Geom& g = K.g;
  double* __restrict__ r = K.r;
  float* __restrict__ r32 = K.r32;
  const int64_t rows = (int64_t)g.n[1] * g.n[2];
  double s = 0.0;
  int64_t rb, re;
  row_range(rows, rb, re);
  for (int64_t row = rb; row < re; row += 2) {
    const bool two = row + 1 < re;
    const int64_t row1 = two ? row + 1 : row;
    for (int xc = threadIdx.x; xc < g.n[0]; xc += kKBlock) {
      const Nbrs<ND> n0 = row_cell<ND>(g, row, xc);
      const Nbrs<ND> n1 = row_cell<ND>(g, row1, xc);
      const double v0 = residual_nb<ND>(K.a, x, b, n0);
      const double v1 = residual_nb<ND>(K.a, x, b, n1);
      r[n0.idx] = v0;
      if (r32) r32[n0.idx] = (float)v0;
      s += v0 * v0;
      if (two) {
        r[n1.idx] = v1;
        if (r32) r32[n1.idx] = (float)v1;
        s += v1 * v1;
      }
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
  const double* __restrict__ q = K.q;
  const int64_t rows = (int64_t)g.n[1] * g.n[2];
  double s = 0.0;
  int64_t rb, re;
  row_range(rows, rb, re);
  const int64_t i1 = re * g.n[0];
#pragma unroll 4
  for (int64_t i = rb * g.n[0] + threadIdx.x; i < i1; i += kKBlock)
    s += load_z(z, i) * q[i];
  const double t = block_sum<kKBlock>(s, sh);
  if (threadIdx.x == 0) K.partials[blockIdx.x] = t;
}

// p = z + beta p_old, q = A p; partials of (p, q) and (p, r)
template <int ND, bool FIRST, typename TZ>
__global__ void __launch_bounds__(kKBlock)
    k_fcg_dir(KrylovArgs K, const TZ* __restrict__ z) {
  __shared__ double sh[kKBlock / 64];
  if (K.ctrl->done != kRunning) return;
  const double beta = FIRST ? 0.0 : K.ctrl->fcg_beta;
  const double* __restrict__ po = K.p_old;
  const double* __restrict__ r = K.r;
  double* __restrict__ pn = K.p_new;
  double* __restrict__ q = K.q;
  const Geom& g = K.g;
  const int64_t rows = (int64_t)g.n[1] * g.n[2];
  double spq = 0.0, spr = 0.0;
  int64_t rb, re;
  row_range(rows, rb, re);
  for (int64_t row = rb; row < re; row += 2) {
    const bool two = row + 1 < re;
    const int64_t row1 = two ? row + 1 : row;
    for (int xc = threadIdx.x; xc < g.n[0]; xc += kKBlock) {
      const Nbrs<ND> n0 = row_cell<ND>(g, row, xc);
      const Nbrs<ND> n1 = row_cell<ND>(g, row1, xc);
      double p0, p1;
      const double q0 = apply_dir<ND, FIRST>(K, z, po, beta, n0, p0);
      const double q1 = apply_dir<ND, FIRST>(K, z, po, beta, n1, p1);
      const double r0 = r[n0.idx], r1 = r[n1.idx];
      pn[n0.idx] = p0;
      q[n0.idx] = q0;
      spq += p0 * q0;
      spr += p0 * r0;
      if (two) {
        pn[n1.idx] = p1;
        q[n1.idx] = q1;
        spq += p1 * q1;
        spr += p1 * r1;
      }
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

// x += alpha p, r -= alpha q (and its FP32 copy); partials of |r|^2.
// Each thread takes kUpd cells per iteration, all loads before any store
// (a store would otherwise order the next cell's loads behind it).
constexpr int kUpd = 4;

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
  const int64_t i0 = rb * g.n[0], i1 = re * g.n[0];
  for (int64_t base = i0 + threadIdx.x; base < i1; base += kUpd * kKBlock) {
    int64_t idx[kUpd];
    double xv[kUpd], pv[kUpd], rv[kUpd], qv[kUpd];
#pragma unroll
    for (int u = 0; u < kUpd; ++u) {
      const int64_t i = base + (int64_t)u * kKBlock;
      idx[u] = i < i1 ? i : base;  // past the end: reload the first cell
      xv[u] = x[idx[u]];
      pv[u] = K.p_new[idx[u]];
      rv[u] = K.r[idx[u]];
      qv[u] = K.q[idx[u]];
    }
#pragma unroll
    for (int u = 0; u < kUpd; ++u) {
      if (base + (int64_t)u * kKBlock >= i1) break;
      const double ri = rv[u] - alpha * qv[u];
      x[idx[u]] = xv[u] + alpha * pv[u];
      K.r[idx[u]] = ri;
      if (K.r32) K.r32[idx[u]] = (float)ri;
      s += ri * ri;
    }
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
  const dim3 grid(krylov_blocks(K.g)), block(kKBlock);
  if (K.g.ndim == 3)
    hipLaunchKernelGGL(k_fcg_init<3>, grid, block, 0, s, K, x, b);
  else if (K.g.ndim == 2)
    hipLaunchKernelGGL(k_fcg_init<2>, grid, block, 0, s, K, x, b);
  else
    hipLaunchKernelGGL(k_fcg_init<1>, grid, block, 0, s, K, x, b);
  return hipGetLastError();
}

template <typename TZ>
hipError_t launch_fcg_zq(const KrylovArgs& K, const TZ* z, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_zq<TZ>, dim3(krylov_blocks(K.g)), dim3(kKBlock), 0,
                     s, K, z);
  return hipGetLastError();
}

template <int ND, typename TZ>
static void dir_nd(const KrylovArgs& K, const TZ* z, int first, hipStream_t s) {
  const dim3 grid(krylov_blocks(K.g)), block(kKBlock);
  if (first)
    hipLaunchKernelGGL((k_fcg_dir<ND, true, TZ>), grid, block, 0, s, K, z);
  else
    hipLaunchKernelGGL((k_fcg_dir<ND, false, TZ>), grid, block, 0, s, K, z);
}

template <typename TZ>
hipError_t launch_fcg_dir(const KrylovArgs& K, const TZ* z, int first,
                          hipStream_t s) {
  if (K.g.ndim == 3)
    dir_nd<3>(K, z, first, s);
  else if (K.g.ndim == 2)
    dir_nd<2>(K, z, first, s);
  else
    dir_nd<1>(K, z, first, s);
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
