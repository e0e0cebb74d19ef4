// HIP kernels of the FLD radiation-energy update for gfx950 (wave64).
//
// Coefficient stage (Sect. 2, eqs. fld_F, fld_lambda, fld_R; gradient by the
// five-point stencil of Sect. 3), the backward-Euler diffusion multigrid
// (Sect. 3 solves div F with geometric multigrid) and the implicit
// gas-radiation exchange quartic (eqs. heating, qdot; Sect. 3).
//
// Every kernel here is memory-bound (well under 10 flop/byte).  Reductions
// are deterministic: a fixed wave-level shuffle tree, then a fixed loop over
// the waves of a block, then one single-block pass over the block partials.
#include "fld_internal.h"

#include <math.h>

namespace fld {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ void coords(const Geom& g, int64_t idx, int c[3]) {
  c[0] = (int)(idx % g.n[0]);
  int64_t t = idx / g.n[0];
  c[1] = (int)(t % g.n[1]);
  c[2] = (int)(t / g.n[1]);
}

__device__ __forceinline__ int64_t stride_of(const Geom& g, int d) {
  return d == 0 ? 1 : (d == 1 ? (int64_t)g.n[0] : (int64_t)g.n[0] * g.n[1]);
}

// Ghost mapping of the coefficient stage: periodic wrap, or mirror ghosts
// (E[-1] = E[0], E[-2] = E[1]; E[n] = E[n-1], E[n+1] = E[n-2]).
__device__ __forceinline__ int ghost(int m, int n, int per) {
  if (per) {
    m %= n;
    return m < 0 ? m + n : m;
  }
  if (m < 0) return -m - 1;
  if (m >= n) return 2 * n - 1 - m;
  return m;
}

// Sum over a block of kBlockSize threads; the result is valid in thread 0.
template <int kBlockSize>
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kBlockSize / 64; ++q) r += sh[q];
  }
  return r;
}

// Lower (-d) and upper (+d) neighbour of a cell with coordinate cd along d,
// with the coefficient of the face between them (0 at a Neumann wall, where
// the "neighbour" is the cell itself and never contributes).
template <typename T>
__device__ __forceinline__ void lower_nb(const Geom& g, const T* a, int d,
                                         int cd, int64_t idx, int64_t st,
                                         int64_t& nb, T& al) {
  if (cd > 0) {
    nb = idx - st;
    al = a[nb];
  } else if (g.per[d]) {
    nb = idx + (int64_t)(g.n[d] - 1) * st;
    al = a[nb];
  } else {
    nb = idx;
    al = T(0);
  }
}

template <typename T>
__device__ __forceinline__ void upper_nb(const Geom& g, const T* a, int d,
                                         int cd, int64_t idx, int64_t st,
                                         int64_t& nb, T& al) {
  al = a[idx];
  if (cd < g.n[d] - 1)
    nb = idx + st;
  else if (g.per[d])
    nb = idx - (int64_t)(g.n[d] - 1) * st;
  else
    nb = idx;  // wall: al == 0
}

// Gauss-Seidel / Jacobi value of cell idx: (b + sum alpha x_nb) / (1 + sum alpha),
// faces taken in the order -x, +x, -y, +y, -z, +z.
template <typename T>
__device__ __forceinline__ T relax_value(const LevelView<T>& L, const int c[3],
                                         int64_t idx, const T* xs) {
  T num = L.b[idx], den = T(1);
  for (int d = 0; d < L.g.ndim; ++d) {
    const int64_t st = stride_of(L.g, d);
    int64_t nl, nu;
    T al, au;
    lower_nb(L.g, L.a[d], d, c[d], idx, st, nl, al);
    upper_nb(L.g, L.a[d], d, c[d], idx, st, nu, au);
    num += al * xs[nl] + au * xs[nu];
    den += al + au;
  }
  return num / den;
}

// r = b - A x at cell idx.
template <typename T>
__device__ __forceinline__ T residual_value(const LevelView<T>& L,
                                            const int c[3], int64_t idx) {
  const T xi = L.x[idx];
  T ax = xi;
  for (int d = 0; d < L.g.ndim; ++d) {
    const int64_t st = stride_of(L.g, d);
    int64_t nl, nu;
    T al, au;
    lower_nb(L.g, L.a[d], d, c[d], idx, st, nl, al);
    upper_nb(L.g, L.a[d], d, c[d], idx, st, nu, au);
    ax += al * (xi - L.x[nl]) + au * (xi - L.x[nu]);
  }
  return L.b[idx] - ax;
}

// ---------------------------------------------------------------------------
// control block
// ---------------------------------------------------------------------------

__global__ void k_ctrl_init(Control* ctrl, double rtol, int max_cycles) {
  if (threadIdx.x == 0) {
    ctrl->bnorm2 = 0.0;
    ctrl->res_initial = 0.0;
    ctrl->res = 0.0;
    ctrl->rtol = rtol;
    ctrl->done = kRunning;
    ctrl->cycles = 0;
    ctrl->max_cycles = max_cycles;
    ctrl->flagged = 0;
  }
}

hipError_t launch_ctrl_init(Control* ctrl, double rtol, int max_cycles,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, s, ctrl, rtol,
                     max_cycles);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
    k_fill(double* __restrict__ x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = v;
}

hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, x, n, v);
  return hipGetLastError();
}

// Single-block reduction of the block partials and the stop decision.
__global__ void __launch_bounds__(kReduceBlock)
    k_finalize(int mode, const double* __restrict__ partials, int count,
               Control* ctrl) {
  __shared__ double sh[kReduceBlock / 64];
  const int done = ctrl->done;
  if (mode != kFinBnorm && done != kRunning) return;
  double v = 0.0;
  for (int i = threadIdx.x; i < count; i += kReduceBlock) v += partials[i];
  const double s = block_sum<kReduceBlock>(v, sh);
  if (threadIdx.x != 0) return;
  if (mode == kFinBnorm) {
    ctrl->bnorm2 = s;
    if (ctrl->flagged > 0 || !(s > 0.0)) ctrl->done = kNonPhysical;
    return;
  }
  const double r = sqrt(s / ctrl->bnorm2);
  ctrl->res = r;
  if (mode == kFinInitial) {
    ctrl->res_initial = r;
    if (r <= ctrl->rtol) ctrl->done = kConverged;
    return;
  }
  ctrl->cycles += 1;
  if (r <= ctrl->rtol)
    ctrl->done = kConverged;
  else if (ctrl->cycles >= ctrl->max_cycles)
    ctrl->done = kCapped;
}

hipError_t launch_finalize(int mode, const double* partials, int count,
                           Control* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kReduceBlock), 0, s, mode,
                     partials, count, ctrl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// coefficient stage
// ---------------------------------------------------------------------------

// Cell-centred D = c lambda / (rho kappa), R = |grad E| / (rho kappa E).
__device__ __forceinline__ double cell_D(const CoefArgs& A, const double* E,
                                         const double* rho,
                                         const double* kappa, const int c[3],
                                         int64_t idx, bool& bad) {
  const double E0 = E[idx];
  const double rk = rho[idx] * kappa[idx];
  double g2 = 0.0;
  for (int d = 0; d < A.g.ndim; ++d) {
    const int64_t st = stride_of(A.g, d);
    const int64_t base = idx - (int64_t)c[d] * st;
    const int n = A.g.n[d], p = A.g.per[d];
    const double em2 = E[base + (int64_t)ghost(c[d] - 2, n, p) * st];
    const double em1 = E[base + (int64_t)ghost(c[d] - 1, n, p) * st];
    const double ep1 = E[base + (int64_t)ghost(c[d] + 1, n, p) * st];
    const double ep2 = E[base + (int64_t)ghost(c[d] + 2, n, p) * st];
    const double G = (em2 - 8.0 * em1 + 8.0 * ep1 - ep2) / (12.0 * A.dx[d]);
    g2 += G * G;
  }
  const double R = sqrt(g2) / (rk * E0);
  const double lam =
      A.limiter == 0 ? (2.0 + R) / (6.0 + 3.0 * R + R * R) : 1.0 / 3.0;
  bad = !(E0 > 0.0) || !(rk > 0.0) || !isfinite(E0) || !isfinite(rk);
  return A.c * lam / rk;
}

__global__ void __launch_bounds__(kBlock)
    k_coef(CoefArgs A, const double* __restrict__ E,
           const double* __restrict__ rho, const double* __restrict__ kappa,
           double* __restrict__ a0, double* __restrict__ a1,
           double* __restrict__ a2, double* __restrict__ copy_dst,
           double* __restrict__ partials, Control* ctrl) {
  __shared__ double sh[kBlock / 64];
  __shared__ int bad_count;
  if (threadIdx.x == 0) bad_count = 0;
  __syncthreads();
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double e2 = 0.0;
  if (idx < A.g.N) {
    int c[3];
    coords(A.g, idx, c);
    bool bad = false;
    const double D0 = cell_D(A, E, rho, kappa, c, idx, bad);
    double* out[3] = {a0, a1, a2};
    for (int d = 0; d < A.g.ndim; ++d) {
      double alpha = 0.0;
      if (c[d] < A.g.n[d] - 1 || A.g.per[d]) {
        int cn[3] = {c[0], c[1], c[2]};
        cn[d] = (c[d] + 1) % A.g.n[d];
        const int64_t nidx =
            cn[0] + (int64_t)A.g.n[0] * (cn[1] + (int64_t)A.g.n[1] * cn[2]);
        bool bad_n = false;
        const double Dn = cell_D(A, E, rho, kappa, cn, nidx, bad_n);
        const double Df =
            A.face_mean == 0 ? 0.5 * (D0 + Dn) : 2.0 * D0 * Dn / (D0 + Dn);
        alpha = A.dt * Df / (A.dx[d] * A.dx[d]);
      }
      out[d][idx] = alpha;
    }
    const double Ei = E[idx];
    if (copy_dst) copy_dst[idx] = Ei;
    e2 = Ei * Ei;
    if (bad) atomicAdd(&bad_count, 1);
  }
  const double s = block_sum<kBlock>(e2, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = s;
    if (bad_count > 0) atomicAdd(&ctrl->flagged, bad_count);
  }
}

hipError_t launch_coef(const CoefArgs& a, const double* E, const double* rho,
                       const double* kappa, double* alpha0, double* alpha1,
                       double* alpha2, double* copy_dst, double* partials,
                       Control* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_coef, dim3(blocks_for(a.g.N)), dim3(kBlock), 0, s, a,
                     E, rho, kappa, alpha0, alpha1, alpha2, copy_dst, partials,
                     ctrl);
  return hipGetLastError();
}

// Coarse face coefficient = 1/4 of the mean over the 2^(d-1) fine faces that
// make up the coarse face (D averaged over the face, dx doubled).
struct CoarsenArgs {
  Geom f, c;
  const double* fa[3];
  double* ca[3];
};

__global__ void __launch_bounds__(kBlock) k_coarsen(CoarsenArgs A) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= A.c.N) return;
  int c[3];
  coords(A.c, idx, c);
  const int nd = A.c.ndim;
  for (int d = 0; d < nd; ++d) {
    double s = 0.0;
    int cnt = 0;
    // fine cell on the lower side of the coarse face: 2c+1 along d,
    // 2c or 2c+1 across.
    const int o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
    for (int q2 = 0; q2 < o2; ++q2)
      for (int q1 = 0; q1 < o1; ++q1) {
        int f[3] = {2 * c[0], 2 * c[1], 2 * c[2]};
        f[d] += 1;
        // the transverse dimensions of d, in increasing order
        int t1 = (d == 0) ? 1 : 0;
        int t2 = (d == 2) ? 1 : 2;
        if (nd > 1) f[t1] += q1;
        if (nd > 2) f[t2] += q2;
        const int64_t fi =
            f[0] + (int64_t)A.f.n[0] * (f[1] + (int64_t)A.f.n[1] * f[2]);
        s += A.fa[d][fi];
        ++cnt;
      }
    A.ca[d][idx] = 0.25 * s / cnt;
  }
}

hipError_t launch_coarsen(const Geom& fine, const Geom& coarse,
                          const double* const fa[3], double* const ca[3],
                          hipStream_t s) {
  CoarsenArgs A;
  A.f = fine;
  A.c = coarse;
  for (int d = 0; d < 3; ++d) {
    A.fa[d] = fa[d];
    A.ca[d] = ca[d];
  }
  hipLaunchKernelGGL(k_coarsen, dim3(blocks_for(coarse.N)), dim3(kBlock), 0, s,
                     A);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// multigrid
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock)
    k_resid_norm(LevelView<double> L, double* __restrict__ partials,
                 const Control* __restrict__ ctrl) {
  __shared__ double sh[kBlock / 64];
  if (ctrl->done != kRunning) return;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double r2 = 0.0;
  if (idx < L.g.N) {
    int c[3];
    coords(L.g, idx, c);
    const double r = residual_value(L, c, idx);
    r2 = r * r;
  }
  const double s = block_sum<kBlock>(r2, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

hipError_t launch_resid_norm(const LevelView<double>& L, double* partials,
                             int* nblocks, const Control* ctrl,
                             hipStream_t s) {
  *nblocks = blocks_for(L.g.N);
  hipLaunchKernelGGL(k_resid_norm, dim3(*nblocks), dim3(kBlock), 0, s, L,
                     partials, ctrl);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
    k_gs_color(LevelView<double> L, int color,
               const Control* __restrict__ ctrl) {
  if (ctrl->done != kRunning) return;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= L.g.N) return;
  int c[3];
  coords(L.g, idx, c);
  if (((c[0] + c[1] + c[2]) & 1) != color) return;
  L.x[idx] = relax_value(L, c, idx, L.x);
}

hipError_t launch_gs_color(const LevelView<double>& L, int color,
                           const Control* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_gs_color, dim3(blocks_for(L.g.N)), dim3(kBlock), 0, s,
                     L, color, ctrl);
  return hipGetLastError();
}

// Coarse rhs = mean of the 2^d fine residuals; coarse x = 0.  With a
// partials buffer, also the block sums of the fine residual squared.
__global__ void __launch_bounds__(kBlock)
    k_resid_restrict(LevelView<double> F, LevelView<double> C,
                     double* __restrict__ partials,
                     const Control* __restrict__ ctrl) {
  __shared__ double sh[kBlock / 64];
  if (ctrl->done != kRunning) return;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double r2 = 0.0;
  if (idx < C.g.N) {
    int c[3];
    coords(C.g, idx, c);
    const int nd = F.g.ndim;
    const int o0 = 2, o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
    double s = 0.0;
    for (int q2 = 0; q2 < o2; ++q2)
      for (int q1 = 0; q1 < o1; ++q1)
        for (int q0 = 0; q0 < o0; ++q0) {
          int f[3] = {2 * c[0] + q0, nd > 1 ? 2 * c[1] + q1 : 0,
                      nd > 2 ? 2 * c[2] + q2 : 0};
          const int64_t fi =
              f[0] + (int64_t)F.g.n[0] * (f[1] + (int64_t)F.g.n[1] * f[2]);
          const double r = residual_value(F, f, fi);
          s += r;
          r2 += r * r;
        }
    C.b[idx] = s / (double)(o0 * o1 * o2);
    C.x[idx] = 0.0;
  }
  if (partials) {
    const double t = block_sum<kBlock>(r2, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
  }
}

hipError_t launch_resid_restrict(const LevelView<double>& fine,
                                 const LevelView<double>& coarse,
                                 double* partials, int* nblocks,
                                 const Control* ctrl, hipStream_t s) {
  *nblocks = blocks_for(coarse.g.N);
  hipLaunchKernelGGL(k_resid_restrict, dim3(*nblocks), dim3(kBlock), 0, s,
                     fine, coarse, partials, ctrl);
  return hipGetLastError();
}

// x_fine += P e_coarse, cell-centred (bi/tri)linear interpolation: weight
// 3/4 on the parent and 1/4 on the next coarse cell on the child's side,
// per dimension; mirror (Neumann) or wrapped (periodic) coarse ghosts.
__global__ void __launch_bounds__(kBlock)
    k_prolong(LevelView<double> C, LevelView<double> F,
              const Control* __restrict__ ctrl) {
  if (ctrl->done != kRunning) return;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= F.g.N) return;
  int f[3];
  coords(F.g, idx, f);
  const int nd = F.g.ndim;
  int p[3], q[3];
  for (int d = 0; d < 3; ++d) {
    if (d < nd) {
      p[d] = f[d] >> 1;
      int o = (f[d] & 1) ? p[d] + 1 : p[d] - 1;
      const int nc = C.g.n[d];
      if (o < 0) o = C.g.per[d] ? nc - 1 : 0;
      if (o >= nc) o = C.g.per[d] ? 0 : nc - 1;
      q[d] = o;
    } else {
      p[d] = 0;
      q[d] = 0;
    }
  }
  const int o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
  double e = 0.0;
  for (int s2 = 0; s2 < o2; ++s2)
    for (int s1 = 0; s1 < o1; ++s1)
      for (int s0 = 0; s0 < 2; ++s0) {
        const int i = s0 ? q[0] : p[0];
        const int j = s1 ? q[1] : p[1];
        const int k = s2 ? q[2] : p[2];
        const double w = (s0 ? 0.25 : 0.75) * (nd > 1 ? (s1 ? 0.25 : 0.75) : 1.0) *
                         (nd > 2 ? (s2 ? 0.25 : 0.75) : 1.0);
        e += w * C.x[i + (int64_t)C.g.n[0] * (j + (int64_t)C.g.n[1] * k)];
      }
  F.x[idx] += e;
}

hipError_t launch_prolong(const LevelView<double>& coarse,
                          const LevelView<double>& fine, const Control* ctrl,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_prolong, dim3(blocks_for(fine.g.N)), dim3(kBlock), 0, s,
                     coarse, fine, ctrl);
  return hipGetLastError();
}

// Coarsest level: Jacobi sweeps in one block until the residual norm has
// dropped by 1e-6 (A = I + L is strictly diagonally dominant, so Jacobi
// converges for any alpha).  tmp holds the next iterate.
__global__ void __launch_bounds__(kReduceBlock)
    k_coarsest(LevelView<double> L, double* __restrict__ tmp,
               const Control* __restrict__ ctrl) {
  __shared__ double sh[kReduceBlock / 64];
  __shared__ double r0, rn;
  if (ctrl->done != kRunning) return;
  const int64_t N = L.g.N;
  for (int it = 0; it < 4000; ++it) {
    if ((it & 7) == 0) {
      double v = 0.0;
      for (int64_t i = threadIdx.x; i < N; i += kReduceBlock) {
        int c[3];
        coords(L.g, i, c);
        const double r = residual_value(L, c, i);
        v += r * r;
      }
      const double s = block_sum<kReduceBlock>(v, sh);
      if (threadIdx.x == 0) {
        if (it == 0) r0 = s;
        rn = s;
      }
      __syncthreads();
      if (!(rn > 1e-12 * r0)) break;
    }
    for (int64_t i = threadIdx.x; i < N; i += kReduceBlock) {
      int c[3];
      coords(L.g, i, c);
      tmp[i] = relax_value(L, c, i, L.x);
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < N; i += kReduceBlock) L.x[i] = tmp[i];
    __syncthreads();
  }
}

hipError_t launch_coarsest(const LevelView<double>& L, double* tmp,
                           const Control* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_coarsest, dim3(1), dim3(kReduceBlock), 0, s, L, tmp,
                     ctrl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// single-workgroup tail of the V-cycle
// ---------------------------------------------------------------------------
//
// Levels small enough for one workgroup (a few thousand cells) are handled
// by one block of kReduceBlock threads with block barriers between phases,
// instead of one launch per phase and level.  With l0 == 0 the whole
// problem fits and the block also runs the cycle loop and the stop test.

__device__ void t_smooth(const LevelView<double>& L, int sweeps) {
  for (int s = 0; s < sweeps; ++s)
    for (int color = 0; color < 2; ++color) {
      for (int64_t i = threadIdx.x; i < L.g.N; i += kReduceBlock) {
        int c[3];
        coords(L.g, i, c);
        if (((c[0] + c[1] + c[2]) & 1) == color)
          L.x[i] = relax_value(L, c, i, L.x);
      }
      __syncthreads();
    }
}

// restriction of the residual; returns this thread's share of sum r^2
__device__ double t_resid_restrict(const LevelView<double>& F,
                                   const LevelView<double>& C) {
  const int nd = F.g.ndim;
  const int o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
  double r2 = 0.0;
  for (int64_t idx = threadIdx.x; idx < C.g.N; idx += kReduceBlock) {
    int c[3];
    coords(C.g, idx, c);
    double s = 0.0;
    for (int q2 = 0; q2 < o2; ++q2)
      for (int q1 = 0; q1 < o1; ++q1)
        for (int q0 = 0; q0 < 2; ++q0) {
          int f[3] = {2 * c[0] + q0, nd > 1 ? 2 * c[1] + q1 : 0,
                      nd > 2 ? 2 * c[2] + q2 : 0};
          const int64_t fi =
              f[0] + (int64_t)F.g.n[0] * (f[1] + (int64_t)F.g.n[1] * f[2]);
          const double r = residual_value(F, f, fi);
          s += r;
          r2 += r * r;
        }
    C.b[idx] = s / (double)(2 * o1 * o2);
    C.x[idx] = 0.0;
  }
  __syncthreads();
  return r2;
}

__device__ void t_prolong(const LevelView<double>& C,
                          const LevelView<double>& F) {
  const int nd = F.g.ndim;
  for (int64_t idx = threadIdx.x; idx < F.g.N; idx += kReduceBlock) {
    int f[3];
    coords(F.g, idx, f);
    int p[3], q[3];
    for (int d = 0; d < 3; ++d) {
      if (d < nd) {
        p[d] = f[d] >> 1;
        int o = (f[d] & 1) ? p[d] + 1 : p[d] - 1;
        const int nc = C.g.n[d];
        if (o < 0) o = C.g.per[d] ? nc - 1 : 0;
        if (o >= nc) o = C.g.per[d] ? 0 : nc - 1;
        q[d] = o;
      } else {
        p[d] = q[d] = 0;
      }
    }
    const int o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
    double e = 0.0;
    for (int s2 = 0; s2 < o2; ++s2)
      for (int s1 = 0; s1 < o1; ++s1)
        for (int s0 = 0; s0 < 2; ++s0) {
          const int i = s0 ? q[0] : p[0];
          const int j = s1 ? q[1] : p[1];
          const int k = s2 ? q[2] : p[2];
          const double w = (s0 ? 0.25 : 0.75) *
                           (nd > 1 ? (s1 ? 0.25 : 0.75) : 1.0) *
                           (nd > 2 ? (s2 ? 0.25 : 0.75) : 1.0);
          e += w * C.x[i + (int64_t)C.g.n[0] * (j + (int64_t)C.g.n[1] * k)];
        }
    F.x[idx] += e;
  }
  __syncthreads();
}

// Jacobi until the residual norm dropped by 1e-6 (or 4000 sweeps).
__device__ void t_coarsest(const LevelView<double>& L, double* tmp,
                           double* sh, double* bc) {
  const int64_t N = L.g.N;
  double r0 = 0.0;
  for (int it = 0; it < 4000; ++it) {
    if ((it & 7) == 0) {
      double v = 0.0;
      for (int64_t i = threadIdx.x; i < N; i += kReduceBlock) {
        int c[3];
        coords(L.g, i, c);
        const double r = residual_value(L, c, i);
        v += r * r;
      }
      const double s = block_sum<kReduceBlock>(v, sh);
      if (threadIdx.x == 0) bc[0] = s;
      __syncthreads();
      const double rn = bc[0];
      __syncthreads();
      if (it == 0) r0 = rn;
      if (!(rn > 1e-12 * r0)) break;
    }
    for (int64_t i = threadIdx.x; i < N; i += kReduceBlock) {
      int c[3];
      coords(L.g, i, c);
      tmp[i] = relax_value(L, c, i, L.x);
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < N; i += kReduceBlock) L.x[i] = tmp[i];
    __syncthreads();
  }
}

// sub-V-cycle from level l0 down to the coarsest and back to l0
__device__ void t_subcycle(const TailArgs& A, int l0, double* sh, double* bc) {
  for (int l = l0; l + 1 < A.L; ++l) {
    t_smooth(A.lv[l], A.pre);
    (void)t_resid_restrict(A.lv[l], A.lv[l + 1]);
  }
  t_coarsest(A.lv[A.L - 1], A.tmp, sh, bc);
  for (int l = A.L - 2; l >= l0; --l) {
    t_prolong(A.lv[l + 1], A.lv[l]);
    t_smooth(A.lv[l], A.post);
  }
}

__global__ void __launch_bounds__(kReduceBlock) k_tail(TailArgs A) {
  __shared__ double sh[kReduceBlock / 64];
  __shared__ double bc[2];
  __shared__ int stop;
  if (A.ctrl->done != kRunning) return;
  if (A.l0 > 0) {
    const LevelView<double>& L = A.lv[A.l0];
    for (int64_t i = threadIdx.x; i < L.g.N; i += kReduceBlock) L.x[i] = 0.0;
    __syncthreads();
    t_subcycle(A, A.l0, sh, bc);
    return;
  }
  // whole problem: cycle loop with the stop test of k_finalize
  for (;;) {
    double r2;
    if (A.L > 1) {
      t_smooth(A.lv[0], A.pre);
      r2 = t_resid_restrict(A.lv[0], A.lv[1]);
    } else {
      t_coarsest(A.lv[0], A.tmp, sh, bc);
      r2 = 0.0;
      for (int64_t i = threadIdx.x; i < A.lv[0].g.N; i += kReduceBlock) {
        int c[3];
        coords(A.lv[0].g, i, c);
        const double r = residual_value(A.lv[0], c, i);
        r2 += r * r;
      }
    }
    const double s = block_sum<kReduceBlock>(r2, sh);
    if (threadIdx.x == 0) {
      Control* C = A.ctrl;
      const double r = sqrt(s / C->bnorm2);
      C->res = r;
      C->cycles += 1;
      if (r <= C->rtol)
        C->done = kConverged;
      else if (C->cycles >= C->max_cycles)
        C->done = kCapped;
      stop = C->done != kRunning;
    }
    __syncthreads();
    if (stop) return;
    if (A.L > 1) {
      t_subcycle(A, 1, sh, bc);
      t_prolong(A.lv[1], A.lv[0]);
      t_smooth(A.lv[0], A.post);
    }
  }
}

hipError_t launch_tail(const TailArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_tail, dim3(1), dim3(kReduceBlock), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exchange and opacity
// ---------------------------------------------------------------------------

// Unique positive root of a4 x^4 + a1 x - c0 (a4 >= 0, a1 > 0, c0 > 0) by
// Newton from the upper bound min(c0/a1, (c0/a4)^(1/4)); on this increasing
// convex function the iterates fall monotonically onto the root.
__device__ __forceinline__ double quartic_root(double a4, double a1,
                                               double c0) {
  const double u1 = c0 / a1;
  const double u4 = a4 > 0.0 ? sqrt(sqrt(c0 / a4)) : u1;
  double x = fmin(u1, u4);
  const double lo = 0.5 * x;  // f(lo) < 0 for this bound
  for (int it = 0; it < 100; ++it) {
    const double x2 = x * x;
    const double f = (a4 * x2) * x2 + a1 * x - c0;
    const double fp = 4.0 * a4 * x2 * x + a1;
    const double step = f / fp;
    double xn = x - step;
    if (xn < lo) xn = lo;
    const bool last = !(fabs(step) > 4.0 * 2.220446049250313e-16 * x);
    x = xn;
    if (last) break;
  }
  // two polishing steps
  for (int it = 0; it < 2; ++it) {
    const double x2 = x * x;
    const double f = (a4 * x2) * x2 + a1 * x - c0;
    const double fp = 4.0 * a4 * x2 * x + a1;
    x -= f / fp;
  }
  return x;
}

__global__ void __launch_bounds__(kBlock)
    k_exchange(int64_t N, double dt, double c, double a_rad, double gm1,
               double gas_const, const double* __restrict__ rho,
               const double* __restrict__ kappa, double* __restrict__ E,
               double* __restrict__ e) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  const double r = rho[i];
  const double beta = dt * c * kappa[i] * r;
  const double Ei = E[i], ei = e[i];
  const double S = Ei + ei;
  const double t = gm1 / (r * gas_const);
  const double t2 = t * t;
  const double a4 = beta * a_rad * (t2 * t2);
  const double x = quartic_root(a4, 1.0 + beta, ei + beta * S);
  e[i] = x;
  E[i] = S - x;
}

hipError_t launch_exchange(int64_t N, double dt, double c, double a_rad,
                           double gamma, double gas_const, const double* rho,
                           const double* kappa, double* E, double* e,
                           hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_exchange, dim3(blocks_for(N)), dim3(kBlock), 0, s, N,
                     dt, c, a_rad, gamma - 1.0, gas_const, rho, kappa, E, e);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
    k_opacity(int64_t N, double gm1, double gas_const,
              const double* __restrict__ rho, const double* __restrict__ e,
              double k0, double pa, double pb, double kmin, double kmax,
              double* __restrict__ kappa) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  const double r = rho[i];
  const double T = gm1 * e[i] / (r * gas_const);
  const double k = k0 * pow(r, pa) * pow(T, pb);
  kappa[i] = fmin(fmax(k, kmin), kmax);
}

hipError_t launch_opacity(int64_t N, double gamma, double gas_const,
                          const double* rho, const double* e, double k0,
                          double pa, double pb, double kmin, double kmax,
                          double* kappa, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_opacity, dim3(blocks_for(N)), dim3(kBlock), 0, s, N,
                     gamma - 1.0, gas_const, rho, e, k0, pa, pb, kmin, kmax,
                     kappa);
  return hipGetLastError();
}

}  // namespace fld
