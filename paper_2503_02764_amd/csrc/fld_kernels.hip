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

#include <limits.h>
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

__global__ void k_ctrl_init(Control* ctrl, double rtol, int max_cycles,
                            int inner, Control* mirror) {
  if (threadIdx.x == 0) {
    ctrl->mirror = mirror;
    ctrl->outer = 0;
    ctrl->inner = inner;
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
                            int inner, Control* mirror, hipStream_t s) {
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, s, ctrl, rtol,
                     max_cycles, inner, mirror);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
    k_fill32(float* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = 0.0f;
}

hipError_t launch_fill32(float* x, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill32, dim3(blocks_for(n)), dim3(kBlock), 0, s, x, n);
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

__device__ __forceinline__ void finalize_update(int mode, double s,
                                                Control* ctrl);

// Single-block reduction of the block partials and the stop decision; the
// control block is then copied to its host-visible mirror.
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
  finalize_update(mode, s, ctrl);
  if (ctrl->mirror) *ctrl->mirror = *ctrl;
}

__device__ __forceinline__ void finalize_update(int mode, double s,
                                                Control* ctrl) {
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
  if (mode == kFinOuter) {
    if (ctrl->outer == 0 && ctrl->cycles == 0) ctrl->res_initial = r;
    if (r <= ctrl->rtol) {
      ctrl->done = kConverged;
    } else if (ctrl->cycles >= ctrl->max_cycles) {
      ctrl->done = kCapped;
    } else {
      ctrl->outer += 1;
      ctrl->cycles += ctrl->inner;
    }
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

struct CoefOut {
  double* a64[3];
  float* a32[3];  // FP32 copies for the mixed-precision hierarchy (or null)
  double* copy_dst;
  double* partials;
  Control* ctrl;
};

__global__ void __launch_bounds__(kBlock)
    k_coef(CoefArgs A, const double* __restrict__ E,
           const double* __restrict__ rho, const double* __restrict__ kappa,
           CoefOut O) {
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
      O.a64[d][idx] = alpha;
      if (O.a32[d]) O.a32[d][idx] = (float)alpha;
    }
    const double Ei = E[idx];
    if (O.copy_dst) O.copy_dst[idx] = Ei;
    e2 = Ei * Ei;
    if (bad) atomicAdd(&bad_count, 1);
  }
  const double s = block_sum<kBlock>(e2, sh);
  if (threadIdx.x == 0) {
    O.partials[blockIdx.x] = s;
    if (bad_count > 0) atomicAdd(&O.ctrl->flagged, bad_count);
  }
}

hipError_t launch_coef(const CoefArgs& a, const double* E, const double* rho,
                       const double* kappa, double* const a64[3],
                       float* const a32[3], double* copy_dst, double* partials,
                       Control* ctrl, hipStream_t s) {
  CoefOut O;
  for (int d = 0; d < 3; ++d) {
    O.a64[d] = a64[d];
    O.a32[d] = a32[d];
  }
  O.copy_dst = copy_dst;
  O.partials = partials;
  O.ctrl = ctrl;
  hipLaunchKernelGGL(k_coef, dim3(blocks_for(a.g.N)), dim3(kBlock), 0, s, a,
                     E, rho, kappa, O);
  return hipGetLastError();
}

// Coarse face coefficient = 1/4 of the mean over the 2^(d-1) fine faces that
// make up the coarse face (D averaged over the face, dx doubled).
template <typename T>
struct CoarsenArgs {
  Geom f, c;
  const T* fa[3];
  T* ca[3];
};

template <typename T>
__global__ void __launch_bounds__(kBlock) k_coarsen(CoarsenArgs<T> A) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= A.c.N) return;
  int c[3];
  coords(A.c, idx, c);
  const int nd = A.c.ndim;
  for (int d = 0; d < nd; ++d) {
    T s = T(0);
    int cnt = 0;
    // fine cell on the lower side of the coarse face: 2c+1 along d,
    // 2c or 2c+1 across.
    const int o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
    for (int q2 = 0; q2 < o2; ++q2)
      for (int q1 = 0; q1 < o1; ++q1) {
        int f[3] = {2 * c[0], 2 * c[1], 2 * c[2]};
        f[d] += 1;
        // the transverse dimensions of d, in increasing order
        const int t1 = (d == 0) ? 1 : 0;
        const int t2 = (d == 2) ? 1 : 2;
        if (nd > 1) f[t1] += q1;
        if (nd > 2) f[t2] += q2;
        const int64_t fi =
            f[0] + (int64_t)A.f.n[0] * (f[1] + (int64_t)A.f.n[1] * f[2]);
        s += A.fa[d][fi];
        ++cnt;
      }
    A.ca[d][idx] = T(0.25) * s / T(cnt);
  }
}

template <typename T>
hipError_t launch_coarsen(const Geom& fine, const Geom& coarse,
                          const T* const fa[3], T* const ca[3],
                          hipStream_t s) {
  CoarsenArgs<T> A;
  A.f = fine;
  A.c = coarse;
  for (int d = 0; d < 3; ++d) {
    A.fa[d] = fa[d];
    A.ca[d] = ca[d];
  }
  hipLaunchKernelGGL(k_coarsen<T>, dim3(blocks_for(coarse.N)), dim3(kBlock), 0,
                     s, A);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// multigrid, one launch per phase (1D/3D levels and the reference path)
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_resid_norm(LevelView<T> L, double* __restrict__ partials,
                 const Control* __restrict__ ctrl) {
  __shared__ double sh[kBlock / 64];
  if (ctrl->done != kRunning) return;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double r2 = 0.0;
  if (idx < L.g.N) {
    int c[3];
    coords(L.g, idx, c);
    const double r = (double)residual_value(L, c, idx);
    r2 = r * r;
  }
  const double s = block_sum<kBlock>(r2, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <typename T>
hipError_t launch_resid_norm(const LevelView<T>& L, double* partials,
                             int* nblocks, const Control* ctrl,
                             hipStream_t s) {
  *nblocks = blocks_for(L.g.N);
  hipLaunchKernelGGL(k_resid_norm<T>, dim3(*nblocks), dim3(kBlock), 0, s, L,
                     partials, ctrl);
  return hipGetLastError();
}

// FP64 residual of the refinement loop, handed to the FP32 hierarchy:
// r32 = (float)(b - A x) and the block sums of r^2.
__global__ void __launch_bounds__(kBlock)
    k_resid_to32(LevelView<double> L, float* __restrict__ r32,
                 double* __restrict__ partials,
                 const Control* __restrict__ ctrl) {
  __shared__ double sh[kBlock / 64];
  if (ctrl->done != kRunning) return;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double r2 = 0.0;
  if (idx < L.g.N) {
    int c[3];
    coords(L.g, idx, c);
    const double r = residual_value(L, c, idx);
    r32[idx] = (float)r;
    r2 = r * r;
  }
  const double s = block_sum<kBlock>(r2, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

hipError_t launch_resid_to32(const LevelView<double>& L, float* r32,
                             double* partials, int* nblocks,
                             const Control* ctrl, hipStream_t s) {
  *nblocks = blocks_for(L.g.N);
  hipLaunchKernelGGL(k_resid_to32, dim3(*nblocks), dim3(kBlock), 0, s, L, r32,
                     partials, ctrl);
  return hipGetLastError();
}

// x64 += e32 (the FP32 correction of one refinement iteration)
__global__ void __launch_bounds__(kBlock)
    k_correct(int64_t N, double* __restrict__ x, const float* __restrict__ e,
              const Control* __restrict__ ctrl) {
  if (ctrl->done != kRunning) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < N) x[i] += (double)e[i];
}

hipError_t launch_correct(int64_t N, double* x, const float* e,
                          const Control* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_correct, dim3(blocks_for(N)), dim3(kBlock), 0, s, N, x,
                     e, ctrl);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_gs_color(LevelView<T> L, int color, const Control* __restrict__ ctrl) {
  if (ctrl->done != kRunning) return;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= L.g.N) return;
  int c[3];
  coords(L.g, idx, c);
  if (((c[0] + c[1] + c[2]) & 1) != color) return;
  L.x[idx] = relax_value(L, c, idx, L.x);
}

template <typename T>
hipError_t launch_gs_color(const LevelView<T>& L, int color,
                           const Control* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_gs_color<T>, dim3(blocks_for(L.g.N)), dim3(kBlock), 0,
                     s, L, color, ctrl);
  return hipGetLastError();
}

// Coarse rhs = mean of the 2^d fine residuals; coarse x = 0.  With a
// partials buffer, also the block sums of the fine residual squared.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_resid_restrict(LevelView<T> F, LevelView<T> C,
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
    const int o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
    T s = T(0);
    for (int q2 = 0; q2 < o2; ++q2)
      for (int q1 = 0; q1 < o1; ++q1)
        for (int q0 = 0; q0 < 2; ++q0) {
          int f[3] = {2 * c[0] + q0, nd > 1 ? 2 * c[1] + q1 : 0,
                      nd > 2 ? 2 * c[2] + q2 : 0};
          const int64_t fi =
              f[0] + (int64_t)F.g.n[0] * (f[1] + (int64_t)F.g.n[1] * f[2]);
          const T r = residual_value(F, f, fi);
          s += r;
          r2 += (double)r * (double)r;
        }
    C.b[idx] = s / T(2 * o1 * o2);
    C.x[idx] = T(0);
  }
  if (partials) {
    const double t = block_sum<kBlock>(r2, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
  }
}

template <typename T>
hipError_t launch_resid_restrict(const LevelView<T>& fine,
                                 const LevelView<T>& coarse, double* partials,
                                 int* nblocks, const Control* ctrl,
                                 hipStream_t s) {
  *nblocks = blocks_for(coarse.g.N);
  hipLaunchKernelGGL(k_resid_restrict<T>, dim3(*nblocks), dim3(kBlock), 0, s,
                     fine, coarse, partials, ctrl);
  return hipGetLastError();
}

// Correction of fine cell f from the coarse level: cell-centred
// (bi/tri)linear interpolation, weight 3/4 on the parent and 1/4 on the next
// coarse cell on the child's side, per dimension; mirror (Neumann) or
// wrapped (periodic) coarse ghosts.
template <typename T>
__device__ __forceinline__ T prolong_value(const LevelView<T>& C,
                                           const int f[3], int nd) {
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
  T e = T(0);
  for (int s2 = 0; s2 < o2; ++s2)
    for (int s1 = 0; s1 < o1; ++s1)
      for (int s0 = 0; s0 < 2; ++s0) {
        const int i = s0 ? q[0] : p[0];
        const int j = s1 ? q[1] : p[1];
        const int k = s2 ? q[2] : p[2];
        const T w = T((s0 ? 0.25 : 0.75) * (nd > 1 ? (s1 ? 0.25 : 0.75) : 1.0) *
                      (nd > 2 ? (s2 ? 0.25 : 0.75) : 1.0));
        e += w * C.x[i + (int64_t)C.g.n[0] * (j + (int64_t)C.g.n[1] * k)];
      }
  return e;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_prolong(LevelView<T> C, LevelView<T> F,
              const Control* __restrict__ ctrl) {
  if (ctrl->done != kRunning) return;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= F.g.N) return;
  int f[3];
  coords(F.g, idx, f);
  F.x[idx] += prolong_value(C, f, F.g.ndim);
}

template <typename T>
hipError_t launch_prolong(const LevelView<T>& coarse, const LevelView<T>& fine,
                          const Control* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_prolong<T>, dim3(blocks_for(fine.g.N)), dim3(kBlock), 0,
                     s, coarse, fine, ctrl);
  return hipGetLastError();
}

// Coarsest level: Jacobi sweeps in one block until the residual norm has
// dropped by 1e-6 (A = I + L is strictly diagonally dominant, so Jacobi
// converges for any alpha).  tmp holds the next iterate.
template <typename T>
__device__ void t_coarsest(const LevelView<T>& L, T* tmp, double* sh,
                           double* bc) {
  const int64_t N = L.g.N;
  double r0 = 0.0;
  for (int it = 0; it < 4000; ++it) {
    if ((it & 7) == 0) {
      double v = 0.0;
      for (int64_t i = threadIdx.x; i < N; i += kReduceBlock) {
        int c[3];
        coords(L.g, i, c);
        const double r = (double)residual_value(L, c, i);
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

template <typename T>
__global__ void __launch_bounds__(kReduceBlock)
    k_coarsest(LevelView<T> L, T* __restrict__ tmp,
               const Control* __restrict__ ctrl) {
  __shared__ double sh[kReduceBlock / 64];
  __shared__ double bc[2];
  if (ctrl->done != kRunning) return;
  t_coarsest(L, tmp, sh, bc);
}

template <typename T>
hipError_t launch_coarsest(const LevelView<T>& L, T* tmp, const Control* ctrl,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_coarsest<T>, dim3(1), dim3(kReduceBlock), 0, s, L, tmp,
                     ctrl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// single-workgroup tail of the V-cycle
// ---------------------------------------------------------------------------
//
// Levels small enough for one workgroup (a few thousand cells) are handled
// by one block of kReduceBlock threads with block barriers between phases,
// instead of one launch per phase and level.  In "whole" mode (l0 == 0 in
// FP64) the block also runs the cycle loop and the stop test.

template <typename T>
__device__ void t_smooth(const LevelView<T>& L, int sweeps) {
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
template <typename T>
__device__ double t_resid_restrict(const LevelView<T>& F,
                                   const LevelView<T>& C) {
  const int nd = F.g.ndim;
  const int o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
  double r2 = 0.0;
  for (int64_t idx = threadIdx.x; idx < C.g.N; idx += kReduceBlock) {
    int c[3];
    coords(C.g, idx, c);
    T s = T(0);
    for (int q2 = 0; q2 < o2; ++q2)
      for (int q1 = 0; q1 < o1; ++q1)
        for (int q0 = 0; q0 < 2; ++q0) {
          int f[3] = {2 * c[0] + q0, nd > 1 ? 2 * c[1] + q1 : 0,
                      nd > 2 ? 2 * c[2] + q2 : 0};
          const int64_t fi =
              f[0] + (int64_t)F.g.n[0] * (f[1] + (int64_t)F.g.n[1] * f[2]);
          const T r = residual_value(F, f, fi);
          s += r;
          r2 += (double)r * (double)r;
        }
    C.b[idx] = s / T(2 * o1 * o2);
    C.x[idx] = T(0);
  }
  __syncthreads();
  return r2;
}

template <typename T>
__device__ void t_prolong(const LevelView<T>& C, const LevelView<T>& F) {
  for (int64_t idx = threadIdx.x; idx < F.g.N; idx += kReduceBlock) {
    int f[3];
    coords(F.g, idx, f);
    F.x[idx] += prolong_value(C, f, F.g.ndim);
  }
  __syncthreads();
}

// The tail levels are copied into LDS first when they fit (kTailLdsCells),
// so every phase works on LDS rather than on L2-resident global memory; the
// result x(l0) is written back at the end.
template <typename T, bool kLds>
__global__ void __launch_bounds__(kReduceBlock) k_tail(TailArgs<T> A) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sh[kReduceBlock / 64];
  __shared__ double bc[2];
  __shared__ int stop;
  __shared__ LevelView<T> lv[kMaxLevels];
  __shared__ T* tmp_s;
  if (A.ctrl->done != kRunning) return;
  const int l0 = A.l0;
  if (threadIdx.x == 0) {
    T* p = (T*)smem;
    for (int l = 0; l < A.L; ++l) {
      lv[l] = A.lv[l];
      if (!kLds || l < l0) continue;
      const int64_t n = A.lv[l].g.N;
      lv[l].x = p;
      p += n;
      lv[l].b = p;
      p += n;
      for (int d = 0; d < A.lv[l].g.ndim; ++d) {
        lv[l].a[d] = p;
        p += n;
      }
    }
    tmp_s = kLds ? p : A.tmp;
  }
  __syncthreads();
  if (kLds) {
    for (int l = l0; l < A.L; ++l) {
      const int n = (int)A.lv[l].g.N;
      for (int d = 0; d < A.lv[l].g.ndim; ++d) {
        T* dst = const_cast<T*>(lv[l].a[d]);
        for (int i = threadIdx.x; i < n; i += kReduceBlock)
          dst[i] = A.lv[l].a[d][i];
      }
    }
    const int n0 = (int)A.lv[l0].g.N;
    for (int i = threadIdx.x; i < n0; i += kReduceBlock) {
      lv[l0].b[i] = A.lv[l0].b[i];
      lv[l0].x[i] = A.zero ? T(0) : A.lv[l0].x[i];
    }
  } else if (A.zero) {
    for (int64_t i = threadIdx.x; i < A.lv[l0].g.N; i += kReduceBlock)
      A.lv[l0].x[i] = T(0);
  }
  __syncthreads();
  TailArgs<T> const& G = A;
  (void)G;
  if (!A.whole) {
    for (int l = l0; l + 1 < A.L; ++l) {
      t_smooth(lv[l], A.pre);
      (void)t_resid_restrict(lv[l], lv[l + 1]);
    }
    t_coarsest(lv[A.L - 1], tmp_s, sh, bc);
    for (int l = A.L - 2; l >= l0; --l) {
      t_prolong(lv[l + 1], lv[l]);
      t_smooth(lv[l], A.post);
    }
  } else {
    // whole problem: cycle loop with the stop test of k_finalize
    for (;;) {
      double r2;
      if (A.L > 1) {
        t_smooth(lv[0], A.pre);
        r2 = t_resid_restrict(lv[0], lv[1]);
      } else {
        t_coarsest(lv[0], tmp_s, sh, bc);
        r2 = 0.0;
        for (int64_t i = threadIdx.x; i < lv[0].g.N; i += kReduceBlock) {
          int c[3];
          coords(lv[0].g, i, c);
          const double r = (double)residual_value(lv[0], c, i);
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
      if (stop) break;
      if (A.L > 1) {
        for (int l = 1; l + 1 < A.L; ++l) {
          t_smooth(lv[l], A.pre);
          (void)t_resid_restrict(lv[l], lv[l + 1]);
        }
        t_coarsest(lv[A.L - 1], tmp_s, sh, bc);
        for (int l = A.L - 2; l >= 0; --l) {
          t_prolong(lv[l + 1], lv[l]);
          t_smooth(lv[l], A.post);
        }
      }
    }
  }
  if (kLds) {
    const int n0 = (int)A.lv[l0].g.N;
    for (int i = threadIdx.x; i < n0; i += kReduceBlock)
      A.lv[l0].x[i] = lv[l0].x[i];
  }
}

template <typename T>
hipError_t launch_tail(const TailArgs<T>& a, hipStream_t s) {
  bool used = false;
  hipError_t e = launch_tail_lds<T>(a, s, &used);
  if (used || e != hipSuccess) return e;
  hipLaunchKernelGGL((k_tail<T, false>), dim3(1), dim3(kReduceBlock), 0, s, a);
  return hipGetLastError();
}

#define FLD_INSTANTIATE_MG(T)                                                  \
  template hipError_t launch_coarsen<T>(const Geom&, const Geom&,              \
                                        const T* const[3], T* const[3],        \
                                        hipStream_t);                          \
  template hipError_t launch_resid_norm<T>(const LevelView<T>&, double*, int*, \
                                           const Control*, hipStream_t);       \
  template hipError_t launch_gs_color<T>(const LevelView<T>&, int,             \
                                         const Control*, hipStream_t);         \
  template hipError_t launch_resid_restrict<T>(                                \
      const LevelView<T>&, const LevelView<T>&, double*, int*, const Control*, \
      hipStream_t);                                                            \
  template hipError_t launch_prolong<T>(const LevelView<T>&,                   \
                                        const LevelView<T>&, const Control*,   \
                                        hipStream_t);                          \
  template hipError_t launch_coarsest<T>(const LevelView<T>&, T*,              \
                                         const Control*, hipStream_t);         \
  template hipError_t launch_tail<T>(const TailArgs<T>&, hipStream_t);

FLD_INSTANTIATE_MG(double)
FLD_INSTANTIATE_MG(float)

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

// x^(h/2) for an integer h: repeated squaring and one square root.
__device__ __forceinline__ double pow_half(double x, int h) {
  const bool neg = h < 0;
  int n = neg ? -h : h;
  double r = 1.0, base = x;
  for (int k = n >> 1; k; k >>= 1) {
    if (k & 1) r *= base;
    base *= base;
  }
  if (n & 1) r *= sqrt(x);
  return neg ? 1.0 / r : r;
}

// ha, hb: twice the exponents when both are half-integers (|2a|, |2b| <= 32),
// so the power law needs no pow(); otherwise ha = INT_MIN and pow() is used.
__global__ void __launch_bounds__(kBlock)
    k_opacity(int64_t N, double gm1, double gas_const,
              const double* __restrict__ rho, const double* __restrict__ e,
              double k0, double pa, double pb, int ha, int hb, double kmin,
              double kmax, double* __restrict__ kappa) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  const double r = rho[i];
  const double T = gm1 * e[i] / (r * gas_const);
  const double k = ha != INT_MIN ? k0 * pow_half(r, ha) * pow_half(T, hb)
                                 : k0 * pow(r, pa) * pow(T, pb);
  kappa[i] = fmin(fmax(k, kmin), kmax);
}

hipError_t launch_opacity(int64_t N, double gamma, double gas_const,
                          const double* rho, const double* e, double k0,
                          double pa, double pb, double kmin, double kmax,
                          double* kappa, hipStream_t s) {
  if (N == 0) return hipSuccess;
  int ha = INT_MIN, hb = INT_MIN;
  if (2.0 * pa == floor(2.0 * pa) && 2.0 * pb == floor(2.0 * pb) &&
      fabs(pa) <= 16.0 && fabs(pb) <= 16.0) {
    ha = (int)(2.0 * pa);
    hb = (int)(2.0 * pb);
  }
  hipLaunchKernelGGL(k_opacity, dim3(blocks_for(N)), dim3(kBlock), 0, s, N,
                     gamma - 1.0, gas_const, rho, e, k0, pa, pb, ha, hb, kmin,
                     kmax, kappa);
  return hipGetLastError();
}

}  // namespace fld
