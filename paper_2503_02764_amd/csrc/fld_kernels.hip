// HIP kernels of the FLD radiation-energy update for gfx950 (wave64).
//
// Coefficient stage (Sect. 2, eqs. fld_F, fld_lambda, fld_R; gradient by the
// five-point stencil of Sect. 3), the backward-Euler diffusion multigrid
// (Sect. 3 solves div F with geometric multigrid) and the implicit
// gas-radiation exchange quartic (eqs. heating, qdot; Sect. 3).
//
// Every kernel here is memory-bound (well under 10 flop/byte).  Reductions
// are deterministic: a fixed wave-level DPP tree, then a fixed loop over the
// waves of a block, then one single-block pass over the block partials.
#include <hip/hip_ext.h>

#include "fld_internal.h"
#include "fld_device.h"

#include <limits.h>
#include <stdlib.h>

#include <algorithm>
#include <math.h>

namespace fld {

// ---------------------------------------------------------------------------
// control block
// ---------------------------------------------------------------------------

__global__ void k_ctrl_init(Control* ctrl, double rtol, int max_cycles,
                            int inner, Control* mirror) {
  ctrl_init_body(ctrl, rtol, max_cycles, inner, mirror);
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

__global__ void __launch_bounds__(kReduceBlock)
    k_finalize(int mode, const double* __restrict__ partials, int count,
               Control* ctrl) {
  finalize_body(mode, partials, count, ctrl);
}

hipError_t launch_finalize(int mode, const double* partials, int count,
                           Control* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kReduceBlock), 0, s, mode,
                     partials, count, ctrl);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kReduceBlock)
    k_guess_judge(int mode, const double* __restrict__ partials, int count,
                  double q2, Control* ctrl) {
  __shared__ double sh[kReduceBlock / 64];
  if (ctrl->done != kRunning) return;
  double v = 0.0;
  for (int i = threadIdx.x; i < count; i += kReduceBlock) v += partials[i];
  const double s = block_sum<kReduceBlock>(v, sh);
  if (threadIdx.x != 0) return;
  if (mode == 0)
    ctrl->guess_ref = s;
  else
    ctrl->guess_rejected = (s < q2 * ctrl->guess_ref) ? 0 : 1;  // NaN: rejected
}

hipError_t launch_guess_judge(int mode, const double* partials, int count,
                              double q2, Control* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_guess_judge, dim3(1), dim3(kReduceBlock), 0, s, mode,
                     partials, count, q2, ctrl);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
    k_guess_take(int64_t n, const double* __restrict__ guess,
                 double* __restrict__ x, const Control* ctrl) {
  if (ctrl->done != kRunning || ctrl->guess_rejected) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = guess[i];
}

hipError_t launch_guess_take(int64_t n, const double* guess, double* x,
                             const Control* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_guess_take, dim3(blocks_for(n)), dim3(kBlock), 0, s,
                     n, guess, x, ctrl);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
    k_take_alt(int64_t n, const double* __restrict__ alt,
               double* __restrict__ x, const Control* ctrl) {
  if (!ctrl->stop_in_down) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = alt[i];
}

hipError_t launch_take_alt(int64_t n, const double* alt, double* x,
                           const Control* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_take_alt, dim3(blocks_for(n)), dim3(kBlock), 0, s, n,
                     alt, x, ctrl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// coefficient stage
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock)
    k_coef(CoefArgs A, const double* __restrict__ E,
           const double* __restrict__ rho, const double* __restrict__ kappa,
           CoefOut O) {
  coef_body(A, E, rho, kappa, O, blockIdx.x);
}

// 3D levels: a block of k3T threads covers a run of k3X cells along x in
// k3Y consecutive rows of one z-plane (thread t: x offset t % k3X, row
// t / k3X), so the cell coordinates come from the block and thread indices
// without divisions; a colour pass covers only the cells of its colour.
// Eight rows rather than four: the rows above and below a block, which its
// stencils read and neighbouring blocks (other XCDs) own, are a smaller share
// of its loads.
constexpr int k3X = 64, k3Y = 8, k3T = k3X * k3Y;
dim3 grid3(int64_t xcells, int ny, int nz);
bool fits3(const Geom& g);

// 3D grids: the same per cell on the 3D launch grid (no index divisions).
__global__ void __launch_bounds__(k3T)
    k_coef_3d(CoefArgs A, const double* __restrict__ E,
              const double* __restrict__ rho, const double* __restrict__ kappa,
              CoefOut O);

// 3D grids with a scratch array: two passes, D once per cell, then the faces.
__global__ void __launch_bounds__(k3T)
    k_cellD_3d(CoefArgs A, const double* __restrict__ E,
               const double* __restrict__ rho, const double* __restrict__ kappa,
               double* __restrict__ Dc, CoefOut O);
__global__ void __launch_bounds__(k3T)
    k_faces_3d(CoefArgs A, const double* __restrict__ Dc, CoefOut O);
__global__ void __launch_bounds__(k3T)
    k_resid_to32_3d(LevelView<double> L, float* __restrict__ r32,
                    double* __restrict__ partials,
                    const Control* __restrict__ ctrl);

hipError_t launch_coef(const CoefArgs& a, const double* E, const double* rho,
                       const double* kappa, double* const a64[3],
                       float* const a32[3], double* copy_dst, double* partials,
                       Control* ctrl, hipStream_t s, int* nblocks,
                       double* dscr, double* sd, double* rhs,
                       const uint8_t* held, const double* hold) {
  CoefOut O;
  for (int d = 0; d < 3; ++d) {
    O.a64[d] = a64[d];
    O.a32[d] = a32[d];
  }
  O.copy_dst = copy_dst;
  O.partials = partials;
  O.ctrl = ctrl;
  O.sd = sd;
  O.rhs = rhs;
  O.held = held;
  O.hold = hold;
  if (rhs) dscr = nullptr;  // the one-pass kernels write the own b
  if (fits3(a.g)) {
    if (nblocks) *nblocks = (int)blocks3(a.g);
    const dim3 grid = grid3(a.g.n[0], a.g.n[1], a.g.n[2]);
    if (dscr) {
      hipLaunchKernelGGL(k_cellD_3d, grid, dim3(k3T), 0, s, a, E, rho,
                         kappa, dscr, O);
      hipLaunchKernelGGL(k_faces_3d, grid, dim3(k3T), 0, s, a,
                         (const double*)dscr, O);
    } else {
      hipLaunchKernelGGL(k_coef_3d, grid, dim3(k3T), 0, s, a, E, rho,
                         kappa, O);
    }
    return hipGetLastError();
  }
  if (nblocks) *nblocks = blocks_for(a.g.N);
  hipLaunchKernelGGL(k_coef, dim3(blocks_for(a.g.N)), dim3(kBlock), 0, s, a,
                     E, rho, kappa, O);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_coarsen(CoarsenArgs<T> A) {
  coarsen_body(A, blockIdx.x);
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

// Dirichlet walls' diagonal term of a coarse level: the coarse wall face
// carries the mean of its fine faces' alpha_w, a quarter as large with the
// spacing doubled, so sd_c = (sum over the 2^d children of sd_f) /
// 2^(d+1) (the children off the wall contribute 0; a corner cell sums its
// walls).
__global__ void __launch_bounds__(kBlock)
    k_coarsen_sd(Geom F, Geom C, const double* __restrict__ sdf,
                 double* __restrict__ sdc) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= C.N) return;
  int c[3];
  coords(C, idx, c);
  const int nd = F.ndim;
  const int o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
  double s = 0.0;
  for (int q2 = 0; q2 < o2; ++q2)
    for (int q1 = 0; q1 < o1; ++q1)
      for (int q0 = 0; q0 < 2; ++q0) {
        const int f0 = 2 * c[0] + q0, f1 = nd > 1 ? 2 * c[1] + q1 : 0;
        const int f2 = nd > 2 ? 2 * c[2] + q2 : 0;
        s += sdf[f0 + (int64_t)F.n[0] * (f1 + (int64_t)F.n[1] * f2)];
      }
  sdc[idx] = s / (double)(2 << nd);
}

hipError_t launch_coarsen_sd(const Geom& fine, const Geom& coarse,
                             const double* sdf, double* sdc, hipStream_t s) {
  hipLaunchKernelGGL(k_coarsen_sd, dim3(blocks_for(coarse.N)), dim3(kBlock), 0,
                     s, fine, coarse, sdf, sdc);
  return hipGetLastError();
}

// Held cells (an interior boundary with prescribed new values) eliminated
// from the free cells' rows: a free cell's face to a held neighbour goes
// onto its diagonal and the neighbour's held value times that face onto its
// right-hand side, exactly as a Dirichlet wall at the neighbour's centre.
// Each thread writes its own cell only (the faces are read here and cut by
// the next kernel), so the two kernels need no ordering inside a launch.
__global__ void __launch_bounds__(kBlock)
    k_held_fold(Geom g, const double* __restrict__ a0,
                const double* __restrict__ a1, const double* __restrict__ a2,
                const uint8_t* __restrict__ held,
                const double* __restrict__ hold, double* __restrict__ sd,
                double* __restrict__ rhs, double* __restrict__ partials) {
  __shared__ double sh[kBlock / 64];
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double b2 = 0.0;
  if (idx < g.N) {
    double bi = rhs[idx];
    if (!held[idx]) {
      const double* a[3] = {a0, a1, a2};
      int c[3];
      coords(g, idx, c);
      double s = 0.0, add = 0.0;
      for (int d = 0; d < g.ndim; ++d) {
        const int64_t st = stride_of(g, d);
        int64_t nl, nu;
        double al, au;
        lower_nb(g, a[d], d, c[d], idx, st, nl, al);
        upper_nb(g, a[d], d, c[d], idx, st, nu, au);
        if (held[nl]) {
          s += al;
          add += al * hold[nl];
        }
        if (held[nu]) {
          s += au;
          add += au * hold[nu];
        }
      }
      sd[idx] += s;
      bi += add;
      rhs[idx] = bi;
    } else {
      sd[idx] = 0.0;  // a held row is x = E_hold, walls or not
    }
    b2 = bi * bi;
  }
  const double t = block_sum<kBlock>(b2, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// Zero every face touching a held cell (each thread its own upper faces).
__global__ void __launch_bounds__(kBlock)
    k_held_cut(Geom g, double* __restrict__ a0, double* __restrict__ a1,
               double* __restrict__ a2, const uint8_t* __restrict__ held) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= g.N) return;
  double* a[3] = {a0, a1, a2};
  int c[3];
  coords(g, idx, c);
  for (int d = 0; d < g.ndim; ++d) {
    const int64_t st = stride_of(g, d);
    int64_t nu;
    double au;
    upper_nb(g, (const double*)a[d], d, c[d], idx, st, nu, au);
    if (held[idx] || held[nu]) a[d][idx] = 0.0;
  }
}

hipError_t launch_held_fold(const Geom& g, double* const a[3],
                            const uint8_t* held, const double* hold,
                            double* sd, double* rhs, double* partials,
                            int* nblocks, hipStream_t s) {
  *nblocks = blocks_for(g.N);
  hipLaunchKernelGGL(k_held_fold, dim3(*nblocks), dim3(kBlock), 0, s, g, a[0],
                     a[1], a[2], held, hold, sd, rhs, partials);
  return hipGetLastError();
}

hipError_t launch_held_cut(const Geom& g, double* const a[3],
                           const uint8_t* held, hipStream_t s) {
  hipLaunchKernelGGL(k_held_cut, dim3(blocks_for(g.N)), dim3(kBlock), 0, s, g,
                     a[0], a[1], a[2], held);
  return hipGetLastError();
}

// Held points of a coarse level: a coarse cell with any held child.  The
// coarse faces come from the finest level's faces before the cut, so a
// free coarse cell next to such a point couples to it as to a Dirichlet
// point of zero correction, which keeps the coarse operator as stiff as
// the fine one near the held cells.
__global__ void __launch_bounds__(kBlock)
    k_coarsen_held(Geom F, Geom C, const uint8_t* __restrict__ hf,
                   uint8_t* __restrict__ hc) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= C.N) return;
  int c[3];
  coords(C, idx, c);
  const int nd = F.ndim;
  const int o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
  bool any = false;
  for (int q2 = 0; q2 < o2; ++q2)
    for (int q1 = 0; q1 < o1; ++q1)
      for (int q0 = 0; q0 < 2; ++q0) {
        const int f0 = 2 * c[0] + q0, f1 = nd > 1 ? 2 * c[1] + q1 : 0;
        const int f2 = nd > 2 ? 2 * c[2] + q2 : 0;
        any = any || hf[f0 + (int64_t)F.n[0] * (f1 + (int64_t)F.n[1] * f2)];
      }
  hc[idx] = any ? 1 : 0;
}

hipError_t launch_coarsen_held(const Geom& fine, const Geom& coarse,
                               const uint8_t* hf, uint8_t* hc, hipStream_t s) {
  hipLaunchKernelGGL(k_coarsen_held, dim3(blocks_for(coarse.N)), dim3(kBlock),
                     0, s, fine, coarse, hf, hc);
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
  if constexpr (sizeof(T) == sizeof(double)) {
    // 3D FP64: the residual kernel of the 3D launch grid, without its FP32
    // output (same residual per cell); a level with Dirichlet walls takes
    // the generic kernel (residual_value has their diagonal term)
    if (fits3(L.g) && !L.sd && !L.held) {
      *nblocks = (int)blocks3(L.g);
      hipLaunchKernelGGL(k_resid_to32_3d, grid3(L.g.n[0], L.g.n[1], L.g.n[2]),
                         dim3(k3T), 0, s, L, (float*)nullptr, partials, ctrl);
      return hipGetLastError();
    }
  }
  *nblocks = blocks_for(L.g.N);
  hipLaunchKernelGGL(k_resid_norm<T>, dim3(*nblocks), dim3(kBlock), 0, s, L,
                     partials, ctrl);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
    k_resid_to32(LevelView<double> L, float* __restrict__ r32,
                 double* __restrict__ partials,
                 const Control* __restrict__ ctrl) {
  resid_to32_body(L, r32, partials, ctrl, blockIdx.x);
}


dim3 grid3(int64_t xcells, int ny, int nz) {
  return dim3((unsigned)((xcells + k3X - 1) / k3X),
              (unsigned)((ny + k3Y - 1) / k3Y), (unsigned)nz);
}

// the 3D launch grid applies (grid dimensions y and z within their limits)
bool fits3(const Geom& g) {
  return g.ndim == 3 && (g.n[1] + k3Y - 1) / k3Y <= 65535 && g.n[2] <= 65535;
}

int64_t blocks3(const Geom& g) {
  const dim3 b = grid3(g.n[0], g.n[1], g.n[2]);
  return (int64_t)b.x * b.y * b.z;
}

__device__ __forceinline__ int block3_id() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

__global__ void __launch_bounds__(k3T)
    k_coef_3d(CoefArgs A, const double* __restrict__ E,
              const double* __restrict__ rho, const double* __restrict__ kappa,
              CoefOut O) {
  __shared__ double sh[k3T / 64];
  __shared__ int bad_count;
  if (threadIdx.x == 0) bad_count = 0;
  __syncthreads();
  const int nx = A.g.n[0], ny = A.g.n[1];
  const int x = blockIdx.x * k3X + (threadIdx.x % k3X);
  const int y = blockIdx.y * k3Y + (threadIdx.x / k3X), z = blockIdx.z;
  double e2 = 0.0;
  if (x < nx && y < ny) {
    const int c[3] = {x, y, z};
    bool bad = false;
    e2 = coef_cell(A, E, rho, kappa, O, c, ((int64_t)z * ny + y) * nx + x, bad);
    if (bad) atomicAdd(&bad_count, 1);
  }
  const double t = block_sum<k3T>(e2, sh);
  if (threadIdx.x == 0) {
    O.partials[block3_id()] = t;
    if (bad_count > 0) atomicAdd(&O.ctrl->flagged, bad_count);
  }
}

__global__ void __launch_bounds__(k3T)
    k_cellD_3d(CoefArgs A, const double* __restrict__ E,
               const double* __restrict__ rho, const double* __restrict__ kappa,
               double* __restrict__ Dc, CoefOut O) {
  __shared__ double sh[k3T / 64];
  __shared__ int bad_count;
  if (threadIdx.x == 0) bad_count = 0;
  __syncthreads();
  const int nx = A.g.n[0], ny = A.g.n[1];
  const int x = blockIdx.x * k3X + (threadIdx.x % k3X);
  const int y = blockIdx.y * k3Y + (threadIdx.x / k3X), z = blockIdx.z;
  double e2 = 0.0;
  if (x < nx && y < ny) {
    const int c[3] = {x, y, z};
    const int64_t idx = ((int64_t)z * ny + y) * nx + x;
    bool bad = false;
    Dc[idx] = cell_D(A, E, rho, kappa, c, idx, bad);
    if (bad) atomicAdd(&bad_count, 1);
    const double Ei = E[idx];
    if (O.copy_dst) O.copy_dst[idx] = Ei;
    e2 = Ei * Ei;
  }
  const double t = block_sum<k3T>(e2, sh);
  if (threadIdx.x == 0) {
    O.partials[block3_id()] = t;
    if (bad_count > 0) atomicAdd(&O.ctrl->flagged, bad_count);
  }
}

__global__ void __launch_bounds__(k3T)
    k_faces_3d(CoefArgs A, const double* __restrict__ Dc, CoefOut O) {
  const int nx = A.g.n[0], ny = A.g.n[1];
  const int x = blockIdx.x * k3X + (threadIdx.x % k3X);
  const int y = blockIdx.y * k3Y + (threadIdx.x / k3X), z = blockIdx.z;
  if (x >= nx || y >= ny) return;
  const int c[3] = {x, y, z};
  faces_from_D(A, Dc, O, c, ((int64_t)z * ny + y) * nx + x);
}

__global__ void __launch_bounds__(k3T)
    k_resid_to32_3d(LevelView<double> L, float* __restrict__ r32,
                    double* __restrict__ partials,
                    const Control* __restrict__ ctrl) {
  __shared__ double sh[k3T / 64];
  if (ctrl->done != kRunning) return;
  const int nx = L.g.n[0], ny = L.g.n[1];
  const int x = blockIdx.x * k3X + (threadIdx.x % k3X);
  const int y = blockIdx.y * k3Y + (threadIdx.x / k3X), z = blockIdx.z;
  double r2 = 0.0;
  if (x < nx && y < ny) {
    const int c[3] = {x, y, z};
    const Nbrs<3> n = neighbours<3>(L.g, c, ((int64_t)z * ny + y) * nx + x);
    const double r = residual_nb<3>(L.a, L.x, L.b, n);
    if (r32) r32[n.idx] = (float)r;
    r2 = r * r;
  }
  const double t = block_sum<k3T>(r2, sh);
  if (threadIdx.x == 0) partials[block3_id()] = t;
}

hipError_t launch_resid_to32(const LevelView<double>& L, float* r32,
                             double* partials, int* nblocks,
                             const Control* ctrl, hipStream_t s) {
  if (fits3(L.g)) {
    *nblocks = (int)blocks3(L.g);
    hipLaunchKernelGGL(k_resid_to32_3d, grid3(L.g.n[0], L.g.n[1], L.g.n[2]),
                       dim3(k3T), 0, s, L, r32, partials, ctrl);
    return hipGetLastError();
  }
  *nblocks = blocks_for(L.g.N);
  hipLaunchKernelGGL(k_resid_to32, dim3(*nblocks), dim3(kBlock), 0, s, L, r32,
                     partials, ctrl);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
    k_correct(int64_t N, double* __restrict__ x, const float* __restrict__ e,
              const Control* __restrict__ ctrl) {
  correct_body(N, x, e, ctrl, blockIdx.x);
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
  if (gs_color(L.g, c) != color) return;
  L.x[idx] = relax_value(L, c, idx, L.x);
}

// 3D colour pass: thread (i, y, z) updates cell x = 2i + ((y + z + color) & 1)
// of row (y, z), the one of this colour in its pair.  A block takes kColRY
// rows: the rows above and below a block, which its stencil also reads and
// which neighbouring blocks (on other XCDs, through another L2) own, are then
// a smaller share of what it loads.  8 rows measured best on 256^3 (FP32
// pass 99 -> 98 us; 16 rows were slower than 4).
constexpr int kColRY = 8;

template <typename T>
__global__ void __launch_bounds__(k3X * kColRY)
    k_gs_color_3d(LevelView<T> L, int color, const Control* __restrict__ ctrl) {
  if (ctrl->done != kRunning) return;
  const int nx = L.g.n[0], ny = L.g.n[1];
  const int i = blockIdx.x * k3X + (threadIdx.x % k3X);
  const int y = blockIdx.y * kColRY + (threadIdx.x / k3X), z = blockIdx.z;
  const int x = 2 * i + ((y + z + color) & 1);
  if (x >= nx || y >= ny) return;
  const int c[3] = {x, y, z};
  const int64_t idx = ((int64_t)z * ny + y) * nx + x;
  L.x[idx] = relax_value(L, c, idx, L.x);
}

template <typename T>
hipError_t launch_gs_color(const LevelView<T>& L, int color,
                           const Control* ctrl, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1) {
  if (fits3(L.g) && gs_colors(L.g) == 2) {
    const dim3 grid((unsigned)(((L.g.n[0] + 1) / 2 + k3X - 1) / k3X),
                    (unsigned)((L.g.n[1] + kColRY - 1) / kColRY),
                    (unsigned)L.g.n[2]);
    const dim3 block(k3X * kColRY);
    if (ev0 && ev1)
      hipExtLaunchKernelGGL(k_gs_color_3d<T>, grid, block, 0, s, ev0, ev1, 0,
                            L, color, ctrl);
    else
      hipLaunchKernelGGL(k_gs_color_3d<T>, grid, block, 0, s, L, color, ctrl);
    return hipGetLastError();
  }
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

// 3D form: a block covers fine cells 64 (x) x 4 (y) x 2 (z), thread t the
// two cells 2 (t % 32) + {0, 1} of row (t / 32) % 4 in plane t / 128; the
// residuals go through LDS, and each of the block's 32 x 2 coarse cells sums
// its eight children in the order of the loop above (z, y, x from the low
// corner), so the coarse right-hand side is the same to the bit.
// A block takes 64 x kRRY x 2 fine cells (kRRY even): the rows above and
// below it, which the residual stencil reads and neighbouring blocks own,
// are a smaller share of its loads than with 4 rows.
constexpr int kRRY = 8;
constexpr int kRRT = 32 * kRRY * 2;  // threads: two fine cells along x each

template <typename T>
__global__ void __launch_bounds__(kRRT)
    k_resid_restrict_3d(LevelView<T> F, LevelView<T> C,
                        double* __restrict__ partials,
                        const Control* __restrict__ ctrl) {
  __shared__ double sh[kRRT / 64];
  __shared__ T R[2][kRRY][64];
  if (ctrl->done != kRunning) return;
  const int nx = F.g.n[0], ny = F.g.n[1];
  const int t = threadIdx.x;
  const int tx = t % 32, ty = (t / 32) % kRRY, tz = t / (32 * kRRY);
  const int y = blockIdx.y * kRRY + ty, z = blockIdx.z * 2 + tz;
  double r2 = 0.0;
#pragma unroll
  for (int q0 = 0; q0 < 2; ++q0) {
    const int x = blockIdx.x * 64 + 2 * tx + q0;
    T r = T(0);
    if (x < nx && y < ny) {
      const int f[3] = {x, y, z};
      r = residual_value(F, f, ((int64_t)z * ny + y) * nx + x);
      r2 += (double)r * (double)r;
    }
    R[tz][ty][2 * tx + q0] = r;
  }
  __syncthreads();
  if (t < 32 * (kRRY / 2)) {
    const int cx = t % 32, cy = t / 32;
    const int ci = blockIdx.x * 32 + cx, cj = blockIdx.y * (kRRY / 2) + cy;
    const int ncx = C.g.n[0], ncy = C.g.n[1];
    if (ci < ncx && cj < ncy) {
      T s = T(0);
#pragma unroll
      for (int q2 = 0; q2 < 2; ++q2)
#pragma unroll
        for (int q1 = 0; q1 < 2; ++q1)
#pragma unroll
          for (int q0 = 0; q0 < 2; ++q0) s += R[q2][2 * cy + q1][2 * cx + q0];
      const int64_t idx = ((int64_t)blockIdx.z * ncy + cj) * ncx + ci;
      C.b[idx] = s / T(8);
      C.x[idx] = T(0);
    }
  }
  if (partials) {
    const double tsum = block_sum<kRRT>(r2, sh);
    if (threadIdx.x == 0) partials[block3_id()] = tsum;
  }
}

// Residual + restriction of a large 3D level marching through z: a block
// owns a tile of 64 x kRRY columns (two cells along x per thread) and walks
// a chunk of `zc` fine planes (even) upwards, keeping the iterate of the
// planes below, at and above the current one, and the face coefficient
// below it, in registers, so each plane of x and of alpha_z is fetched once
// instead of again as the neighbour of the next block's plane pair.  The
// residual takes the faces in residual_value's order (-x, +x, -y, +y, -z,
// +z) and each coarse cell sums its eight children in the same order as
// k_resid_restrict_3d.  A 1D launch: tiles are numbered x fastest, then y,
// then z chunk, and each XCD (blocks are dealt round-robin over the 8)
// takes a contiguous run of tile numbers, so a tile's neighbours in y share
// its XCD's L2.
template <typename T>
__global__ void __launch_bounds__(32 * kRRY)
    k_resid_restrict_3dm(LevelView<T> F, LevelView<T> C, int zc, int gx,
                         int gy, double* __restrict__ partials,
                         const Control* __restrict__ ctrl) {
  __shared__ double sh[32 * kRRY / 64];
  __shared__ T R[2][kRRY][64];
  if (ctrl->done != kRunning) return;
  const int nbk = gridDim.x, bk = blockIdx.x;
  const int tile = (nbk % 8 == 0) ? (bk % 8) * (nbk / 8) + bk / 8 : bk;
  const int bxi = tile % gx, byi = (tile / gx) % gy, bzi = tile / (gx * gy);
  const Geom& g = F.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2], perz = g.per[2];
  const int64_t st = (int64_t)nx * ny;
  const int t = threadIdx.x;
  const int tx = t % 32, ty = t / 32;
  const int y = byi * kRRY + ty;
  const int z0 = bzi * zc, z1 = min(z0 + zc, nz);
  bool act[2];
  int64_t col[2];
  T xm[2], x0[2], az[2], re[2] = {T(0), T(0)};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int x = bxi * 64 + 2 * tx + q;
    act[q] = x < nx && y < ny;
    col[q] = act[q] ? (int64_t)y * nx + x : 0;
    const int64_t i0 = (int64_t)z0 * st + col[q];
    x0[q] = act[q] ? F.x[i0] : T(0);
    if (!act[q]) {
      xm[q] = az[q] = T(0);
    } else if (z0 > 0) {
      xm[q] = F.x[i0 - st];
      az[q] = F.a[2][i0 - st];
    } else if (perz) {
      xm[q] = F.x[i0 + (int64_t)(nz - 1) * st];
      az[q] = F.a[2][i0 + (int64_t)(nz - 1) * st];
    } else {
      xm[q] = x0[q];
      az[q] = T(0);
    }
  }
  double r2 = 0.0;
  for (int z = z0; z < z1; ++z) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      T r = T(0);
      T xp = x0[q], au = T(0);
      if (act[q]) {
        const int64_t idx = (int64_t)z * st + col[q];
        if (z + 1 < nz)
          xp = F.x[idx + st];
        else if (perz)
          xp = F.x[col[q]];
        au = F.a[2][idx];
        const int c[3] = {bxi * 64 + 2 * tx + q, y, z};
        const T xi = x0[q];
        T ax = xi;
        for (int d = 0; d < 2; ++d) {
          const int64_t sd = d == 0 ? 1 : (int64_t)nx;
          int64_t nl, nu;
          T al, aup;
          lower_nb(g, F.a[d], d, c[d], idx, sd, nl, al);
          upper_nb(g, F.a[d], d, c[d], idx, sd, nu, aup);
          ax += al * (xi - F.x[nl]) + aup * (xi - F.x[nu]);
        }
        ax += az[q] * (xi - xm[q]) + au * (xi - xp);
        r = F.b[idx] - ax;
        r2 += (double)r * (double)r;
      }
      if ((z & 1) == 0) {
        re[q] = r;
      } else {
        R[0][ty][2 * tx + q] = re[q];
        R[1][ty][2 * tx + q] = r;
      }
      xm[q] = x0[q];
      x0[q] = xp;
      az[q] = au;
    }
    if (z & 1) {
      __syncthreads();
      if (t < 32 * (kRRY / 2)) {
        const int cx = t % 32, cy = t / 32;
        const int ci = bxi * 32 + cx, cj = byi * (kRRY / 2) + cy;
        const int ncx = C.g.n[0], ncy = C.g.n[1];
        if (ci < ncx && cj < ncy) {
          T s = T(0);
#pragma unroll
          for (int q2 = 0; q2 < 2; ++q2)
#pragma unroll
            for (int q1 = 0; q1 < 2; ++q1)
#pragma unroll
              for (int q0 = 0; q0 < 2; ++q0) s += R[q2][2 * cy + q1][2 * cx + q0];
          const int64_t idx = ((int64_t)(z >> 1) * ncy + cj) * ncx + ci;
          C.b[idx] = s / T(8);
          C.x[idx] = T(0);
        }
      }
      __syncthreads();
    }
  }
  if (partials) {
    const double tsum = block_sum<32 * kRRY>(r2, sh);
    if (threadIdx.x == 0)
      partials[bk] = tsum;
  }
}

// z planes per block of the marching residual + restriction: about 1024
// blocks in all, an even count of at least 2 (0: the one-plane-pair kernel)
int rr3_chunk(const Geom& g) {
  if (g.ndim != 3 || (g.n[2] & 1) || getenv("FLD_RR3_PAIRS")) return 0;
  const int64_t cols = (int64_t)((g.n[0] + 63) / 64) * ((g.n[1] + kRRY - 1) / kRRY);
  int64_t zc = (int64_t)g.n[2] * cols / 1024;
  zc = std::max<int64_t>(2, zc & ~(int64_t)1);
  return (int)std::min<int64_t>(zc, g.n[2]);
}

template <typename T>
hipError_t launch_resid_restrict(const LevelView<T>& fine,
                                 const LevelView<T>& coarse, double* partials,
                                 int* nblocks, const Control* ctrl,
                                 hipStream_t s) {
  // the z-marching kernel has no Dirichlet diagonal term and no held cells
  const int zc =
      fits3(fine.g) && !fine.sd && !fine.held ? rr3_chunk(fine.g) : 0;
  if (zc > 0) {
    const int gx = (fine.g.n[0] + 63) / 64, gy = (fine.g.n[1] + kRRY - 1) / kRRY;
    const int gz = (fine.g.n[2] + zc - 1) / zc;
    *nblocks = gx * gy * gz;
    hipLaunchKernelGGL(k_resid_restrict_3dm<T>, dim3(*nblocks), dim3(32 * kRRY),
                       0, s, fine, coarse, zc, gx, gy, partials, ctrl);
    return hipGetLastError();
  }
  if (fits3(fine.g)) {
    // fine blocks of 64 x kRRY x 2 cells (the fine sides are even)
    const dim3 g((fine.g.n[0] + 63) / 64, (fine.g.n[1] + kRRY - 1) / kRRY,
                 fine.g.n[2] / 2);
    *nblocks = (int)(g.x * g.y * g.z);
    hipLaunchKernelGGL(k_resid_restrict_3d<T>, g, dim3(kRRT), 0, s, fine,
                       coarse, partials, ctrl);
    return hipGetLastError();
  }
  *nblocks = blocks_for(coarse.g.N);
  hipLaunchKernelGGL(k_resid_restrict<T>, dim3(*nblocks), dim3(kBlock), 0, s,
                     fine, coarse, partials, ctrl);
  return hipGetLastError();
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
__global__ void __launch_bounds__(k3T)
    k_prolong_3d(LevelView<T> C, LevelView<T> F,
                 const Control* __restrict__ ctrl) {
  if (ctrl->done != kRunning) return;
  const int nx = F.g.n[0], ny = F.g.n[1];
  const int x = blockIdx.x * k3X + (threadIdx.x % k3X);
  const int y = blockIdx.y * k3Y + (threadIdx.x / k3X), z = blockIdx.z;
  if (x >= nx || y >= ny) return;
  const int f[3] = {x, y, z};
  F.x[((int64_t)z * ny + y) * nx + x] += prolong_value(C, f, 3);
}

template <typename T>
hipError_t launch_prolong(const LevelView<T>& coarse, const LevelView<T>& fine,
                          const Control* ctrl, hipStream_t s) {
  if (fits3(fine.g)) {
    hipLaunchKernelGGL(k_prolong_3d<T>,
                       grid3(fine.g.n[0], fine.g.n[1], fine.g.n[2]),
                       dim3(k3T), 0, s, coarse, fine, ctrl);
    return hipGetLastError();
  }
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
  // red-black Gauss-Seidel sweeps until |r| dropped by 1e-3, tested every
  // 2 sweeps (the LDS tail does the same)
  (void)tmp;
  const int64_t N = L.g.N;
  double r0 = 0.0;
  for (int it = 0; it < 4000; it += 2) {
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
    if (!(rn > 1e-6 * r0)) break;  // squared norms
    for (int sw = 0; sw < 2; ++sw)
      for (int color = 0; color < gs_colors(L.g); ++color) {
        for (int64_t i = threadIdx.x; i < N; i += kReduceBlock) {
          int c[3];
          coords(L.g, i, c);
          if (gs_color(L.g, c) == color)
            L.x[i] = relax_value(L, c, i, L.x);
        }
        __syncthreads();
      }
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
    for (int color = 0; color < gs_colors(L.g); ++color) {
      for (int64_t i = threadIdx.x; i < L.g.N; i += kReduceBlock) {
        int c[3];
        coords(L.g, i, c);
        if (gs_color(L.g, c) == color)
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
        // the host reads the outcome from the mirror after this launch
        if (stop && C->mirror) *C->mirror = *C;
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
                                         const Control*, hipStream_t,          \
                                         hipEvent_t, hipEvent_t);              \
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

__global__ void __launch_bounds__(kBlock)
    k_exchange(int64_t N, double dt, double c, double a_rad, double gm1,
               double gas_const, const double* __restrict__ rho,
               const double* __restrict__ kappa, double* __restrict__ E,
               double* __restrict__ e) {
  exchange_body(N, dt, c, a_rad, gm1, gas_const, rho, kappa, E, e, blockIdx.x);
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
              double k0, double pa, double pb, int ha, int hb, double kmin,
              double kmax, double* __restrict__ kappa) {
  opacity_body(N, gm1, gas_const, rho, e, k0, pa, pb, ha, hb, kmin, kmax,
               kappa, blockIdx.x);
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
