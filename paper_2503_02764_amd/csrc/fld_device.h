// Device-side helpers and kernel bodies of the FLD library, shared by the
// single-grid kernels (fld_kernels.hip) and their batched forms
// (fld_batch.hip).  A body takes its block index as an argument so that a
// batched launch can map blocks onto many grids.
#pragma once

#include <limits.h>
#include <math.h>

#include "fld_internal.h"
#include "fld_wave.h"

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

// Flux limiter lambda(R): 0 Levermore-Pomraning (eq. fld_lambda), 1 the
// diffusion value 1/3, 2 Minerbo's (named in Sect. 2 without a formula; its
// published piecewise form: 2 / (3 + sqrt(9 + 12 R^2)) for R <= 3/2,
// 1 / (1 + R + sqrt(1 + 2 R)) above, continuous at 2/9).
__device__ __forceinline__ double flux_limiter(int kind, double R) {
  if (kind == 0) return (2.0 + R) / (6.0 + 3.0 * R + R * R);
  if (kind == 1) return 1.0 / 3.0;
  return R <= 1.5 ? 2.0 / (3.0 + sqrt(9.0 + 12.0 * R * R))
                  : 1.0 / (1.0 + R + sqrt(1.0 + 2.0 * R));
}

// Sum over a block of kBlockSize threads; the result is valid in thread 0.
template <int kBlockSize>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
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

// A cell and its two neighbours along each of the first ND dimensions
// (periodic wrap, or the cell itself at a Neumann wall), taken before any
// load and without branches so that a stencil's loads issue together.
// lo_face[d] is false where the lower face is a wall (the upper face
// coefficient there is stored as 0).
template <int ND>
struct Nbrs {
  int64_t idx, lo[ND], up[ND];
  bool lo_face[ND];
};

template <int ND>
__device__ __forceinline__ Nbrs<ND> neighbours(const Geom& g, const int c[3],
                                               int64_t idx) {
  Nbrs<ND> n;
  n.idx = idx;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const int64_t st =
        d == 0 ? 1 : (d == 1 ? (int64_t)g.n[0] : (int64_t)g.n[0] * g.n[1]);
    const int64_t wrap = (int64_t)(g.n[d] - 1) * st;
    const bool per = g.per[d] != 0;
    n.lo_face[d] = c[d] > 0 || per;
    n.lo[d] = c[d] > 0 ? idx - st : (per ? idx + wrap : idx);
    n.up[d] = c[d] < g.n[d] - 1 ? idx + st : (per ? idx - wrap : idx);
  }
  return n;
}

// r = b - A x at the cell of n: the operations of residual_value in the
// same order (same bits), loads first.
template <int ND, typename T>
__device__ __forceinline__ T residual_nb(const T* const a[3],
                                         const T* __restrict__ x,
                                         const T* __restrict__ b,
                                         const Nbrs<ND>& n) {
  T xl[ND], xu[ND], al[ND], au[ND];
  const T xi = x[n.idx], bi = b[n.idx];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    xl[d] = x[n.lo[d]];
    xu[d] = x[n.up[d]];
    al[d] = a[d][n.lo[d]];
    au[d] = a[d][n.idx];
  }
  T ax = xi;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const T a_l = n.lo_face[d] ? al[d] : T(0);
    ax += a_l * (xi - xl[d]) + au[d] * (xi - xu[d]);
  }
  return bi - ax;
}

// Gauss-Seidel / Jacobi value of cell idx: (b + sum alpha x_nb) / (1 + sum alpha),
// faces taken in the order -x, +x, -y, +y, -z, +z.
template <typename T>
__device__ __forceinline__ T relax_value(const LevelView<T>& L, const int c[3],
                                         int64_t idx, const T* xs) {
  if (L.held && L.held[idx]) return T(0);  // a coarse held point
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
  if (L.sd) den += L.sd[idx];  // Dirichlet walls of this cell
  return num / den;
}

// r = b - A x at cell idx.
template <typename T>
__device__ __forceinline__ T residual_value(const LevelView<T>& L,
                                            const int c[3], int64_t idx) {
  const T xi = L.x[idx];
  if (L.held && L.held[idx]) return T(0);  // a coarse held point
  T ax = xi;
  for (int d = 0; d < L.g.ndim; ++d) {
    const int64_t st = stride_of(L.g, d);
    int64_t nl, nu;
    T al, au;
    lower_nb(L.g, L.a[d], d, c[d], idx, st, nl, al);
    upper_nb(L.g, L.a[d], d, c[d], idx, st, nu, au);
    ax += al * (xi - L.x[nl]) + au * (xi - L.x[nu]);
  }
  if (L.sd) ax += L.sd[idx] * xi;  // Dirichlet walls of this cell
  return L.b[idx] - ax;
}

__device__ __forceinline__ void ctrl_init_body(Control* ctrl, double rtol,
                                               int max_cycles, int inner,
                                               Control* mirror) {
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
    ctrl->guess_ref = 0.0;
    ctrl->guess_rejected = 0;
    ctrl->stop_in_down = 0;
    ctrl->fcg_beta = 0.0;
    ctrl->fcg_alpha = 0.0;
    ctrl->fcg_pq = 0.0;
  }
}


__device__ __forceinline__ void finalize_update(int mode, double s,
                                                Control* ctrl);

// Single-block reduction of the block partials and the stop decision; the
// control block is then copied to its host-visible mirror.
__device__ __forceinline__ void finalize_body(int mode,
                                              const double* __restrict__ partials,
                                              int count, Control* ctrl) {
  __shared__ double sh[kReduceBlock / 64];
  const int done = ctrl->done;
  if (mode == kFinCoef) {
    double v1 = 0.0, v2 = 0.0;
    for (int i = threadIdx.x; i < count; i += kReduceBlock) {
      v1 += partials[i];
      v2 += partials[count + i];
    }
    const double s1 = block_sum<kReduceBlock>(v1, sh);
    __syncthreads();
    const double s2 = block_sum<kReduceBlock>(v2, sh);
    if (threadIdx.x != 0) return;
    finalize_update(kFinBnorm, s1, ctrl);
    if (ctrl->done == kRunning) finalize_update(kFinInitial, s2, ctrl);
    if (ctrl->mirror) *ctrl->mirror = *ctrl;
    return;
  }
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
  if (mode == kFinRestart) {
    ctrl->inner = 1;
    if (r <= ctrl->rtol) ctrl->done = kConverged;
    return;
  }
  if (mode == kFinKrylov) {
    ctrl->outer += 1;
    ctrl->cycles += ctrl->inner;
    if (r <= ctrl->rtol)
      ctrl->done = kConverged;
    else if (ctrl->cycles >= ctrl->max_cycles)
      ctrl->done = kCapped;
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
  if (ctrl->done != kRunning) ctrl->stop_in_down = 1;
}


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
    double em2 = E[base + (int64_t)ghost(c[d] - 2, n, p) * st];
    double em1 = E[base + (int64_t)ghost(c[d] - 1, n, p) * st];
    double ep1 = E[base + (int64_t)ghost(c[d] + 1, n, p) * st];
    double ep2 = E[base + (int64_t)ghost(c[d] + 2, n, p) * st];
    // a Dirichlet wall's ghosts: the mirror ghosts reflected about the
    // wall value (2 E_w - E_mirror), which continue a line through E_w
    const int w = A.g.dirw[d];
    if (w & 1) {
      const double Ew = A.wall[d][0];
      if (c[d] - 2 < 0) em2 = 2.0 * Ew - em2;
      if (c[d] - 1 < 0) em1 = 2.0 * Ew - em1;
    }
    if (w & 2) {
      const double Ew = A.wall[d][1];
      if (c[d] + 1 >= n) ep1 = 2.0 * Ew - ep1;
      if (c[d] + 2 >= n) ep2 = 2.0 * Ew - ep2;
    }
    const double G = (em2 - 8.0 * em1 + 8.0 * ep1 - ep2) * A.gscale[d];
    g2 += G * G;
  }
  const double R = sqrt(g2) / (rk * E0);
  const double lam = flux_limiter(A.limiter, R);
  bad = !(E0 > 0.0) || !(rk > 0.0) || !isfinite(E0) || !isfinite(rk);
  return A.c * lam / rk;
}

struct CoefOut {
  double* a64[3];
  float* a32[3];  // FP32 copies for the mixed-precision hierarchy (or null)
  double* copy_dst;
  double* partials;
  Control* ctrl;
  // the finest level's own right-hand side (null: b is E^n itself), with
  // Dirichlet walls (A.g.dirw) E^n + sum alpha_w E_w and their diagonal
  // term sd (null without such walls), and with held cells (mask `held`,
  // null without them) the prescribed value `hold` in the held cells
  double* sd;
  double* rhs;
  const uint8_t* held;
  const double* hold;
};

// One cell's face coefficients (and its copy of E); returns E^2 and sets
// `bad` for a non-physical cell.
__device__ __forceinline__ double coef_cell(const CoefArgs& A,
                                            const double* __restrict__ E,
                                            const double* __restrict__ rho,
                                            const double* __restrict__ kappa,
                                            const CoefOut& O, const int c[3],
                                            int64_t idx, bool& bad) {
  bad = false;
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
  if (O.rhs) {
    // Dirichlet walls: the wall face lies half a cell away with this
    // cell's D, alpha_w = 2 dt D / dx^2 on the diagonal, alpha_w E_w on the
    // right-hand side; a held cell's right-hand side is its prescribed
    // value (its row is x = b).  The square norm of this b is the stop
    // test's |b|^2.
    double sd = 0.0, bw = 0.0;
    if (O.sd) {
      for (int d = 0; d < A.g.ndim; ++d) {
        const double aw = 2.0 * A.dt * D0 / (A.dx[d] * A.dx[d]);
        if ((A.g.dirw[d] & 1) && c[d] == 0) {
          sd += aw;
          bw += aw * A.wall[d][0];
        }
        if ((A.g.dirw[d] & 2) && c[d] == A.g.n[d] - 1) {
          sd += aw;
          bw += aw * A.wall[d][1];
        }
      }
      O.sd[idx] = sd;
    }
    const double bi = (O.held && O.held[idx]) ? O.hold[idx] : Ei + bw;
    O.rhs[idx] = bi;
    return bi * bi;
  }
  return Ei * Ei;
}

// The face coefficients of cell c from cell-centred D already computed for
// every cell (Dc): coef_cell's arithmetic with D read instead of recomputed.
__device__ __forceinline__ void faces_from_D(const CoefArgs& A,
                                             const double* __restrict__ Dc,
                                             const CoefOut& O, const int c[3],
                                             int64_t idx) {
  const double D0 = Dc[idx];
  for (int d = 0; d < A.g.ndim; ++d) {
    double alpha = 0.0;
    if (c[d] < A.g.n[d] - 1 || A.g.per[d]) {
      int cn[3] = {c[0], c[1], c[2]};
      cn[d] = (c[d] + 1) % A.g.n[d];
      const int64_t nidx =
          cn[0] + (int64_t)A.g.n[0] * (cn[1] + (int64_t)A.g.n[1] * cn[2]);
      const double Dn = Dc[nidx];
      const double Df =
          A.face_mean == 0 ? 0.5 * (D0 + Dn) : 2.0 * D0 * Dn / (D0 + Dn);
      alpha = A.dt * Df / (A.dx[d] * A.dx[d]);
    }
    O.a64[d][idx] = alpha;
    if (O.a32[d]) O.a32[d][idx] = (float)alpha;
  }
}

__device__ __forceinline__ void coef_body(const CoefArgs& A,
                                          const double* __restrict__ E,
                                          const double* __restrict__ rho,
                                          const double* __restrict__ kappa,
                                          const CoefOut& O, int bid) {
  __shared__ double sh[kBlock / 64];
  __shared__ int bad_count;
  if (threadIdx.x == 0) bad_count = 0;
  __syncthreads();
  const int64_t idx = (int64_t)bid * kBlock + threadIdx.x;
  double e2 = 0.0;
  if (idx < A.g.N) {
    int c[3];
    coords(A.g, idx, c);
    bool bad = false;
    e2 = coef_cell(A, E, rho, kappa, O, c, idx, bad);
    if (bad) atomicAdd(&bad_count, 1);
  }
  const double s = block_sum<kBlock>(e2, sh);
  if (threadIdx.x == 0) {
    O.partials[bid] = s;
    if (bad_count > 0) atomicAdd(&O.ctrl->flagged, bad_count);
  }
}


// Series conductance of one fine path across a coarse face: half of the face
// inside the lower coarse cell, the face on the coarse face, half of the face
// inside the upper coarse cell; 0 if any of them is 0 (a wall on the path).
template <typename T>
__device__ __forceinline__ T series_path(T a0, T a1, T a2) {
  T path = T(0);
  if (a0 > T(0) && a1 > T(0) && a2 > T(0))
    path = T(2) / (T(0.5) / a0 + T(1) / a1 + T(0.5) / a2);
  return path;
}

// Coarse face coefficient = 1/4 of the mean, over the 2^(d-1) fine paths
// crossing the coarse face, of their series conductance (series_path).
template <typename T>
struct CoarsenArgs {
  Geom f, c;
  const T* fa[3];
  T* ca[3];
};

template <typename T>
__device__ __forceinline__ void coarsen_body(const CoarsenArgs<T>& A, int bid) {
  const int64_t idx = (int64_t)bid * kBlock + threadIdx.x;
  if (idx >= A.c.N) return;
  int c[3];
  coords(A.c, idx, c);
  const int nd = A.c.ndim;
  for (int d = 0; d < nd; ++d) {
    // the coarse face between coarse cells c and c+1 along d: on a Neumann
    // wall it stays a wall
    if (c[d] == A.c.n[d] - 1 && !A.c.per[d]) {
      A.ca[d][idx] = T(0);
      continue;
    }
    T s = T(0);
    int cnt = 0;
    const int o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
    for (int q2 = 0; q2 < o2; ++q2)
      for (int q1 = 0; q1 < o1; ++q1) {
        // one fine path along d at a fixed transverse position: the face
        // inside coarse cell c (2c | 2c+1), the face on the coarse face
        // (2c+1 | 2c+2) and the face inside coarse cell c+1 (2c+2 | 2c+3),
        // conductances in series
        int f[3] = {2 * c[0], 2 * c[1], 2 * c[2]};
        const int t1 = (d == 0) ? 1 : 0;
        const int t2 = (d == 2) ? 1 : 2;
        if (nd > 1) f[t1] += q1;
        if (nd > 2) f[t2] += q2;
        T a3[3];
        for (int k = 0; k < 3; ++k) {
          int g[3] = {f[0], f[1], f[2]};
          g[d] = (2 * c[d] + k) % A.f.n[d];  // wraps only when periodic
          const int64_t fi =
              g[0] + (int64_t)A.f.n[0] * (g[1] + (int64_t)A.f.n[1] * g[2]);
          a3[k] = A.fa[d][fi];
        }
        s += series_path(a3[0], a3[1], a3[2]);
        ++cnt;
      }
    A.ca[d][idx] = T(0.25) * s / T(cnt);
  }
}


// FP64 residual of the refinement loop, handed to the FP32 hierarchy:
// r32 = (float)(b - A x) and the block sums of r^2.
__device__ __forceinline__ void resid_to32_body(
    const LevelView<double>& L, float* __restrict__ r32,
    double* __restrict__ partials, const Control* __restrict__ ctrl, int bid) {
  __shared__ double sh[kBlock / 64];
  if (ctrl->done != kRunning) return;
  const int64_t idx = (int64_t)bid * kBlock + threadIdx.x;
  double r2 = 0.0;
  if (idx < L.g.N) {
    int c[3];
    coords(L.g, idx, c);
    const double r = residual_value(L, c, idx);
    if (r32) r32[idx] = (float)r;
    r2 = r * r;
  }
  const double s = block_sum<kBlock>(r2, sh);
  if (threadIdx.x == 0) partials[bid] = s;
}


// x64 += e32 (the FP32 correction of one refinement iteration)
__device__ __forceinline__ void correct_body(int64_t N, double* __restrict__ x,
                                             const float* __restrict__ e,
                                             const Control* __restrict__ ctrl,
                                             int bid) {
  if (ctrl->done != kRunning) return;
  const int64_t i = (int64_t)bid * kBlock + threadIdx.x;
  if (i < N) x[i] += (double)e[i];
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


// Unique positive root of a4 x^4 + a1 x - c0 (a4 >= 0, a1 > 0, c0 > 0) by
// Newton from `start` (the current gas energy, usually close), capped at the
// upper bound min(c0/a1, (c0/a4)^(1/4)).  On this increasing convex function
// a start below the root steps once above it; from above the iterates fall
// monotonically onto the root.
__device__ __forceinline__ double quartic_root(double a4, double a1,
                                               double c0, double start) {
  const double u1 = c0 / a1;
  const double u4 = a4 > 0.0 ? sqrt(sqrt(c0 / a4)) : u1;
  const double ub = fmin(u1, u4);
  double x = start > 0.0 ? fmin(start, ub) : ub;
  const double lo = 0.5 * ub;  // f(lo) < 0: the root lies above it
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

__device__ __forceinline__ void exchange_body(
    int64_t N, double dt, double c, double a_rad, double gm1, double gas_const,
    const double* __restrict__ rho, const double* __restrict__ kappa,
    double* __restrict__ E, double* __restrict__ e, int bid) {
  const int64_t i = (int64_t)bid * kBlock + threadIdx.x;
  if (i >= N) return;
  const double r = rho[i];
  const double beta = dt * c * kappa[i] * r;
  const double Ei = E[i], ei = e[i];
  const double S = Ei + ei;
  const double t = gm1 / (r * gas_const);
  const double t2 = t * t;
  const double a4 = beta * a_rad * (t2 * t2);
  const double x = quartic_root(a4, 1.0 + beta, ei + beta * S, ei);
  e[i] = x;
  E[i] = S - x;
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
__device__ __forceinline__ void opacity_body(
    int64_t N, double gm1, double gas_const, const double* __restrict__ rho,
    const double* __restrict__ e, double k0, double pa, double pb, int ha,
    int hb, double kmin, double kmax, double* __restrict__ kappa, int bid) {
  const int64_t i = (int64_t)bid * kBlock + threadIdx.x;
  if (i >= N) return;
  const double r = rho[i];
  const double T = gm1 * e[i] / (r * gas_const);
  const double k = ha != INT_MIN ? k0 * pow_half(r, ha) * pow_half(T, hb)
                                 : k0 * pow(r, pa) * pow(T, pb);
  kappa[i] = fmin(fmax(k, kmin), kmax);
}


}  // namespace fld
