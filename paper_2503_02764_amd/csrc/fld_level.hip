// Small 3D multigrid levels in one workgroup (gfx950).
//
// On a level of a few thousand cells every colour pass of the smoother is a
// launch whose cost is its issue and memory latency, not its bytes: with
// several sweeps per pass of the V-cycle (Sect. 3's multigrid solve of the
// backward-Euler system), a 16^3 level takes two dozen such launches per
// cycle.  Here one workgroup of kLvT threads holds the whole level: the
// iterate in LDS, each thread's cells' right-hand side and face
// coefficients in registers, and the colour passes are separated by block
// barriers only.
//
//   down: pre-smoothing, residual, restriction (coarse rhs = mean of the
//         eight children's residuals, coarse x = 0), one launch;
//   up:   trilinear prolongation of the coarse correction, post-smoothing,
//         one launch.
//
// Every cell gets the operations of the colour-pass, residual-restriction
// and prolongation kernels in the same order (relax_value, residual_value,
// prolong_value; the children summed z, y, x from the low corner), so the
// results are the same to the bit.
#include "fld_internal.h"
#include "fld_device.h"

namespace fld {

namespace {

constexpr int kLvT = 1024;                  // threads of the workgroup
constexpr int kLvCpt = kLevelLdsCells / kLvT;  // cells per thread

template <typename T>
struct LvCell {
  T b, al[3], au[3];
  int pc;     // coordinates, 10 bits each (sides <= 1024)
  int color;
};

// right-hand side, faces (lower_nb / upper_nb rules) and colour of cell i
template <typename T>
__device__ __forceinline__ void lv_load(const LevelView<T>& L, int i,
                                        LvCell<T>& c) {
  int cc[3];
  coords(L.g, i, cc);
  c.b = L.b[i];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t st = stride_of(L.g, d);
    int64_t nb;
    lower_nb(L.g, L.a[d], d, cc[d], (int64_t)i, st, nb, c.al[d]);
    upper_nb(L.g, L.a[d], d, cc[d], (int64_t)i, st, nb, c.au[d]);
  }
  c.pc = cc[0] | (cc[1] << 10) | (cc[2] << 20);
  c.color = gs_color(L.g, cc);
}

// lower and upper neighbour of cell i along d (lower_nb / upper_nb)
__device__ __forceinline__ void lv_nb(const Geom& g, int i, int pc, int d,
                                      int& nl, int& nu) {
  const int cd = (pc >> (10 * d)) & 1023, n = g.n[d];
  const int st = d == 0 ? 1 : (d == 1 ? g.n[0] : g.n[0] * g.n[1]);
  nl = cd > 0 ? i - st : (g.per[d] ? i + (n - 1) * st : i);
  nu = cd < n - 1 ? i + st : (g.per[d] ? i - (n - 1) * st : i);
}

// relax_value with the iterate in LDS
template <typename T>
__device__ __forceinline__ T lv_relax(const Geom& g, int i, const LvCell<T>& c,
                                      const T* xs) {
  T num = c.b, den = T(1);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int nl, nu;
    lv_nb(g, i, c.pc, d, nl, nu);
    num += c.al[d] * xs[nl] + c.au[d] * xs[nu];
    den += c.al[d] + c.au[d];
  }
  return num / den;
}

template <typename T>
__device__ __forceinline__ void lv_smooth(const Geom& g, const LvCell<T> (&cl)[kLvCpt],
                                          T* xs, int N, int sweeps) {
  const int ncol = gs_colors(g);
  for (int s = 0; s < sweeps; ++s)
    for (int col = 0; col < ncol; ++col) {
#pragma unroll
      for (int k = 0; k < kLvCpt; ++k) {
        const int i = threadIdx.x + k * kLvT;
        if (i < N && cl[k].color == col) xs[i] = lv_relax(g, i, cl[k], xs);
      }
      __syncthreads();
    }
}

}  // namespace

template <typename T>
__global__ void __launch_bounds__(kLvT)
    k_level_down(LevelView<T> F, LevelView<T> C, int sweeps,
                 const Control* __restrict__ ctrl) {
  __shared__ T xs[kLevelLdsCells];
  __shared__ T rs[kLevelLdsCells];
  if (ctrl->done != kRunning) return;
  const int N = (int)F.g.N;
  LvCell<T> cl[kLvCpt];
#pragma unroll
  for (int k = 0; k < kLvCpt; ++k) {
    const int i = threadIdx.x + k * kLvT;
    if (i < N) {
      lv_load(F, i, cl[k]);
      xs[i] = F.x[i];
    }
  }
  __syncthreads();
  lv_smooth(F.g, cl, xs, N, sweeps);
  // residual_value on the smoothed iterate, which also goes back to HBM
#pragma unroll
  for (int k = 0; k < kLvCpt; ++k) {
    const int i = threadIdx.x + k * kLvT;
    if (i < N) {
      const T xi = xs[i];
      T ax = xi;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int nl, nu;
        lv_nb(F.g, i, cl[k].pc, d, nl, nu);
        ax += cl[k].al[d] * (xi - xs[nl]) + cl[k].au[d] * (xi - xs[nu]);
      }
      rs[i] = cl[k].b - ax;
      F.x[i] = xi;
    }
  }
  __syncthreads();
  // coarse rhs = mean of the eight children's residuals, coarse x = 0
  const int Nc = (int)C.g.N;
  for (int I = threadIdx.x; I < Nc; I += kLvT) {
    int c[3];
    coords(C.g, I, c);
    T s = T(0);
    for (int q2 = 0; q2 < 2; ++q2)
      for (int q1 = 0; q1 < 2; ++q1)
        for (int q0 = 0; q0 < 2; ++q0) {
          const int fi = 2 * c[0] + q0 +
                         F.g.n[0] * (2 * c[1] + q1 + F.g.n[1] * (2 * c[2] + q2));
          s += rs[fi];
        }
    C.b[I] = s / T(8);
    C.x[I] = T(0);
  }
}

template <typename T>
__global__ void __launch_bounds__(kLvT)
    k_level_up(LevelView<T> F, LevelView<T> C, int sweeps,
               const Control* __restrict__ ctrl) {
  __shared__ T xs[kLevelLdsCells];
  if (ctrl->done != kRunning) return;
  const int N = (int)F.g.N;
  LvCell<T> cl[kLvCpt];
#pragma unroll
  for (int k = 0; k < kLvCpt; ++k) {
    const int i = threadIdx.x + k * kLvT;
    if (i < N) {
      lv_load(F, i, cl[k]);
      int f[3];
      coords(F.g, i, f);
      T x = F.x[i];
      x += prolong_value(C, f, 3);
      xs[i] = x;
    }
  }
  __syncthreads();
  lv_smooth(F.g, cl, xs, N, sweeps);
#pragma unroll
  for (int k = 0; k < kLvCpt; ++k) {
    const int i = threadIdx.x + k * kLvT;
    if (i < N) F.x[i] = xs[i];
  }
}

bool level_lds_ok(const Geom& g, const Geom& coarse) {
  if (g.ndim != 3 || g.N > kLevelLdsCells || g.N < 1) return false;
  for (int d = 0; d < 3; ++d)
    if (g.n[d] > 1024) return false;  // packed coordinates
  for (int d = 0; d < 3; ++d)
    if (coarse.n[d] * 2 != g.n[d]) return false;
  return true;
}

template <typename T>
hipError_t launch_level_down(const LevelView<T>& F, const LevelView<T>& C,
                             int sweeps, const Control* ctrl, hipStream_t s) {
  if (!level_lds_ok(F.g, C.g)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_level_down<T>, dim3(1), dim3(kLvT), 0, s, F, C, sweeps,
                     ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_level_up(const LevelView<T>& F, const LevelView<T>& C,
                           int sweeps, const Control* ctrl, hipStream_t s) {
  if (!level_lds_ok(F.g, C.g)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_level_up<T>, dim3(1), dim3(kLvT), 0, s, F, C, sweeps,
                     ctrl);
  return hipGetLastError();
}

template hipError_t launch_level_down<double>(const LevelView<double>&,
                                              const LevelView<double>&, int,
                                              const Control*, hipStream_t);
template hipError_t launch_level_down<float>(const LevelView<float>&,
                                             const LevelView<float>&, int,
                                             const Control*, hipStream_t);
template hipError_t launch_level_up<double>(const LevelView<double>&,
                                            const LevelView<double>&, int,
                                            const Control*, hipStream_t);
template hipError_t launch_level_up<float>(const LevelView<float>&,
                                           const LevelView<float>&, int,
                                           const Control*, hipStream_t);

}  // namespace fld
