// Batched forms of the per-grid kernels (see fld_batch.h): the same bodies
// as the single-grid kernels, with the block index mapped onto a grid.
#include "fld_batch.h"

namespace fld {

namespace {

// last g with start[g] <= b (start[0] = 0, increasing)
__device__ __forceinline__ int find_grid(const int* __restrict__ start,
                                         int ng, int b) {
  int lo = 0, hi = ng - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void k_ctrl_init_batch(const JobCtrl* __restrict__ tab) {
  const JobCtrl& J = tab[blockIdx.x];
  ctrl_init_body(J.ctrl, J.rtol, J.max_cycles, J.inner, J.mirror);
}

__global__ void __launch_bounds__(kBlock)
    k_coef_batch(const JobCoef* __restrict__ tab,
                 const int* __restrict__ start, int ng) {
  const int g = find_grid(start, ng, blockIdx.x);
  const JobCoef& J = tab[g];
  coef_body(J.A, J.E, J.rho, J.kappa, J.O, blockIdx.x - start[g]);
}

__global__ void __launch_bounds__(kReduceBlock)
    k_finalize_batch(int mode, const JobFinalize* __restrict__ tab) {
  const JobFinalize& J = tab[blockIdx.x];
  finalize_body(mode, J.partials, J.count, J.ctrl);
}

__global__ void __launch_bounds__(kBlock)
    k_resid_batch(const JobResid* __restrict__ tab,
                  const int* __restrict__ start, int ng) {
  const int g = find_grid(start, ng, blockIdx.x);
  const JobResid& J = tab[g];
  resid_to32_body(J.L, J.r32, J.partials, J.ctrl, blockIdx.x - start[g]);
}

__global__ void __launch_bounds__(kBlock)
    k_correct_batch(const JobCorrect* __restrict__ tab,
                    const int* __restrict__ start, int ng) {
  const int g = find_grid(start, ng, blockIdx.x);
  const JobCorrect& J = tab[g];
  correct_body(J.N, J.x, J.e, J.ctrl, blockIdx.x - start[g]);
}

__global__ void __launch_bounds__(kBlock)
    k_take_batch(const JobTake* __restrict__ tab, const int* __restrict__ start,
                 int ng) {
  const int g = find_grid(start, ng, blockIdx.x);
  const JobTake& J = tab[g];
  if (!J.ctrl->stop_in_down) return;
  const int64_t i = (int64_t)(blockIdx.x - start[g]) * kBlock + threadIdx.x;
  if (i < J.N) J.x[i] = J.alt[i];
}

__global__ void __launch_bounds__(kBlock)
    k_opacity_batch(const JobOpacity* __restrict__ tab,
                    const int* __restrict__ start, int ng) {
  const int g = find_grid(start, ng, blockIdx.x);
  const JobOpacity& J = tab[g];
  opacity_body(J.N, J.gm1, J.gas_const, J.rho, J.e, J.k0, J.pa, J.pb, J.ha,
               J.hb, J.kmin, J.kmax, J.kappa, blockIdx.x - start[g]);
}

__global__ void __launch_bounds__(kBlock)
    k_exchange_batch(const JobExchange* __restrict__ tab,
                     const int* __restrict__ start, int ng) {
  const int g = find_grid(start, ng, blockIdx.x);
  const JobExchange& J = tab[g];
  exchange_body(J.N, J.dt, J.c, J.a_rad, J.gm1, J.gas_const, J.rho, J.kappa,
                J.E, J.e, blockIdx.x - start[g]);
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_coarsen_batch(const CoarsenArgs<T>* __restrict__ tab,
                    const int* __restrict__ start, int ng) {
  const int g = find_grid(start, ng, blockIdx.x);
  coarsen_body(tab[g], blockIdx.x - start[g]);
}

}  // namespace

hipError_t launch_ctrl_init_batch(const JobCtrl* tab, int ng, hipStream_t s) {
  if (ng == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ctrl_init_batch, dim3(ng), dim3(64), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_coef_batch(const JobCoef* tab, const int* start, int ng,
                             int nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_coef_batch, dim3(nblocks), dim3(kBlock), 0, s, tab,
                     start, ng);
  return hipGetLastError();
}

hipError_t launch_finalize_batch(int mode, const JobFinalize* tab, int ng,
                                 hipStream_t s) {
  if (ng == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize_batch, dim3(ng), dim3(kReduceBlock), 0, s,
                     mode, tab);
  return hipGetLastError();
}

hipError_t launch_resid_batch(const JobResid* tab, const int* start, int ng,
                              int nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_resid_batch, dim3(nblocks), dim3(kBlock), 0, s, tab,
                     start, ng);
  return hipGetLastError();
}

hipError_t launch_correct_batch(const JobCorrect* tab, const int* start,
                                int ng, int nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_correct_batch, dim3(nblocks), dim3(kBlock), 0, s, tab,
                     start, ng);
  return hipGetLastError();
}

hipError_t launch_take_batch(const JobTake* tab, const int* start, int ng,
                             int nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_take_batch, dim3(nblocks), dim3(kBlock), 0, s, tab,
                     start, ng);
  return hipGetLastError();
}

hipError_t launch_opacity_batch(const JobOpacity* tab, const int* start,
                                int ng, int nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_opacity_batch, dim3(nblocks), dim3(kBlock), 0, s, tab,
                     start, ng);
  return hipGetLastError();
}

hipError_t launch_exchange_batch(const JobExchange* tab, const int* start,
                                 int ng, int nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_exchange_batch, dim3(nblocks), dim3(kBlock), 0, s, tab,
                     start, ng);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarsen_batch(const CoarsenArgs<T>* tab, const int* start,
                                int ng, int nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarsen_batch<T>, dim3(nblocks), dim3(kBlock), 0, s,
                     tab, start, ng);
  return hipGetLastError();
}

template hipError_t launch_coarsen_batch<double>(const CoarsenArgs<double>*,
                                                 const int*, int, int,
                                                 hipStream_t);
template hipError_t launch_coarsen_batch<float>(const CoarsenArgs<float>*,
                                                const int*, int, int,
                                                hipStream_t);

}  // namespace fld
