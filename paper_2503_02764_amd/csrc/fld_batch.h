// Batched forms of the per-grid kernels: one launch covers many independent
// grids.  Each launch reads a table of per-grid arguments from device memory;
// for kernels with many blocks per grid, block b belongs to the grid g with
// start[g] <= b < start[g + 1] (start[] in device memory, ng + 1 entries).
#pragma once

#include "fld_device.h"

namespace fld {

struct JobCtrl {
  Control* ctrl;
  double rtol;
  int max_cycles, inner;
  Control* mirror;
};

struct JobCoef {
  CoefArgs A;
  const double* E;
  const double* rho;
  const double* kappa;
  CoefOut O;
};

struct JobFinalize {
  const double* partials;
  int count;
  Control* ctrl;
};

struct JobResid {  // FP64 residual (to an FP32 rhs, or only its norm)
  LevelView<double> L;
  float* r32;  // null: norm only
  double* partials;
  Control* ctrl;
};

struct JobCorrect {
  int64_t N;
  double* x;
  const float* e;
  Control* ctrl;
};

struct JobTake {  // x = alt where the grid stopped after its finest down pass
  int64_t N;
  const double* alt;
  double* x;
  const Control* ctrl;
};

struct JobOpacity {
  int64_t N;
  double gm1, gas_const;
  const double* rho;
  const double* e;
  double k0, pa, pb;
  int ha, hb;
  double kmin, kmax;
  double* kappa;
};

struct JobExchange {
  int64_t N;
  double dt, c, a_rad, gm1, gas_const;
  const double* rho;
  const double* kappa;
  double* E;
  double* e;
};

hipError_t launch_ctrl_init_batch(const JobCtrl* tab, int ng, hipStream_t s);
hipError_t launch_coef_batch(const JobCoef* tab, const int* start, int ng,
                             int nblocks, hipStream_t s);
hipError_t launch_finalize_batch(int mode, const JobFinalize* tab, int ng,
                                 hipStream_t s);
hipError_t launch_resid_batch(const JobResid* tab, const int* start, int ng,
                              int nblocks, hipStream_t s);
hipError_t launch_correct_batch(const JobCorrect* tab, const int* start,
                                int ng, int nblocks, hipStream_t s);
hipError_t launch_take_batch(const JobTake* tab, const int* start, int ng,
                             int nblocks, hipStream_t s);
hipError_t launch_opacity_batch(const JobOpacity* tab, const int* start,
                                int ng, int nblocks, hipStream_t s);
hipError_t launch_exchange_batch(const JobExchange* tab, const int* start,
                                 int ng, int nblocks, hipStream_t s);
template <typename T>
hipError_t launch_coarsen_batch(const CoarsenArgs<T>* tab, const int* start,
                                int ng, int nblocks, hipStream_t s);

}  // namespace fld
