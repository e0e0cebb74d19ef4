// Hooks of a single-grid context for the block-adaptive step (fld_amr.cpp),
// defined in fld_capi.cpp: the context's FP64 V-cycle as a preconditioner
// on its own (base) grid.
#pragma once

#include <hip/hip_runtime.h>

#include "fld.h"

namespace fld {

// Face coefficients of the context's grid from (E, rho, kappa) (device
// arrays of its cells), their coarse levels, and a control block armed for
// V-cycles without a stop test.
fld_status precond_begin(fld_ctx* c, double dt, const double* E,
                         const double* rho, const double* kappa);
// One V-cycle for A z = rhs from z = 0 (device arrays of the grid's cells),
// enqueued on the context's stream.
fld_status precond_vcycle(fld_ctx* c, const double* rhs, double* z);
// The finest level's face coefficients along x and y (alpha between a cell
// and its upper neighbour), as precond_begin computed them.
void base_faces(const fld_ctx* c, const double** ax, const double** ay);
// Leaves the preconditioner mode.
void precond_end(fld_ctx* c);
hipStream_t ctx_stream(const fld_ctx* c);
const char* ctx_error(const fld_ctx* c);

}  // namespace fld
