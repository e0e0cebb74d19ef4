/*
 * fldnn.h - the learned initial guess of the FLD diffusion solve: a small 2D
 * U-Net (BF16 matrix-core convolutions, FP32 accumulation), with inference
 * and training kernels written for gfx950.
 *
 * Not part of the paper's method: the network only proposes the starting
 * iterate E_guess = E^n (1 + delta) of the multigrid solve; the solve still
 * runs to the same tolerance, and a guess whose residual is worse than the
 * residual of E^n is discarded (fld_step with FLD_GUESS_LEARNED).
 *
 * Architecture (NHWC, 'same' 3x3 convolutions with zero padding, ReLU):
 *   encoder 4 -> 16 -> 16 | pool | 32, 32 | pool | 64, 64 | pool | 128, 128
 *   decoder up + concat skip: 192 -> 64, 64 | 96 -> 32, 32 | 48 -> 16, 16
 *   head: 1x1 convolution 16 -> 1 (delta), no activation.
 * Pooling is a 2x2 mean, upsampling 2x nearest.
 * Parameters are exchanged as one FP32 host array in layer order
 * (e0a, e0b, e1a, e1b, e2a, e2b, e3a, e3b, d2a, d2b, d1a, d1b, d0a, d0b,
 * head), each layer's weights W[ky][kx][ci][co] followed by its bias[co].
 * Network inputs: 4 FP32 channels per pixel, NHWC (see fld_step for the
 * features the solver uses).  H and W must be multiples of 8.
 */
#ifndef FLDNN_H
#define FLDNN_H

#include <stddef.h>
#include <stdint.h>

#include "fld.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fldnn fldnn;

/* Number of FP32 values in the parameter array. */
size_t fldnn_param_count(void);

/* Device workspace for a network on N images of H x W (training = 1 also
 * holds gradients and optimizer moments); 0 if the shape is invalid. */
size_t fldnn_workspace_bytes(int32_t N, int32_t H, int32_t W, int32_t training);

/* Carve a network out of `workspace` (device, 256-byte aligned).  The
 * parameters start at zero: set them with fldnn_set_params. */
fld_status fldnn_create(int32_t N, int32_t H, int32_t W, int32_t training,
                        void* workspace, size_t ws_bytes, void* hip_stream,
                        fldnn** out);

/* Copy `count` FP32 parameters from / to host memory (count must equal
 * fldnn_param_count()).  set_params also resets the optimizer moments. */
fld_status fldnn_set_params(fldnn* net, const float* host, size_t count);
fld_status fldnn_get_params(fldnn* net, float* host, size_t count);

/* delta = net(inputs): inputs device FP32 [N][H][W][4], delta device FP32
 * [N][H][W].  Asynchronous. */
fld_status fldnn_forward(fldnn* net, const float* inputs, float* delta);

/* Training loss.  FLDNN_LOSS_MSE: mean of (delta - target)^2.
 * FLDNN_LOSS_ENERGY: the inputs must be fld_features and the targets
 * delta* = (E* - E^n) / E^n of the solve; with E = exp(f0), face
 * coefficients alpha = expm1(4 f2), expm1(4 f3) and the guess error
 * e = E (delta - delta*), the loss is the mean over images of
 * |e|_A^2 / |E delta*|_A^2, |v|_A^2 = sum v^2 + sum_faces alpha dv^2 (the
 * energy norm of the backward-Euler operator; faces inside each image).
 * The second norm is that of the plain guess E^n, so the loss is 1 for
 * delta = 0 and 0 for a perfect guess. */
typedef enum { FLDNN_LOSS_MSE = 0, FLDNN_LOSS_ENERGY = 1 } fldnn_loss;
fld_status fldnn_set_loss(fldnn* net, int32_t kind);

/* The training loss (fldnn_set_loss; MSE by default) against targets
 * (device FP32 [N][H][W]) and its gradient with respect to every
 * parameter, written to host memory in the parameter layout.  Blocks.
 * Needs training = 1. */
fld_status fldnn_gradients(fldnn* net, const float* inputs,
                           const float* targets, float* loss_host,
                           float* grads_host, size_t count);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the loss above;
 * `step` counts from 1.  loss_host (nullable) receives the loss before the
 * update; non-null makes the call block. */
fld_status fldnn_train_step(fldnn* net, const float* inputs,
                            const float* targets, float lr, int32_t step,
                            float* loss_host);

void fldnn_destroy(fldnn* net);

/* Message of the last failed fldnn_* call on this thread ("" if none). */
const char* fldnn_last_error(void);

/* The network inputs fld_step computes for its learned guess, for training:
 * per cell, FP32 [4] = (log E - mean over the cell's z-slice of log E,
 * log(rho kappa dx[0]) / 4, log(1 + alpha_x) / 4, log(1 + alpha_y) / 4),
 * where alpha_d = dt D_face / dx_d^2 are the face coefficients of the
 * backward-Euler operator (eq. for the diffusion coefficient with the flux
 * limiter, Sect. 2; the face of a cell toward +d, 0 on a Neumann wall).
 * rho, kappa, E: device FP64 fields of the context's grid; out: device FP32
 * [cells][4], x fastest.  ndim >= 2 (3D: one image per z-slice).  Uses the
 * context's workspace; asynchronous on its stream. */
fld_status fld_features(fld_ctx* ctx, double dt, const double* rho,
                        const double* kappa, const double* E, float* out);

/* Give a solver context a trained network (for FLD_GUESS_LEARNED).  The
 * context must have been set up with guess = FLD_GUESS_LEARNED, whose
 * workspace includes the network.  FLD_ERR_MODEL if count is wrong or a
 * parameter is not finite. */
fld_status fld_set_model(fld_ctx* ctx, const float* host, size_t count);

#ifdef __cplusplus
}
#endif
#endif /* FLDNN_H */
