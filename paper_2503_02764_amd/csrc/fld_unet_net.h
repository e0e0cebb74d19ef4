// Host-side U-Net object (fld_unet_net.cpp): the solver's learned guess and
// the fldnn.h C ABI both drive the network through these calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

namespace fld {
namespace nn {

constexpr int kNumLayers = 15;  // 14 convolutions + the 1x1 head

struct Net;

size_t param_count();
// Device bytes for N images of H x W (0: invalid shape).
size_t workspace_bytes(int N, int H, int W, int training);
// Carves the buffers out of `ws`; zeroes parameters and moments
// (asynchronously, on s).  Null with *err set on failure.
Net* create(int N, int H, int W, int training, char* ws, size_t bytes,
            hipStream_t s, std::string* err);
void destroy(Net* n);
// Canonical FP32 host array <-> device parameters (blocking).
bool set_params(Net* n, const float* host, size_t count);
bool get_params(Net* n, float* host, size_t count);
// FP32 [N][H][W][4] device inputs -> the BF16 input tensor.
hipError_t set_input(Net* n, const float* inputs);
// delta (FP32 [N][H][W], device) from the BF16 input tensor.
hipError_t forward_x(Net* n);
// MSE loss against targets and every parameter gradient (after forward_x).
// (inputs: the FP32 features, read by the energy-norm loss)
hipError_t backward(Net* n, const float* targets, const float* inputs);
hipError_t adam(Net* n, float lr, int step);
bool gradients(Net* n, float* loss, float* host, size_t count);
bool read_loss(Net* n, float* loss);

float* delta_ptr(Net* n);
uint16_t* input_ptr(Net* n);  // BF16 [N][H][W][16]
double* mean_ptr(Net* n);     // N doubles (per-image mean of log E)

}  // namespace nn
}  // namespace fld
