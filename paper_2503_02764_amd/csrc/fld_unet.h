// Kernel arguments and launchers of the U-Net (fld_unet.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fld {
namespace nn {

// 'same' convolution: out = act(bias + sum_taps in * W), NHWC views.
struct ConvArgs {
  const void* in;  // BF16 (in_f32 = 0) or FP32 (converted to BF16) input
  int in_f32;
  int N, H, W;
  int in_stride, in_off, cin_pad;  // cin_pad: multiple of 16
  const uint16_t* w;               // BF16 [taps][cout_pad][cin_pad]
  const float* bias;               // [cout] or null
  void* out;                       // BF16 (out_f32 = 0) or FP32 output view
  int out_f32;
  int out_stride, out_off, cout, cout_pad;
  int relu, accumulate, ksize;
  // 3x3 BF16 convolutions only (null: unused):
  // input channels from up_c0 on are read from up_in, nearest-upsampled by
  // 2 on the fly (channel c at (y, x) = up_in[y / 2][x / 2][c - up_c0]);
  const uint16_t* up_in;
  int up_stride, up_off, up_c0;
  // the 2x2 average pool of the (BF16) output is also written to pool_out,
  // with the roundings of the separate pool kernel
  uint16_t* pool_out;
  int pool_stride, pool_off;
};

// dW[t][co][ci] += sum_p in[p + off_t][ci] dz[p][co]
struct WgradArgs {
  const uint16_t* in;  // BF16 input view
  int in_stride, in_off, cin_pad;
  const float* dz;  // FP32 output gradient view
  int dz_stride, dz_off, cout_pad;
  float* dw;  // FP32 [taps][cout_pad][cin_pad]
  int N, H, W, ksize;
  int rows;  // set by the launcher
};

hipError_t launch_conv(const ConvArgs& a, hipStream_t s);
hipError_t launch_wgrad(const WgradArgs& a, hipStream_t s);
hipError_t launch_bgrad(const float* dz, int64_t P, int stride, int off,
                        int cout, float* db, hipStream_t s);
hipError_t launch_pool(const uint16_t* in, int is, int io, uint16_t* out,
                       int os, int oo, int N, int Ho, int Wo, int C,
                       hipStream_t s);
hipError_t launch_pool_bwd(const float* gout, int gs, int go, float* gin,
                           int is, int io, int N, int Ho, int Wo, int C,
                           hipStream_t s);
hipError_t launch_up(const uint16_t* in, int is, int io, uint16_t* out, int os,
                     int oo, int N, int Hi, int Wi, int C, hipStream_t s);
hipError_t launch_up_bwd(const float* gout, int gs, int go, float* gin, int is,
                         int io, int N, int Hi, int Wi, int C, hipStream_t s);
hipError_t launch_relu_bwd(float* g, int gs, int go, const uint16_t* a, int as,
                           int ao, int64_t P, int C, hipStream_t s);
hipError_t launch_head(const uint16_t* u, int us, int uo, const float* w,
                       const float* b, int C, int64_t P, float* delta,
                       hipStream_t s);
hipError_t launch_mse(const float* delta, const float* target, int64_t P,
                      float* g, float* loss, hipStream_t s);
// Energy-norm loss and its gradient g (see k_eloss_norms); acc: 2N floats.
hipError_t launch_energy_loss(const float* delta, const float* target,
                              const float* feats, int N, int H, int W,
                              float* acc, float* g, float* loss, hipStream_t s);
hipError_t launch_head_bwd(const float* g, const uint16_t* u, int us, int uo,
                           const float* w, int C, int64_t P, float* du,
                           int dus, int duo, float* dw, float* db,
                           hipStream_t s);
hipError_t launch_adam(float* w, uint16_t* w16, const float* g, float* m,
                       float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s);
hipError_t launch_zero(float* x, int64_t n, hipStream_t s);
hipError_t launch_to_bf16(const float* w, uint16_t* w16, int64_t n,
                          hipStream_t s);
hipError_t launch_flip(const uint16_t* w, uint16_t* wd, int taps, int cout_pad,
                       int cin_pad, hipStream_t s);
hipError_t launch_features(const double* E, const double* rho,
                           const double* kappa, const double* ax,
                           const double* ay, double dx, const double* mean_logE,
                           int64_t P, int64_t slice, uint16_t* bf16, float* f32,
                           hipStream_t s);
hipError_t launch_input(const float* in, int64_t P, uint16_t* x,
                        hipStream_t s);
// Per-slice mean of log E; scratch holds mean_log_scratch() doubles.
int64_t mean_log_scratch(int64_t slice, int nslices);
hipError_t launch_mean_log(const double* E, int64_t slice, int nslices,
                           double* mean, double* scratch, hipStream_t s);
hipError_t launch_apply_guess(const double* E, const float* delta, int64_t P,
                              double* x, hipStream_t s);

}  // namespace nn
}  // namespace fld
