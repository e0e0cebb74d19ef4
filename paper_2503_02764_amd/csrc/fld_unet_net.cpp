// Host driver of the U-Net (fldnn.h): parameter layout, activation and
// gradient buffers, and the launch sequence of the forward pass, the
// backward pass and the Adam step.  All arithmetic runs in fld_unet.hip.
#include "fldnn.h"
#include "fld_unet.h"
#include "fld_unet_net.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace fld {
namespace nn {

namespace {

struct LayerDef {
  const char* name;
  int ci, co, k;
};

// The architecture of fldnn.h, in parameter order.
const LayerDef kLayers[kNumLayers] = {
    {"e0a", 4, 16, 3},    {"e0b", 16, 16, 3},   {"e1a", 16, 32, 3},
    {"e1b", 32, 32, 3},   {"e2a", 32, 64, 3},   {"e2b", 64, 64, 3},
    {"e3a", 64, 128, 3},  {"e3b", 128, 128, 3}, {"d2a", 192, 64, 3},
    {"d2b", 64, 64, 3},   {"d1a", 96, 32, 3},   {"d1b", 32, 32, 3},
    {"d0a", 48, 16, 3},   {"d0b", 16, 16, 3},   {"head", 16, 1, 1},
};

int pad16(int c) { return (c + 15) / 16 * 16; }
size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

size_t param_count() {
  size_t n = 0;
  for (const LayerDef& L : kLayers) n += (size_t)L.k * L.k * L.ci * L.co + L.co;
  return n;
}

// Device parameter layout: the 14 convolutions as [tap][co_pad][ci_pad]
// (+ bias[co_pad]), then the head weights [16] and bias [1], all FP32.
static void param_layout(size_t* woff, size_t* boff, size_t* total) {
  size_t o = 0;
  for (int i = 0; i < kNumLayers; ++i) {
    const LayerDef& L = kLayers[i];
    woff[i] = o;
    o += (size_t)L.k * L.k * pad16(L.co) * pad16(L.ci);
    boff[i] = o;
    o += pad16(L.co);
  }
  *total = o;
}

// Activation tensors: (level, channels); levels l have H >> l rows.
enum Tensor {
  T_X, T_E0A, T_C0, T_P0, T_E1A, T_C1, T_P1, T_E2A, T_C2, T_P2, T_E3A, T_BT,
  T_D2A, T_U2, T_D1A, T_U1, T_D0A, T_U0, T_COUNT
};
static const int kTLevel[T_COUNT] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3,
                                     2, 2, 1, 1, 0, 0};
static const int kTChan[T_COUNT] = {16, 16, 48, 16, 32, 96, 32, 64, 192, 64,
                                    128, 128, 64, 64, 32, 32, 16, 16};

struct Net {
  int N, H, W, training;
  hipStream_t stream;
  size_t woff[kNumLayers], boff[kNumLayers], nparam;
  float* w32;       // FP32 master parameters
  uint16_t* w16;    // BF16 copy (GEMM operands)
  float* grad;      // FP32 gradients (training)
  float* mom1;
  float* mom2;
  uint16_t* wflip;  // scratch: weights of an input-gradient convolution
  uint16_t* act[T_COUNT];
  float* gact[T_COUNT];  // training
  float* delta;     // FP32 [P0]
  float* gdelta;    // training
  float* loss;      // FP32 scalar
  float* eacc;      // energy-norm loss: per-image sums (training)
  int loss_kind;    // FLDNN_LOSS_*
  float* host_loss;
  double* mean;     // per-image mean of log E (solver features)
  std::string err;
};

static int64_t pix(const Net& n, int level) {
  return (int64_t)n.N * (n.H >> level) * (n.W >> level);
}

size_t workspace_bytes(int N, int H, int W, int training) {
  if (N < 1 || H < 8 || W < 8 || H % 8 || W % 8) return 0;
  size_t woff[kNumLayers], boff[kNumLayers], np;
  param_layout(woff, boff, &np);
  Net n{};
  n.N = N;
  n.H = H;
  n.W = W;
  size_t o = 0;
  o += align256(np * 4) + align256(np * 2) + align256(147456 * 2);
  if (training) o += 3 * align256(np * 4);
  for (int t = 0; t < T_COUNT; ++t) {
    const size_t e = (size_t)pix(n, kTLevel[t]) * kTChan[t];
    o += align256(e * 2);
    if (training && t != T_X) o += align256(e * 4);
  }
  o += align256((size_t)pix(n, 0) * 4) * (training ? 2 : 1);
  o += 256 + align256((size_t)N * 8);
  if (training) o += align256((size_t)N * 8);
  return o;
}

// zero fill by a kernel (a memset node would not replay correctly in a
// captured graph)
static hipError_t zero_f32(float* p, size_t n, hipStream_t s) {
  return launch_zero(p, (int64_t)n, s);
}

Net* create(int N, int H, int W, int training, char* ws, size_t bytes,
            hipStream_t s, std::string* err) {
  const size_t need = workspace_bytes(N, H, W, training);
  if (need == 0) {
    *err = "H and W must be multiples of 8 (>= 8), N >= 1";
    return nullptr;
  }
  if (bytes < need) {
    *err = "network workspace too small";
    return nullptr;
  }
  Net* n = new Net();
  n->N = N;
  n->H = H;
  n->W = W;
  n->training = training;
  n->stream = s;
  param_layout(n->woff, n->boff, &n->nparam);
  size_t o = 0;
  auto take = [&](size_t b) {
    char* p = ws + o;
    o += align256(b);
    return p;
  };
  n->w32 = (float*)take(n->nparam * 4);
  n->w16 = (uint16_t*)take(n->nparam * 2);
  n->wflip = (uint16_t*)take(147456 * 2);
  if (training) {
    n->grad = (float*)take(n->nparam * 4);
    n->mom1 = (float*)take(n->nparam * 4);
    n->mom2 = (float*)take(n->nparam * 4);
  }
  for (int t = 0; t < T_COUNT; ++t) {
    const size_t e = (size_t)pix(*n, kTLevel[t]) * kTChan[t];
    n->act[t] = (uint16_t*)take(e * 2);
    n->gact[t] = (training && t != T_X) ? (float*)take(e * 4) : nullptr;
  }
  n->delta = (float*)take((size_t)pix(*n, 0) * 4);
  n->gdelta = training ? (float*)take((size_t)pix(*n, 0) * 4) : nullptr;
  n->loss = (float*)take(256);
  n->mean = (double*)take((size_t)N * 8);
  n->eacc = training ? (float*)take((size_t)N * 8) : nullptr;
  n->loss_kind = FLDNN_LOSS_MSE;
  // zero everything that must start at zero (padding channels of the
  // parameters, of the input tensor, optimizer moments)
  hipError_t e = zero_f32(n->w32, n->nparam, s);
  if (e == hipSuccess) e = launch_to_bf16(n->w32, n->w16, (int64_t)n->nparam, s);
  if (e == hipSuccess && training) e = zero_f32(n->mom1, n->nparam, s);
  if (e == hipSuccess && training) e = zero_f32(n->mom2, n->nparam, s);
  if (e != hipSuccess) {
    delete n;
    *err = std::string("device error: ") + hipGetErrorString(e);
    return nullptr;
  }
  if (hipHostMalloc((void**)&n->host_loss, 256, hipHostMallocDefault) != hipSuccess) {
    delete n;
    *err = "hipHostMalloc failed";
    return nullptr;
  }
  return n;
}

void destroy(Net* n) {
  if (!n) return;
  if (n->host_loss) (void)hipHostFree(n->host_loss);
  delete n;
}

// canonical FP32 array (W[ky][kx][ci][co], b[co] per layer) <-> device layout
bool set_params(Net* n, const float* host, size_t count) {
  if (count != param_count()) return false;
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(host[i])) return false;
  std::vector<float> dev(n->nparam, 0.f);
  size_t src = 0;
  for (int i = 0; i < kNumLayers; ++i) {
    const LayerDef& L = kLayers[i];
    const int cip = pad16(L.ci), cop = pad16(L.co);
    for (int t = 0; t < L.k * L.k; ++t)
      for (int ci = 0; ci < L.ci; ++ci)
        for (int co = 0; co < L.co; ++co)
          dev[n->woff[i] + ((size_t)t * cop + co) * cip + ci] = host[src++];
    for (int co = 0; co < L.co; ++co) dev[n->boff[i] + co] = host[src++];
  }
  hipMemcpyAsync(n->w32, dev.data(), n->nparam * 4, hipMemcpyHostToDevice,
                 n->stream);
  launch_to_bf16(n->w32, n->w16, (int64_t)n->nparam, n->stream);
  if (n->training) {
    zero_f32(n->mom1, n->nparam, n->stream);
    zero_f32(n->mom2, n->nparam, n->stream);
  }
  return hipStreamSynchronize(n->stream) == hipSuccess;
}

static void to_canonical(const Net* n, const std::vector<float>& dev,
                         float* host) {
  size_t dst = 0;
  for (int i = 0; i < kNumLayers; ++i) {
    const LayerDef& L = kLayers[i];
    const int cip = pad16(L.ci), cop = pad16(L.co);
    for (int t = 0; t < L.k * L.k; ++t)
      for (int ci = 0; ci < L.ci; ++ci)
        for (int co = 0; co < L.co; ++co)
          host[dst++] = dev[n->woff[i] + ((size_t)t * cop + co) * cip + ci];
    for (int co = 0; co < L.co; ++co) host[dst++] = dev[n->boff[i] + co];
  }
}

bool get_params(Net* n, float* host, size_t count) {
  if (count != param_count()) return false;
  std::vector<float> dev(n->nparam);
  if (hipMemcpy(dev.data(), n->w32, n->nparam * 4, hipMemcpyDeviceToHost) !=
      hipSuccess)
    return false;
  to_canonical(n, dev, host);
  return true;
}

// conv layer i: input view -> output view (BF16), ReLU; optionally the
// 2x2 pool of the output to `pool` (channel stride ps) and the input's
// channels from up_c0 on read upsampled from `up` (channel stride us)
static hipError_t conv_fwd(Net* n, int i, int level, const uint16_t* in,
                           int is, int io, uint16_t* out, int os, int oo,
                           uint16_t* pool = nullptr, int ps = 0,
                           const uint16_t* up = nullptr, int us = 0,
                           int up_c0 = 0) {
  const LayerDef& L = kLayers[i];
  ConvArgs a{};
  a.in = in;
  a.in_f32 = 0;
  a.N = n->N;
  a.H = n->H >> level;
  a.W = n->W >> level;
  a.in_stride = is;
  a.in_off = io;
  a.cin_pad = pad16(L.ci);
  a.w = n->w16 + n->woff[i];
  a.bias = n->w32 + n->boff[i];
  a.out = out;
  a.out_f32 = 0;
  a.out_stride = os;
  a.out_off = oo;
  a.cout = L.co;
  a.cout_pad = pad16(L.co);
  a.relu = 1;
  a.accumulate = 0;
  a.ksize = L.k;
  a.pool_out = pool;
  a.pool_stride = ps;
  a.up_in = up;
  a.up_stride = us;
  a.up_c0 = up_c0;
  return launch_conv(a, n->stream);
}

#define NN_TRY(expr)                 \
  do {                               \
    hipError_t e_ = (expr);          \
    if (e_ != hipSuccess) return e_; \
  } while (0)

// Forward from the BF16 input tensor T_X to delta (FP32).  The encoders'
// second convolutions also write the pooled tensor the next level reads;
// without training, the decoders' first convolutions read the upsampled
// half of their input straight from the coarser level (training keeps the
// upsampled copy in the concatenation buffer: the weight gradients read it).
hipError_t forward_x(Net* n) {
  uint16_t** a = n->act;
  const int N = n->N, H = n->H, W = n->W;
  hipStream_t s = n->stream;
  const bool fuse_up = !n->training;
  NN_TRY(conv_fwd(n, 0, 0, a[T_X], 16, 0, a[T_E0A], 16, 0));
  NN_TRY(conv_fwd(n, 1, 0, a[T_E0A], 16, 0, a[T_C0], 48, 0, a[T_P0], 16));
  NN_TRY(conv_fwd(n, 2, 1, a[T_P0], 16, 0, a[T_E1A], 32, 0));
  NN_TRY(conv_fwd(n, 3, 1, a[T_E1A], 32, 0, a[T_C1], 96, 0, a[T_P1], 32));
  NN_TRY(conv_fwd(n, 4, 2, a[T_P1], 32, 0, a[T_E2A], 64, 0));
  NN_TRY(conv_fwd(n, 5, 2, a[T_E2A], 64, 0, a[T_C2], 192, 0, a[T_P2], 64));
  NN_TRY(conv_fwd(n, 6, 3, a[T_P2], 64, 0, a[T_E3A], 128, 0));
  NN_TRY(conv_fwd(n, 7, 3, a[T_E3A], 128, 0, a[T_BT], 128, 0));
  if (fuse_up) {
    NN_TRY(conv_fwd(n, 8, 2, a[T_C2], 192, 0, a[T_D2A], 64, 0, nullptr, 0,
                    a[T_BT], 128, 64));
  } else {
    NN_TRY(launch_up(a[T_BT], 128, 0, a[T_C2], 192, 64, N, H / 8, W / 8, 128, s));
    NN_TRY(conv_fwd(n, 8, 2, a[T_C2], 192, 0, a[T_D2A], 64, 0));
  }
  NN_TRY(conv_fwd(n, 9, 2, a[T_D2A], 64, 0, a[T_U2], 64, 0));
  if (fuse_up) {
    NN_TRY(conv_fwd(n, 10, 1, a[T_C1], 96, 0, a[T_D1A], 32, 0, nullptr, 0,
                    a[T_U2], 64, 32));
  } else {
    NN_TRY(launch_up(a[T_U2], 64, 0, a[T_C1], 96, 32, N, H / 4, W / 4, 64, s));
    NN_TRY(conv_fwd(n, 10, 1, a[T_C1], 96, 0, a[T_D1A], 32, 0));
  }
  NN_TRY(conv_fwd(n, 11, 1, a[T_D1A], 32, 0, a[T_U1], 32, 0));
  if (fuse_up) {
    NN_TRY(conv_fwd(n, 12, 0, a[T_C0], 48, 0, a[T_D0A], 16, 0, nullptr, 0,
                    a[T_U1], 32, 16));
  } else {
    NN_TRY(launch_up(a[T_U1], 32, 0, a[T_C0], 48, 16, N, H / 2, W / 2, 32, s));
    NN_TRY(conv_fwd(n, 12, 0, a[T_C0], 48, 0, a[T_D0A], 16, 0));
  }
  NN_TRY(conv_fwd(n, 13, 0, a[T_D0A], 16, 0, a[T_U0], 16, 0));
  NN_TRY(launch_head(a[T_U0], 16, 0, n->w32 + n->woff[14], n->w32 + n->boff[14],
                     16, pix(*n, 0), n->delta, s));
  return hipSuccess;
}

hipError_t set_input(Net* n, const float* inputs) {
  return launch_input(inputs, pix(*n, 0), n->act[T_X], n->stream);
}

// backward of conv+ReLU layer i: g_out (in place) masked by the ReLU, weight
// and bias gradients, and (if g_in) the input gradient.
static hipError_t layer_bwd(Net* n, int i, int level, const uint16_t* in,
                            int is, int io, const uint16_t* out, int os,
                            int oo, float* gout, int gs, int go, float* gin,
                            int gis, int gio) {
  const LayerDef& L = kLayers[i];
  hipStream_t s = n->stream;
  const int Hl = n->H >> level, Wl = n->W >> level;
  const int64_t P = pix(*n, level);
  const int cip = pad16(L.ci), cop = pad16(L.co);
  NN_TRY(launch_relu_bwd(gout, gs, go, out, os, oo, P, L.co, s));
  WgradArgs w{};
  w.in = in;
  w.in_stride = is;
  w.in_off = io;
  w.cin_pad = cip;
  w.dz = gout;
  w.dz_stride = gs;
  w.dz_off = go;
  w.cout_pad = cop;
  w.dw = n->grad + n->woff[i];
  w.N = n->N;
  w.H = Hl;
  w.W = Wl;
  w.ksize = L.k;
  NN_TRY(launch_wgrad(w, s));
  NN_TRY(launch_bgrad(gout, P, gs, go, L.co, n->grad + n->boff[i], s));
  if (!gin) return hipSuccess;
  const int taps = L.k * L.k;
  NN_TRY(launch_flip(n->w16 + n->woff[i], n->wflip, taps, cop, cip, s));
  ConvArgs a{};
  a.in = gout;
  a.in_f32 = 1;
  a.N = n->N;
  a.H = Hl;
  a.W = Wl;
  a.in_stride = gs;
  a.in_off = go;
  a.cin_pad = cop;
  a.w = n->wflip;
  a.bias = nullptr;
  a.out = gin;
  a.out_f32 = 1;
  a.out_stride = gis;
  a.out_off = gio;
  a.cout = L.ci;
  a.cout_pad = cip;
  a.relu = 0;
  a.accumulate = 0;
  a.ksize = L.k;
  return launch_conv(a, s);
}

// Loss and all parameter gradients (after forward_x), into n->grad.
hipError_t backward(Net* n, const float* targets, const float* inputs) {
  uint16_t** a = n->act;
  float** g = n->gact;
  const int N = n->N, H = n->H, W = n->W;
  hipStream_t s = n->stream;
  const int64_t P0 = pix(*n, 0);
  NN_TRY(zero_f32(n->grad, n->nparam, s));
  NN_TRY(zero_f32(n->loss, 1, s));
  if (n->loss_kind == FLDNN_LOSS_ENERGY)
    NN_TRY(launch_energy_loss(n->delta, targets, inputs, N, H, W, n->eacc,
                              n->gdelta, n->loss, s));
  else
    NN_TRY(launch_mse(n->delta, targets, P0, n->gdelta, n->loss, s));
  NN_TRY(launch_head_bwd(n->gdelta, a[T_U0], 16, 0, n->w32 + n->woff[14], 16,
                         P0, g[T_U0], 16, 0, n->grad + n->woff[14],
                         n->grad + n->boff[14], s));
  NN_TRY(layer_bwd(n, 13, 0, a[T_D0A], 16, 0, a[T_U0], 16, 0, g[T_U0], 16, 0,
                   g[T_D0A], 16, 0));
  NN_TRY(layer_bwd(n, 12, 0, a[T_C0], 48, 0, a[T_D0A], 16, 0, g[T_D0A], 16, 0,
                   g[T_C0], 48, 0));
  NN_TRY(launch_up_bwd(g[T_C0], 48, 16, g[T_U1], 32, 0, N, H / 2, W / 2, 32, s));
  NN_TRY(layer_bwd(n, 11, 1, a[T_D1A], 32, 0, a[T_U1], 32, 0, g[T_U1], 32, 0,
                   g[T_D1A], 32, 0));
  NN_TRY(layer_bwd(n, 10, 1, a[T_C1], 96, 0, a[T_D1A], 32, 0, g[T_D1A], 32, 0,
                   g[T_C1], 96, 0));
  NN_TRY(launch_up_bwd(g[T_C1], 96, 32, g[T_U2], 64, 0, N, H / 4, W / 4, 64, s));
  NN_TRY(layer_bwd(n, 9, 2, a[T_D2A], 64, 0, a[T_U2], 64, 0, g[T_U2], 64, 0,
                   g[T_D2A], 64, 0));
  NN_TRY(layer_bwd(n, 8, 2, a[T_C2], 192, 0, a[T_D2A], 64, 0, g[T_D2A], 64, 0,
                   g[T_C2], 192, 0));
  NN_TRY(launch_up_bwd(g[T_C2], 192, 64, g[T_BT], 128, 0, N, H / 8, W / 8, 128,
                       s));
  NN_TRY(layer_bwd(n, 7, 3, a[T_E3A], 128, 0, a[T_BT], 128, 0, g[T_BT], 128, 0,
                   g[T_E3A], 128, 0));
  NN_TRY(layer_bwd(n, 6, 3, a[T_P2], 64, 0, a[T_E3A], 128, 0, g[T_E3A], 128, 0,
                   g[T_P2], 64, 0));
  NN_TRY(launch_pool_bwd(g[T_P2], 64, 0, g[T_C2], 192, 0, N, H / 8, W / 8, 64, s));
  NN_TRY(layer_bwd(n, 5, 2, a[T_E2A], 64, 0, a[T_C2], 192, 0, g[T_C2], 192, 0,
                   g[T_E2A], 64, 0));
  NN_TRY(layer_bwd(n, 4, 2, a[T_P1], 32, 0, a[T_E2A], 64, 0, g[T_E2A], 64, 0,
                   g[T_P1], 32, 0));
  NN_TRY(launch_pool_bwd(g[T_P1], 32, 0, g[T_C1], 96, 0, N, H / 4, W / 4, 32, s));
  NN_TRY(layer_bwd(n, 3, 1, a[T_E1A], 32, 0, a[T_C1], 96, 0, g[T_C1], 96, 0,
                   g[T_E1A], 32, 0));
  NN_TRY(layer_bwd(n, 2, 1, a[T_P0], 16, 0, a[T_E1A], 32, 0, g[T_E1A], 32, 0,
                   g[T_P0], 16, 0));
  NN_TRY(launch_pool_bwd(g[T_P0], 16, 0, g[T_C0], 48, 0, N, H / 2, W / 2, 16, s));
  NN_TRY(layer_bwd(n, 1, 0, a[T_E0A], 16, 0, a[T_C0], 48, 0, g[T_C0], 48, 0,
                   g[T_E0A], 16, 0));
  NN_TRY(layer_bwd(n, 0, 0, a[T_X], 16, 0, a[T_E0A], 16, 0, g[T_E0A], 16, 0,
                   nullptr, 0, 0));
  return hipSuccess;
}

bool gradients(Net* n, float* loss, float* host, size_t count) {
  if (count != param_count() || !n->training) return false;
  std::vector<float> dev(n->nparam);
  if (hipMemcpyAsync(dev.data(), n->grad, n->nparam * 4, hipMemcpyDeviceToHost,
                     n->stream) != hipSuccess)
    return false;
  if (hipMemcpyAsync(n->host_loss, n->loss, 4, hipMemcpyDeviceToHost,
                     n->stream) != hipSuccess)
    return false;
  if (hipStreamSynchronize(n->stream) != hipSuccess) return false;
  if (loss) *loss = *n->host_loss;
  to_canonical(n, dev, host);
  return true;
}

hipError_t adam(Net* n, float lr, int step) {
  return launch_adam(n->w32, n->w16, n->grad, n->mom1, n->mom2,
                     (int64_t)n->nparam, lr, 0.9f, 0.999f, 1e-8f, step,
                     n->stream);
}

float* delta_ptr(Net* n) { return n->delta; }
uint16_t* input_ptr(Net* n) { return n->act[T_X]; }
double* mean_ptr(Net* n) { return n->mean; }
bool read_loss(Net* n, float* loss) {
  if (hipMemcpyAsync(n->host_loss, n->loss, 4, hipMemcpyDeviceToHost,
                     n->stream) != hipSuccess)
    return false;
  if (hipStreamSynchronize(n->stream) != hipSuccess) return false;
  *loss = *n->host_loss;
  return true;
}

}  // namespace nn
}  // namespace fld

// ---- C ABI ----------------------------------------------------------------

struct fldnn {
  fld::nn::Net* net;
};

namespace {
thread_local std::string g_nn_err;

fld_status nn_fail(fld_status st, const std::string& msg) {
  g_nn_err = msg;
  return st;
}

fld_status nn_dev(hipError_t e, const char* what) {
  if (e == hipSuccess) return FLD_OK;
  return nn_fail(FLD_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define NN_OK(expr)                \
  do {                             \
    const fld_status s_ = (expr);  \
    if (s_ != FLD_OK) return s_;   \
  } while (0)
}  // namespace

extern "C" {

size_t fldnn_param_count(void) { return fld::nn::param_count(); }

size_t fldnn_workspace_bytes(int32_t N, int32_t H, int32_t W, int32_t training) {
  return fld::nn::workspace_bytes(N, H, W, training);
}

const char* fldnn_last_error(void) { return g_nn_err.c_str(); }

fld_status fldnn_create(int32_t N, int32_t H, int32_t W, int32_t training,
                        void* workspace, size_t ws_bytes, void* hip_stream,
                        fldnn** out) {
  if (!out) return nn_fail(FLD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (fld::nn::workspace_bytes(N, H, W, training) == 0)
    return nn_fail(FLD_ERR_INVALID_ARG,
                   "N >= 1 and H, W multiples of 8 (>= 8) are required");
  if (!workspace || (uintptr_t)workspace % 256)
    return nn_fail(FLD_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
  std::string err;
  fld::nn::Net* n = fld::nn::create(N, H, W, training, (char*)workspace,
                                    ws_bytes, (hipStream_t)hip_stream, &err);
  if (!n) return nn_fail(FLD_ERR_WORKSPACE, err);
  *out = new fldnn{n};
  return FLD_OK;
}

fld_status fldnn_set_params(fldnn* net, const float* host, size_t count) {
  if (!net || !host) return nn_fail(FLD_ERR_INVALID_ARG, "NULL argument");
  if (count != fld::nn::param_count())
    return nn_fail(FLD_ERR_MODEL, "wrong parameter count");
  return fld::nn::set_params(net->net, host, count)
             ? FLD_OK
             : nn_fail(FLD_ERR_MODEL, "non-finite parameter or device error");
}

fld_status fldnn_get_params(fldnn* net, float* host, size_t count) {
  if (!net || !host) return nn_fail(FLD_ERR_INVALID_ARG, "NULL argument");
  if (count != fld::nn::param_count())
    return nn_fail(FLD_ERR_INVALID_ARG, "wrong parameter count");
  return fld::nn::get_params(net->net, host, count)
             ? FLD_OK
             : nn_fail(FLD_ERR_DEVICE, "copy of the parameters failed");
}

fld_status fldnn_forward(fldnn* net, const float* inputs, float* delta) {
  if (!net || !inputs || !delta)
    return nn_fail(FLD_ERR_INVALID_ARG, "NULL argument");
  fld::nn::Net* n = net->net;
  NN_OK(nn_dev(fld::nn::set_input(n, inputs), "input conversion"));
  NN_OK(nn_dev(fld::nn::forward_x(n), "forward pass"));
  const size_t bytes = (size_t)n->N * n->H * n->W * sizeof(float);
  return nn_dev(hipMemcpyAsync(delta, n->delta, bytes, hipMemcpyDeviceToDevice,
                               n->stream),
                "copy of delta");
}

fld_status fldnn_gradients(fldnn* net, const float* inputs,
                           const float* targets, float* loss_host,
                           float* grads_host, size_t count) {
  if (!net || !inputs || !targets || !grads_host)
    return nn_fail(FLD_ERR_INVALID_ARG, "NULL argument");
  fld::nn::Net* n = net->net;
  if (!n->training)
    return nn_fail(FLD_ERR_INVALID_ARG, "the network was created without training buffers");
  if (count != fld::nn::param_count())
    return nn_fail(FLD_ERR_INVALID_ARG, "wrong parameter count");
  NN_OK(nn_dev(fld::nn::set_input(n, inputs), "input conversion"));
  NN_OK(nn_dev(fld::nn::forward_x(n), "forward pass"));
  NN_OK(nn_dev(fld::nn::backward(n, targets, inputs), "backward pass"));
  return fld::nn::gradients(n, loss_host, grads_host, count)
             ? FLD_OK
             : nn_fail(FLD_ERR_DEVICE, "copy of the gradients failed");
}

fld_status fldnn_train_step(fldnn* net, const float* inputs,
                            const float* targets, float lr, int32_t step,
                            float* loss_host) {
  if (!net || !inputs || !targets || step < 1)
    return nn_fail(FLD_ERR_INVALID_ARG, "NULL argument or step < 1");
  fld::nn::Net* n = net->net;
  if (!n->training)
    return nn_fail(FLD_ERR_INVALID_ARG, "the network was created without training buffers");
  NN_OK(nn_dev(fld::nn::set_input(n, inputs), "input conversion"));
  NN_OK(nn_dev(fld::nn::forward_x(n), "forward pass"));
  NN_OK(nn_dev(fld::nn::backward(n, targets, inputs), "backward pass"));
  NN_OK(nn_dev(fld::nn::adam(n, lr, step), "Adam update"));
  if (loss_host && !fld::nn::read_loss(n, loss_host))
    return nn_fail(FLD_ERR_DEVICE, "reading the loss failed");
  return FLD_OK;
}

fld_status fldnn_set_loss(fldnn* net, int32_t kind) {
  if (!net || (kind != FLDNN_LOSS_MSE && kind != FLDNN_LOSS_ENERGY))
    return nn_fail(FLD_ERR_INVALID_ARG, "NULL network or unknown loss");
  net->net->loss_kind = kind;
  return FLD_OK;
}

void fldnn_destroy(fldnn* net) {
  if (!net) return;
  fld::nn::destroy(net->net);
  delete net;
}

}  // extern "C"
