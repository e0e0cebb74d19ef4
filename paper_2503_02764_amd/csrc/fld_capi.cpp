// C ABI of the FLD library: parameter validation, workspace layout, the
// multigrid level list and the host driver of the V-cycles.
//
// The solve runs entirely in the kernels of fld_kernels.hip and
// fld_tile2d.hip.  The host only enqueues launches on the caller's stream
// and, once per batch of cycles, reads back the control block to learn
// whether the device-side stop test (relative residual <= rtol, or the
// cycle cap) has fired.
//
// Two solvers:
//   FP64:     V-cycles on the FP64 operator, residual tested after the
//             finest-level pre-smoothing of every cycle.
//   FP32_IR:  iterative refinement. Each outer iteration computes the FP64
//             residual r = b - A x (and tests it), solves A e = r with
//             `inner` FP32 V-cycles from e = 0 on FP32 copies of the face
//             coefficients, and adds e to the FP64 iterate.
#include "fld.h"
#include "fld_internal.h"
#include "fld_tile2d.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace fld;

namespace {

template <typename T>
struct Levels {
  T* x[kMaxLevels] = {};
  T* b[kMaxLevels] = {};
  T* a[kMaxLevels][3] = {};
  T* tmp = nullptr;  // coarsest-level scratch (global-memory tail only)
};

}  // namespace

struct fld_ctx {
  fld_params p;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int L = 0;
  Geom geom[kMaxLevels];
  Levels<double> h64;          // FP64 hierarchy (level 0 only in FP32_IR)
  Levels<float> h32;           // FP32 hierarchy (FP32_IR only)
  double* bcopy = nullptr;     // level-0 rhs copy when E_out aliases E_in
  double* partials = nullptr;  // block partial sums
  Control* ctrl = nullptr;     // device control block
  Control* host_ctrl = nullptr;  // pinned host mirror, written by the GPU
  Control* host_ctrl_dev = nullptr;  // its device-side address
  bool mixed = false;
  int inner = 2;               // FP32 V-cycles per refinement iteration
  int last_batch = 4;          // cycles (or outer iterations) last step
  std::string err;
  // timing of the dominant kernel (finest-level down pass)
  bool timing = false;
  double t_ms = 0.0;
  int64_t t_launches = 0;
  double t_bytes = 0.0;
  const char* t_name = "none";
  std::vector<hipEvent_t> ev;    // pool, used in (start, stop) pairs
  std::vector<double> ev_bytes;  // algorithmic bytes of each timed launch
  size_t ev_used = 0;
  bool fast = true;  // tiled kernels + single-workgroup tail
  int tail_l0 = 0;   // first level handled by the single-workgroup tail
};

namespace {

thread_local std::string g_err;

fld_status fail(fld_ctx* ctx, fld_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx)
    ctx->err = buf;
  else
    g_err = buf;
  return st;
}

#define HIP_TRY(ctx, expr)                                                   \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return fail(ctx, FLD_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define FLD_TRY(expr)              \
  do {                             \
    fld_status s_ = (expr);        \
    if (s_ != FLD_OK) return s_;   \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int64_t kMaxCoarsestCells = 1 << 16;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Plan {
  int L = 0;
  Geom g[kMaxLevels];
  size_t a64[kMaxLevels][3] = {}, x64[kMaxLevels] = {}, b64[kMaxLevels] = {};
  size_t a32[kMaxLevels][3] = {}, x32[kMaxLevels] = {}, b32[kMaxLevels] = {};
  size_t bcopy = 0, partials = 0, tmp = 0, ctrl = 0;
  int64_t n_partials = 0;
  size_t total = 0;
};

// Returns an empty string when the parameters are valid.
std::string validate(const fld_params* p) {
  char buf[256];
  if (!p) return "params is NULL";
  if (p->ndim < 1 || p->ndim > 3) return "ndim must be 1, 2 or 3";
  int64_t N = 1;
  for (int d = 0; d < 3; ++d) {
    if (d < p->ndim) {
      if (p->n[d] < 1) {
        snprintf(buf, sizeof buf, "n[%d] must be >= 1", d);
        return buf;
      }
      if (!(p->dx[d] > 0.0) || !std::isfinite(p->dx[d])) {
        snprintf(buf, sizeof buf, "dx[%d] must be positive and finite", d);
        return buf;
      }
      if (p->bc_lo[d] < 0 || p->bc_lo[d] > 1 || p->bc_hi[d] < 0 ||
          p->bc_hi[d] > 1) {
        snprintf(buf, sizeof buf, "bc[%d]: only periodic and neumann", d);
        return buf;
      }
      if ((p->bc_lo[d] == FLD_BC_PERIODIC) != (p->bc_hi[d] == FLD_BC_PERIODIC)) {
        snprintf(buf, sizeof buf, "bc[%d]: periodic must be set on both sides", d);
        return buf;
      }
      if (p->bc_lo[d] == FLD_BC_NEUMANN && p->n[d] < 2) {
        snprintf(buf, sizeof buf, "n[%d] must be >= 2 with Neumann walls", d);
        return buf;
      }
      if (p->n[d] > (int64_t)1 << 30) return "n too large";
      N *= p->n[d];
    } else if (p->n[d] != 1) {
      snprintf(buf, sizeof buf, "n[%d] must be 1 for ndim=%d", d, p->ndim);
      return buf;
    }
  }
  if (N > (int64_t)INT32_MAX) return "more than 2^31-1 cells";
  if (!(p->c > 0.0) || !std::isfinite(p->c)) return "c must be > 0";
  if (!(p->a_rad > 0.0) || !std::isfinite(p->a_rad)) return "a_rad must be > 0";
  if (!(p->gamma > 1.0) || !std::isfinite(p->gamma)) return "gamma must be > 1";
  if (!(p->gas_const > 0.0) || !std::isfinite(p->gas_const))
    return "gas_const must be > 0";
  if (p->limiter < 0 || p->limiter > 1) return "unknown limiter";
  if (p->face_mean < 0 || p->face_mean > 1) return "unknown face mean";
  if (p->precision != FLD_PREC_FP64 && p->precision != FLD_PREC_FP32_IR)
    return "unknown precision";
  if (p->guess != FLD_GUESS_PREV && p->guess != FLD_GUESS_ZERO)
    return "guess: only FLD_GUESS_PREV and FLD_GUESS_ZERO are built";
  if (!(p->rtol > 0.0) || !(p->rtol < 1.0)) return "rtol must be in (0, 1)";
  if (p->max_cycles < 1) return "max_cycles must be >= 1";
  if (p->pre_smooth < 0 || p->post_smooth < 0 ||
      p->pre_smooth + p->post_smooth < 1 || p->pre_smooth > 16 ||
      p->post_smooth > 16)
    return "pre_smooth/post_smooth must be in [0, 16], not both 0";
  return "";
}

void make_plan(const fld_params* p, Plan* P) {
  Geom g;
  g.ndim = p->ndim;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = (int)p->n[d];
    g.per[d] = (d < p->ndim && p->bc_lo[d] == FLD_BC_PERIODIC) ? 1 : 0;
  }
  g.N = (int64_t)g.n[0] * g.n[1] * g.n[2];
  P->L = 0;
  while (true) {
    P->g[P->L++] = g;
    if (P->L == kMaxLevels) break;
    bool ok = true;
    for (int d = 0; d < g.ndim; ++d)
      if ((g.n[d] & 1) || g.n[d] / 2 < 3) ok = false;
    if (!ok) break;
    for (int d = 0; d < g.ndim; ++d) g.n[d] /= 2;
    g.N = (int64_t)g.n[0] * g.n[1] * g.n[2];
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  const int nd = p->ndim;
  const bool mixed = p->precision == FLD_PREC_FP32_IR;
  for (int l = 0; l < P->L; ++l) {
    const size_t cells = (size_t)P->g[l].N;
    if (l == 0 || !mixed) {
      for (int d = 0; d < nd; ++d) P->a64[l][d] = take(cells * 8);
      if (l > 0) {
        P->x64[l] = take(cells * 8);
        P->b64[l] = take(cells * 8);
      }
    }
    if (mixed) {
      for (int d = 0; d < nd; ++d) P->a32[l][d] = take(cells * 4);
      P->x32[l] = take(cells * 4);
      P->b32[l] = take(cells * 4);
    }
  }
  P->bcopy = take((size_t)P->g[0].N * 8);
  int64_t nparts = blocks_for(P->g[0].N);
  if (p->ndim == 2)
    for (int nu = 1; nu <= 3; ++nu) {
      const int64_t t = tile2d_blocks(P->g[0], nu, true);
      if (t > nparts) nparts = t;
    }
  P->n_partials = nparts + 64;
  P->partials = take((size_t)P->n_partials * 8);
  P->tmp = take((size_t)P->g[P->L - 1].N * 8);
  P->ctrl = take(sizeof(Control));
  P->total = o;
}

template <typename T>
LevelView<T> view(const fld_ctx* c, const Levels<T>& H, int l) {
  LevelView<T> v;
  v.g = c->geom[l];
  v.x = H.x[l];
  v.b = H.b[l];
  for (int d = 0; d < 3; ++d) v.a[d] = H.a[l][d];
  return v;
}

hipEvent_t next_event(fld_ctx* c) {
  if (c->ev_used == c->ev.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev.push_back(e);
  }
  return c->ev[c->ev_used++];
}

// Event pair around one launch of the timed kernel.
struct TimedLaunch {
  fld_ctx* c;
  hipEvent_t e1 = nullptr;
  fld_status st = FLD_OK;
  TimedLaunch(fld_ctx* cc, bool on, double bytes, const char* name) : c(cc) {
    if (!on || !c->timing) return;
    hipEvent_t e0 = next_event(c);
    e1 = next_event(c);
    if (!e0 || !e1) {
      st = fail(c, FLD_ERR_DEVICE, "hipEventCreate failed");
      e1 = nullptr;
      return;
    }
    c->ev_bytes.push_back(bytes);
    c->t_name = name;
    if (hipEventRecord(e0, c->stream) != hipSuccess)
      st = fail(c, FLD_ERR_DEVICE, "hipEventRecord failed");
  }
  fld_status close() {
    if (e1 && hipEventRecord(e1, c->stream) != hipSuccess)
      return fail(c, FLD_ERR_DEVICE, "hipEventRecord failed");
    return st;
  }
};

bool tile_path(const fld_ctx* c) {
  return c->fast && c->p.ndim == 2 && c->p.pre_smooth >= 1 &&
         c->p.pre_smooth <= 3 && c->p.post_smooth >= 1 &&
         c->p.post_smooth <= 3;
}

template <typename T>
fld_status fill_zero(fld_ctx* c, T* x, int64_t n);

template <>
fld_status fill_zero<double>(fld_ctx* c, double* x, int64_t n) {
  HIP_TRY(c, launch_fill(x, n, 0.0, c->stream));
  return FLD_OK;
}

template <>
fld_status fill_zero<float>(fld_ctx* c, float* x, int64_t n) {
  HIP_TRY(c, launch_fill32(x, n, c->stream));
  return FLD_OK;
}

// Simple path: one launch per colour pass.
template <typename T>
fld_status smooth_simple(fld_ctx* c, const Levels<T>& H, int l, int sweeps) {
  LevelView<T> v = view(c, H, l);
  for (int s = 0; s < sweeps; ++s)
    for (int color = 0; color < 2; ++color)
      HIP_TRY(c, launch_gs_color<T>(v, color, c->ctrl, c->stream));
  return FLD_OK;
}

// Down pass on level l (above the tail): pre-smoothing, residual,
// restriction.  `zero_init`: x starts at zero.  On the finest FP64 level
// the residual norm feeds the stop test.
template <typename T>
fld_status down(fld_ctx* c, const Levels<T>& H, int l, bool zero_init) {
  const bool norm = (sizeof(T) == 8) && l == 0;
  int nb = 0;
  if (tile_path(c)) {
    Tile2DArgs<T> a{};
    a.g = c->geom[l];
    a.x = H.x[l];
    a.b = H.b[l];
    a.ax = H.a[l][0];
    a.ay = H.a[l][1];
    a.gc = c->geom[l + 1];
    a.cb = H.b[l + 1];
    a.ce = nullptr;
    a.partials = norm ? c->partials : nullptr;
    a.zero_init = zero_init;
    a.ctrl = c->ctrl;
    // x (unless zero), b, two face arrays read; x and the coarse rhs written
    const double w = sizeof(T);
    const double bytes = (double)c->geom[l].N *
                         (w * (zero_init ? 4.0 : 5.0) + w / 4.0);
    TimedLaunch t(c, l == 0, bytes,
                  sizeof(T) == 8 ? "k_tile2d<double,down>" : "k_tile2d<float,down>");
    FLD_TRY(t.st);
    HIP_TRY(c, launch_tile2d<T>(a, c->p.pre_smooth, true, c->stream, &nb));
    FLD_TRY(t.close());
  } else {
    if (zero_init && l == 0) FLD_TRY(fill_zero<T>(c, H.x[0], c->geom[0].N));
    FLD_TRY(smooth_simple<T>(c, H, l, c->p.pre_smooth));
    HIP_TRY(c, launch_resid_restrict<T>(view(c, H, l), view(c, H, l + 1),
                                        norm ? c->partials : nullptr, &nb,
                                        c->ctrl, c->stream));
  }
  if (norm)
    HIP_TRY(c, launch_finalize(kFinCycle, c->partials, nb, c->ctrl, c->stream));
  return FLD_OK;
}

// Up pass on level l: prolongation of level l+1 and post-smoothing.
template <typename T>
fld_status up(fld_ctx* c, const Levels<T>& H, int l) {
  if (tile_path(c)) {
    Tile2DArgs<T> a{};
    a.g = c->geom[l];
    a.x = H.x[l];
    a.b = H.b[l];
    a.ax = H.a[l][0];
    a.ay = H.a[l][1];
    a.gc = c->geom[l + 1];
    a.cb = nullptr;
    a.ce = H.x[l + 1];
    a.partials = nullptr;
    a.zero_init = 0;
    a.ctrl = c->ctrl;
    int nb = 0;
    HIP_TRY(c, launch_tile2d<T>(a, c->p.post_smooth, false, c->stream, &nb));
    return FLD_OK;
  }
  HIP_TRY(c, launch_prolong<T>(view(c, H, l + 1), view(c, H, l), c->ctrl,
                               c->stream));
  return smooth_simple<T>(c, H, l, c->p.post_smooth);
}

template <typename T>
TailArgs<T> tail_args(fld_ctx* c, const Levels<T>& H, int l0, bool whole) {
  TailArgs<T> t;
  t.l0 = l0;
  t.L = c->L;
  t.pre = c->p.pre_smooth;
  t.post = c->p.post_smooth;
  t.whole = whole;
  t.zero = !whole;
  for (int l = 0; l < c->L; ++l) t.lv[l] = view(c, H, l);
  t.tmp = H.tmp;
  t.ctrl = c->ctrl;
  return t;
}

// One V-cycle.  `zero_first`: the finest iterate starts at zero (the FP32
// correction of a refinement iteration).
template <typename T>
fld_status vcycle(fld_ctx* c, const Levels<T>& H, bool zero_first) {
  if (c->L == 1 && !c->fast) {
    if (zero_first) FLD_TRY(fill_zero<T>(c, H.x[0], c->geom[0].N));
    HIP_TRY(c, launch_coarsest<T>(view(c, H, 0), H.tmp, c->ctrl, c->stream));
    if (sizeof(T) == 8) {
      int nb = 0;
      HIP_TRY(c, launch_resid_norm<T>(view(c, H, 0), c->partials, &nb, c->ctrl,
                                      c->stream));
      HIP_TRY(c, launch_finalize(kFinCycle, c->partials, nb, c->ctrl, c->stream));
    }
    return FLD_OK;
  }
  const int l0 = c->fast ? c->tail_l0 : c->L - 1;
  for (int l = 0; l < l0; ++l)
    FLD_TRY(down<T>(c, H, l, l > 0 || zero_first));
  if (!c->fast) {
    // reference path: coarsest Jacobi, one launch per level otherwise
    HIP_TRY(c, launch_coarsest<T>(view(c, H, l0), H.tmp, c->ctrl, c->stream));
  } else {
    TailArgs<T> ta = tail_args<T>(c, H, l0, false);
    ta.zero = l0 > 0 || zero_first;
    HIP_TRY(c, launch_tail<T>(ta, c->stream));
  }
  for (int l = l0 - 1; l >= 0; --l) FLD_TRY(up<T>(c, H, l));
  return FLD_OK;
}

fld_status collect_timing(fld_ctx* c) {
  if (!c->timing) return FLD_OK;
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
    c->t_ms += ms;
    c->t_launches += 1;
    c->t_bytes += c->ev_bytes[i / 2];
  }
  c->ev_used = 0;
  c->ev_bytes.clear();
  return FLD_OK;
}

// The kernels that decide the stop flag also write the control block into
// host-visible pinned memory, so reading it needs only the stream sync.
fld_status read_control(fld_ctx* c) {
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return FLD_OK;
}

// FP64 V-cycles until the device stop flag is set.
fld_status solve_fp64(fld_ctx* c) {
  int nb = 0;
  HIP_TRY(c, launch_resid_norm<double>(view(c, c->h64, 0), c->partials, &nb,
                                       c->ctrl, c->stream));
  HIP_TRY(c, launch_finalize(kFinInitial, c->partials, nb, c->ctrl, c->stream));
  if (c->fast && c->tail_l0 == 0) {
    // the whole problem fits one workgroup: one launch runs every cycle
    HIP_TRY(c, launch_tail<double>(tail_args<double>(c, c->h64, 0, true),
                                   c->stream));
    return read_control(c);
  }
  int enqueued = 0;
  int batch = c->last_batch < 1 ? 1 : c->last_batch;
  for (;;) {
    if (batch > c->p.max_cycles - enqueued) batch = c->p.max_cycles - enqueued;
    for (int k = 0; k < batch; ++k)
      FLD_TRY(vcycle<double>(c, c->h64, false));
    enqueued += batch;
    FLD_TRY(read_control(c));
    if (c->host_ctrl->done != kRunning || enqueued >= c->p.max_cycles) break;
    batch = 2;
  }
  if (c->host_ctrl->done == kConverged) c->last_batch = c->host_ctrl->cycles;
  return FLD_OK;
}

// FP32 V-cycles inside an FP64 iterative refinement.
fld_status solve_mixed(fld_ctx* c) {
  const Geom& g0 = c->geom[0];
  int enqueued = 0;
  int batch = c->last_batch < 1 ? 1 : c->last_batch;
  const int max_outer = c->p.max_cycles / c->inner + 2;
  for (;;) {
    for (int k = 0; k < batch; ++k) {
      int nb = 0;
      HIP_TRY(c, launch_resid_to32(view(c, c->h64, 0), c->h32.b[0],
                                   c->partials, &nb, c->ctrl, c->stream));
      HIP_TRY(c, launch_finalize(kFinOuter, c->partials, nb, c->ctrl, c->stream));
      for (int i = 0; i < c->inner; ++i)
        FLD_TRY(vcycle<float>(c, c->h32, i == 0));
      HIP_TRY(c, launch_correct(g0.N, c->h64.x[0], c->h32.x[0], c->ctrl,
                                c->stream));
    }
    enqueued += batch;
    FLD_TRY(read_control(c));
    if (c->host_ctrl->done != kRunning || enqueued >= max_outer) break;
    batch = 1;
  }
  if (c->host_ctrl->done == kRunning) c->host_ctrl->done = kCapped;
  if (c->host_ctrl->done == kConverged)
    c->last_batch = c->host_ctrl->outer + 1;
  return FLD_OK;
}

}  // namespace

extern "C" {

void fld_params_default(fld_params* p) {
  if (!p) return;
  memset(p, 0, sizeof *p);
  p->ndim = 1;
  for (int d = 0; d < 3; ++d) {
    p->n[d] = 1;
    p->dx[d] = 1.0;
    p->bc_lo[d] = p->bc_hi[d] = FLD_BC_PERIODIC;
  }
  p->c = 1.0;
  p->a_rad = 1.0;
  p->gamma = 5.0 / 3.0;
  p->gas_const = 1.0;
  p->limiter = FLD_LIMITER_LP;
  p->face_mean = FLD_FACE_ARITH;
  p->precision = FLD_PREC_FP64;
  p->guess = FLD_GUESS_PREV;
  p->rtol = 1e-8;
  p->max_cycles = 50;
  p->pre_smooth = 2;
  p->post_smooth = 2;
}

size_t fld_workspace_bytes(const fld_params* p) {
  if (!validate(p).empty()) return 0;
  Plan P;
  make_plan(p, &P);
  return P.total;
}

fld_status fld_setup(const fld_params* p, void* workspace, size_t ws_bytes,
                     void* hip_stream, fld_ctx** out) {
  if (!out) return fail(nullptr, FLD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  std::string why = validate(p);
  if (!why.empty()) return fail(nullptr, FLD_ERR_INVALID_ARG, "%s", why.c_str());
  Plan P;
  make_plan(p, &P);
  if (P.g[P.L - 1].N > kMaxCoarsestCells)
    return fail(nullptr, FLD_ERR_INVALID_ARG,
                "coarsest grid has %lld cells (> %lld): sides must be "
                "divisible by 2 more often",
                (long long)P.g[P.L - 1].N, (long long)kMaxCoarsestCells);
  if (!workspace) return fail(nullptr, FLD_ERR_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)workspace % kAlign)
    return fail(nullptr, FLD_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < P.total)
    return fail(nullptr, FLD_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu",
                ws_bytes, P.total);
  fld_ctx* c = new fld_ctx();
  c->p = *p;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace;
  c->ws_bytes = ws_bytes;
  c->L = P.L;
  c->mixed = p->precision == FLD_PREC_FP32_IR;
  char* w = c->ws;
  for (int l = 0; l < P.L; ++l) {
    c->geom[l] = P.g[l];
    const bool has64 = l == 0 || !c->mixed;
    for (int d = 0; d < p->ndim; ++d) {
      c->h64.a[l][d] = has64 ? (double*)(w + P.a64[l][d]) : nullptr;
      c->h32.a[l][d] = c->mixed ? (float*)(w + P.a32[l][d]) : nullptr;
    }
    c->h64.x[l] = (has64 && l > 0) ? (double*)(w + P.x64[l]) : nullptr;
    c->h64.b[l] = (has64 && l > 0) ? (double*)(w + P.b64[l]) : nullptr;
    c->h32.x[l] = c->mixed ? (float*)(w + P.x32[l]) : nullptr;
    c->h32.b[l] = c->mixed ? (float*)(w + P.b32[l]) : nullptr;
  }
  const char* path = getenv("FLD_KERNEL_PATH");
  c->fast = !(path && strcmp(path, "simple") == 0);
  c->tail_l0 = c->L - 1;
  for (int l = 0; l < c->L; ++l)
    if (c->geom[l].N <= kTailLdsCells) {
      c->tail_l0 = l;
      break;
    }
  c->bcopy = (double*)(w + P.bcopy);
  c->partials = (double*)(w + P.partials);
  c->h64.tmp = (double*)(w + P.tmp);
  c->h32.tmp = (float*)(w + P.tmp);
  c->ctrl = (Control*)(w + P.ctrl);
  hipError_t he = hipHostMalloc((void**)&c->host_ctrl, sizeof(Control),
                                hipHostMallocMapped | hipHostMallocCoherent);
  if (he == hipSuccess)
    he = hipHostGetDevicePointer((void**)&c->host_ctrl_dev, c->host_ctrl, 0);
  if (he != hipSuccess) {
    delete c;
    return fail(nullptr, FLD_ERR_DEVICE,
                "hipHostMalloc of the control mirror failed: %s",
                hipGetErrorString(he));
  }
  memset(c->host_ctrl, 0, sizeof(Control));
  *out = c;
  return FLD_OK;
}

fld_status fld_step(fld_ctx* c, double dt, const double* rho,
                    const double* kappa, const double* E_in, double* E_out,
                    fld_stats* stats) {
  if (!c) return fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (!rho || !kappa || !E_in || !E_out)
    return fail(c, FLD_ERR_INVALID_ARG, "NULL field pointer");
  if (!(dt > 0.0) || !std::isfinite(dt))
    return fail(c, FLD_ERR_INVALID_ARG, "dt must be positive and finite");
  const bool aliased = (E_in == E_out);
  const Geom& g0 = c->geom[0];
  // level 0: x = E_out, b = E_in (or its copy when E_out overwrites it)
  c->h64.x[0] = E_out;
  c->h64.b[0] = aliased ? c->bcopy : const_cast<double*>(E_in);
  double* copy_dst = aliased ? c->bcopy
                             : (c->p.guess == FLD_GUESS_ZERO ? nullptr : E_out);
  HIP_TRY(c, launch_ctrl_init(c->ctrl, c->p.rtol, c->p.max_cycles, c->inner,
                             c->host_ctrl_dev, c->stream));
  CoefArgs A;
  A.g = g0;
  for (int d = 0; d < 3; ++d) A.dx[d] = c->p.dx[d];
  A.dt = dt;
  A.c = c->p.c;
  A.limiter = c->p.limiter;
  A.face_mean = c->p.face_mean;
  HIP_TRY(c, launch_coef(A, E_in, rho, kappa, c->h64.a[0], c->h32.a[0],
                         copy_dst, c->partials, c->ctrl, c->stream));
  HIP_TRY(c, launch_finalize(kFinBnorm, c->partials, blocks_for(g0.N), c->ctrl,
                             c->stream));
  for (int l = 0; l + 1 < c->L; ++l) {
    if (c->mixed) {
      const float* fa[3] = {c->h32.a[l][0], c->h32.a[l][1], c->h32.a[l][2]};
      float* ca[3] = {c->h32.a[l + 1][0], c->h32.a[l + 1][1],
                      c->h32.a[l + 1][2]};
      HIP_TRY(c, launch_coarsen<float>(c->geom[l], c->geom[l + 1], fa, ca,
                                       c->stream));
    } else {
      const double* fa[3] = {c->h64.a[l][0], c->h64.a[l][1], c->h64.a[l][2]};
      double* ca[3] = {c->h64.a[l + 1][0], c->h64.a[l + 1][1],
                       c->h64.a[l + 1][2]};
      HIP_TRY(c, launch_coarsen<double>(c->geom[l], c->geom[l + 1], fa, ca,
                                        c->stream));
    }
  }
  if (c->p.guess == FLD_GUESS_ZERO)
    HIP_TRY(c, launch_fill(E_out, g0.N, 0.0, c->stream));
  FLD_TRY(c->mixed ? solve_mixed(c) : solve_fp64(c));
  FLD_TRY(collect_timing(c));
  const Control& h = *c->host_ctrl;
  if (stats) {
    memset(stats, 0, sizeof *stats);
    stats->cycles = h.cycles;
    stats->outer_iters = c->mixed ? h.outer : 0;
    stats->flagged_cells = h.flagged;
    stats->rel_res_initial = h.res_initial;
    stats->rel_res_final = h.res;
  }
  if (h.done == kNonPhysical)
    return fail(c, FLD_ERR_NONPHYSICAL,
                "%d cells with E <= 0, rho*kappa <= 0 or non-finite input",
                h.flagged);
  if (h.done != kConverged)
    return fail(c, FLD_ERR_NOT_CONVERGED,
                "relative residual %.3e > rtol %.3e after %d V-cycles", h.res,
                c->p.rtol, h.cycles);
  return FLD_OK;
}

fld_status fld_exchange(fld_ctx* c, double dt, const double* rho,
                        const double* kappa, double* E, double* e_int) {
  if (!c) return fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (!rho || !kappa || !E || !e_int)
    return fail(c, FLD_ERR_INVALID_ARG, "NULL field pointer");
  if (!(dt > 0.0) || !std::isfinite(dt))
    return fail(c, FLD_ERR_INVALID_ARG, "dt must be positive and finite");
  HIP_TRY(c, launch_exchange(c->geom[0].N, dt, c->p.c, c->p.a_rad, c->p.gamma,
                             c->p.gas_const, rho, kappa, E, e_int, c->stream));
  return FLD_OK;
}

fld_status fld_opacity_powerlaw(fld_ctx* c, const double* rho,
                                const double* e_int, double k0, double a,
                                double b, double kmin, double kmax,
                                double* kappa) {
  if (!c) return fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (!rho || !e_int || !kappa)
    return fail(c, FLD_ERR_INVALID_ARG, "NULL field pointer");
  if (!(k0 > 0.0) || !(kmin > 0.0) || !(kmax >= kmin) || !std::isfinite(a) ||
      !std::isfinite(b) || !std::isfinite(kmax))
    return fail(c, FLD_ERR_INVALID_ARG,
                "need k0 > 0, 0 < kmin <= kmax, finite exponents");
  HIP_TRY(c, launch_opacity(c->geom[0].N, c->p.gamma, c->p.gas_const, rho,
                            e_int, k0, a, b, kmin, kmax, kappa, c->stream));
  return FLD_OK;
}

fld_status fld_kernel_timing_enable(fld_ctx* c, int32_t on) {
  if (!c) return fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  c->timing = on != 0;
  c->ev_used = 0;
  c->ev_bytes.clear();
  return FLD_OK;
}

fld_status fld_kernel_timing_read(fld_ctx* c, double* ms_total,
                                  int64_t* launches, double* bytes_total,
                                  const char** kernel_name) {
  if (!c) return fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (ms_total) *ms_total = c->t_ms;
  if (launches) *launches = c->t_launches;
  if (bytes_total) *bytes_total = c->t_bytes;
  if (kernel_name) *kernel_name = c->t_name;
  c->t_ms = 0.0;
  c->t_launches = 0;
  c->t_bytes = 0.0;
  return FLD_OK;
}

void fld_destroy(fld_ctx* c) {
  if (!c) return;
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->host_ctrl) (void)hipHostFree(c->host_ctrl);
  delete c;
}

const char* fld_status_str(int32_t s) {
  switch (s) {
    case FLD_OK: return "FLD_OK";
    case FLD_ERR_INVALID_ARG: return "FLD_ERR_INVALID_ARG";
    case FLD_ERR_WORKSPACE: return "FLD_ERR_WORKSPACE";
    case FLD_ERR_DEVICE: return "FLD_ERR_DEVICE";
    case FLD_ERR_NONPHYSICAL: return "FLD_ERR_NONPHYSICAL";
    case FLD_ERR_NOT_CONVERGED: return "FLD_ERR_NOT_CONVERGED";
    case FLD_ERR_MODEL: return "FLD_ERR_MODEL";
    default: return "FLD_STATUS_UNKNOWN";
  }
}

const char* fld_last_error(const fld_ctx* c) {
  return c ? c->err.c_str() : g_err.c_str();
}

}  // extern "C"
