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
//
// Initial guess: E^n, zero, or the learned guess E^n (1 + delta) of the
// U-Net (fld_unet_net.cpp), kept only when its FP64 residual is smaller
// than that of E^n.
#include "fld.h"
#include "fldnn.h"
#include "fld_internal.h"
#include "fld_hooks.h"
#include "fld_tile2d.h"
#include "fld_batch.h"
#include "fld_unet.h"
#include "fld_unet_net.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace fld;

namespace {

template <typename T>
struct Levels {
  T* x[kMaxLevels] = {};
  T* b[kMaxLevels] = {};
  T* a[kMaxLevels][3] = {};
  // extra diagonal term (or null): Dirichlet walls, and on the finest
  // level the faces of free cells to held cells
  T* sd[kMaxLevels] = {};
  // coarse levels' held points (or null): some child held
  uint8_t* held[kMaxLevels] = {};
  T* alt[kMaxLevels] = {};  // second iterate buffer of the tiled 2D levels
  T* tmp = nullptr;  // coarsest-level scratch (global-memory tail only)
};

}  // namespace

struct BatchState;

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
  double* dscr = nullptr;      // 3D: cell-centred D of the coefficient stage
  double* partials = nullptr;  // block partial sums
  Control* ctrl = nullptr;     // device control block
  Control* host_ctrl = nullptr;  // pinned host mirror, written by the GPU
  Control* host_ctrl_dev = nullptr;  // its device-side address
  // contexts without a mapped mirror (the allocation-free step) copy the
  // control block here after each synchronisation
  Control host_copy{};
  bool ctrl_by_copy = false;  // read_control copies ctrl into host_copy
  bool mixed = false;
  int inner = 2;               // FP32 V-cycles per refinement iteration
  int last_batch = 4;          // cycles (or outer iterations) last step
  std::string err;
  // timing of the dominant kernel (finest-level down pass)
  bool timing = false;
  bool init_fused = false;  // this step's coefficient stage formed the initial residual
  int fin_cycle = -1;       // index of the FP64 V-cycle being enqueued
  int pending_fin = 0;      // finest down partials awaiting their stop test
  double t_ms = 0.0;
  int64_t t_launches = 0;
  double t_bytes = 0.0;
  const char* t_name = "none";
  std::vector<hipEvent_t> ev;    // pool, used in (start, stop) pairs
  std::vector<double> ev_bytes;  // algorithmic bytes of each timed launch
  size_t ev_used = 0;
  bool fast = true;  // tiled kernels + single-workgroup tail
  int tail_l0 = 0;   // first level handled by the single-workgroup tail
  bool coarsen_multi = true;  // 2D: several coarse levels per launch
  bool sweep3d = true;        // 3D: fused red-black sweeps where planned
  bool level_lds = true;      // small 3D coarse levels in one workgroup
  bool tile3d = true;         // 3D: tiled sweeps below the marching ones
  bool tile3d_all = false;    // 3D: tiled sweeps on the large levels too
  bool tail_big = true;       // 2D: tail from a level of up to 4096 cells
  // held cells (fld_params.held_cells): the caller's mask and prescribed
  // values, given by fld_set_held
  const uint8_t* held_mask = nullptr;
  const double* held_vals = nullptr;
  int sweep_zc = 0;           // z planes per block of a fused sweep (0: auto)
  int tile_var[kMaxLevels][2] = {};  // tile shape per level: down, up
  BatchState* batch = nullptr;  // set for a batched context (sub-grids)
  // learned guess: network carved out of net_ws by fld_set_model
  nn::Net* net = nullptr;
  char* net_ws = nullptr;
  size_t net_bytes = 0;
  double* mean = nullptr;  // per-slice mean of log E (network features)
  double* guess = nullptr;  // the network's candidate iterate (FP64)
  // adaptive network policy: steps left without the network, the length
  // of the next pause, and the work (V-cycles, or refinement iterations)
  // of the last step without it
  int net_skip = 1;
  int net_span = 0;
  int plain_units = -1;
  // the judge's bar on the guess's squared residual relative to that of
  // E^n: 1, or (adaptive policy, once a step without the network has run)
  // the square of that step's contraction per V-cycle or refinement
  // iteration, so that an accepted guess is predicted to save one
  double judge_q2 = 1.0;
  // the policy's clock (events on the stream): [0] before the network,
  // [1] before the solve, [2] at the solve's last control read; the
  // solve's time per unit on the last step without the network
  hipEvent_t net_ev[3] = {nullptr, nullptr, nullptr};
  bool net_clock = false;
  bool net_ev_end = false;  // net_ev[2] recorded during this solve
  double unit_ms = -1.0;
  // flexible CG around the V-cycle (fld_params.krylov)
  bool krylov = false;
  bool precond = false;  // V-cycles run as a preconditioner: no stop test
  double* kr_r = nullptr;
  double* kr_p[2] = {};
  double* kr_q = nullptr;
  double* kr_z = nullptr;
  // FP32_IR + flexible CG: steps left that start with FP64 V-cycles after
  // the FP32 ones stalled, the current pause, and this step's fallback
  int pre64_skip = 0, pre64_span = 0;
  bool pre64_used = false;
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

// Static scratch of fld_step_noalloc: the workspace of a step carved out of
// a file-scope device array instead of caller or library allocations.  Each
// device that loads this library holds its own copy until the process ends.
// Host code must use the address hipGetSymbolAddress returns on the device
// (the array's name in host code is only a stand-in), kept per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

fld_status static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return fail(nullptr, FLD_ERR_DEVICE, "hipGetDevice: %s",
                hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(nullptr, FLD_ERR_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(nullptr, FLD_ERR_DEVICE,
                  "hipGetSymbolAddress of the static scratch: %s",
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FLD_OK;
}

constexpr int64_t kMaxCoarsestCells = 1 << 16;
// tile shape the autotuner tries first (32x32/256)
constexpr int kTilePreferred = 3;
// pauses of the adaptive policy: 2, 4, ... up to this many steps without
// the network after each try that saved nothing
constexpr int kMaxNetPause = 32;
// 3D levels of at least this many cells smooth by fused sweeps (smaller
// ones are launch-latency bound, where a block's march through its planes
// costs more than the second colour launch)
constexpr int64_t kSweepMinCells = 1 << 22;

// FLD_SWEEP3D set to a number > 1 (planes per block) also takes fused sweeps
// on the smaller levels (tests on small grids)
int64_t sweep_min_cells() {
  const char* sw = getenv("FLD_SWEEP3D");
  return (sw && atoi(sw) > 1) ? 0 : kSweepMinCells;
}

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Plan {
  int L = 0;
  Geom g[kMaxLevels];
  size_t a64[kMaxLevels][3] = {}, x64[kMaxLevels] = {}, b64[kMaxLevels] = {};
  size_t a32[kMaxLevels][3] = {}, x32[kMaxLevels] = {}, b32[kMaxLevels] = {};
  size_t alt[kMaxLevels] = {};  // tiled 2D levels: iterate double buffer
  size_t alt64[kMaxLevels] = {};  // FP64 ones beside FP32 (see pre64)
  size_t bcopy = 0, partials = 0, tmp = 0, ctrl = 0, mean = 0, net = 0;
  size_t dscr = 0;  // 3D coefficient stage: D per cell
  size_t sd64[kMaxLevels] = {};  // extra diagonal term per level
  size_t held[kMaxLevels] = {};  // coarse levels' held points
  size_t guess = 0;
  size_t kr_r = 0, kr_p[2] = {}, kr_q = 0, kr_z = 0;  // flexible CG vectors
  size_t net_bytes = 0;
  int64_t n_partials = 0;
  size_t total = 0;
};

// Whether some wall holds E (FLD_BC_DIRICHLET).
inline bool has_dirichlet(const fld_params& p);
// Whether the system has rows of its own beside E^n's: Dirichlet walls or
// held cells (FP64 V-cycles on the one-launch-per-pass kernels).
inline bool own_rows(const fld_params& p) {
  return has_dirichlet(p) || p.held_cells != 0;
}
inline bool has_dirichlet(const fld_params& p) {
  for (int d = 0; d < p.ndim; ++d)
    if (p.bc_lo[d] == FLD_BC_DIRICHLET || p.bc_hi[d] == FLD_BC_DIRICHLET)
      return true;
  return false;
}

// Smoothing sweeps on level l: the finest level's pre/post_smooth, the
// coarse levels' coarse_pre/coarse_post_smooth (0: the same as the finest).
inline int nu_pre(const fld_params& p, int l) {
  return (l > 0 && p.coarse_pre_smooth > 0) ? p.coarse_pre_smooth : p.pre_smooth;
}
inline int nu_post(const fld_params& p, int l) {
  return (l > 0 && p.coarse_post_smooth > 0) ? p.coarse_post_smooth
                                              : p.post_smooth;
}

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
      if (p->bc_lo[d] < 0 || p->bc_lo[d] > 2 || p->bc_hi[d] < 0 ||
          p->bc_hi[d] > 2) {
        snprintf(buf, sizeof buf, "bc[%d]: periodic, neumann or dirichlet", d);
        return buf;
      }
      for (int side = 0; side < 2; ++side) {
        const int bc = side ? p->bc_hi[d] : p->bc_lo[d];
        const double v = side ? p->bc_value_hi[d] : p->bc_value_lo[d];
        if (bc == FLD_BC_DIRICHLET && !(v > 0.0 && std::isfinite(v))) {
          snprintf(buf, sizeof buf,
                   "bc_value[%d]: a Dirichlet wall's E must be > 0", d);
          return buf;
        }
      }
      if ((p->bc_lo[d] == FLD_BC_PERIODIC) != (p->bc_hi[d] == FLD_BC_PERIODIC)) {
        snprintf(buf, sizeof buf, "bc[%d]: periodic must be set on both sides", d);
        return buf;
      }
      if (p->bc_lo[d] != FLD_BC_PERIODIC && p->n[d] < 2) {
        snprintf(buf, sizeof buf, "n[%d] must be >= 2 with walls", d);
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
  if (p->limiter < 0 || p->limiter > 2) return "unknown limiter";
  if (p->face_mean < 0 || p->face_mean > 1) return "unknown face mean";
  if (p->precision != FLD_PREC_FP64 && p->precision != FLD_PREC_FP32_IR)
    return "unknown precision";
  if (p->guess != FLD_GUESS_PREV && p->guess != FLD_GUESS_ZERO &&
      p->guess != FLD_GUESS_LEARNED)
    return "unknown guess";
  if (p->guess == FLD_GUESS_LEARNED &&
      (p->ndim < 2 || p->n[0] % 8 || p->n[1] % 8))
    return "the learned guess needs ndim >= 2 and n[0], n[1] multiples of 8";
  if (p->guess == FLD_GUESS_LEARNED && p->n[2] > 16384)
    return "the learned guess takes at most 16384 z-slices";
  if (p->guess_policy != FLD_GUESS_ADAPTIVE &&
      p->guess_policy != FLD_GUESS_EVERY_STEP)
    return "unknown guess_policy";
  if (p->krylov != 0 && p->krylov != 1) return "krylov must be 0 or 1";
  if (p->held_cells != 0 && p->held_cells != 1) return "held_cells must be 0 or 1";
  if (own_rows(*p) &&
      (p->precision != FLD_PREC_FP64 || p->krylov ||
       p->guess == FLD_GUESS_LEARNED))
    return "Dirichlet walls and held cells: precision FP64, krylov 0, guess "
           "E^n or zero";
  if (!(p->rtol > 0.0) || !(p->rtol < 1.0)) return "rtol must be in (0, 1)";
  if (p->ir_inner < 0 || p->ir_inner > 8) return "ir_inner must be in [0, 8]";
  if (p->max_cycles < 1) return "max_cycles must be >= 1";
  if (p->pre_smooth < 0 || p->post_smooth < 0 ||
      p->pre_smooth + p->post_smooth < 1 || p->pre_smooth > 16 ||
      p->post_smooth > 16)
    return "pre_smooth/post_smooth must be in [0, 16], not both 0";
  if (p->coarse_pre_smooth < 0 || p->coarse_post_smooth < 0 ||
      p->coarse_pre_smooth > 16 || p->coarse_post_smooth > 16 ||
      nu_pre(*p, 1) + nu_post(*p, 1) < 1)
    return "coarse_pre_smooth/coarse_post_smooth must be in [0, 16] (0: the "
           "finest level's), the resulting coarse sweeps not both 0";
  return "";
}

void make_plan(const fld_params* p, Plan* P) {
  Geom g;
  g.ndim = p->ndim;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = (int)p->n[d];
    g.per[d] = (d < p->ndim && p->bc_lo[d] == FLD_BC_PERIODIC) ? 1 : 0;
    g.dirw[d] = d < p->ndim ? (p->bc_lo[d] == FLD_BC_DIRICHLET ? 1 : 0) |
                                  (p->bc_hi[d] == FLD_BC_DIRICHLET ? 2 : 0)
                            : 0;
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
  // FP32_IR with flexible CG keeps an FP64 hierarchy as well: its
  // preconditioner falls back to FP64 V-cycles where FP32 ones stall
  const bool pre64 = mixed && p->krylov;
  for (int l = 0; l < P->L; ++l) {
    const size_t cells = (size_t)P->g[l].N;
    if (l == 0 || !mixed || pre64) {
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
    // 2D: the tiled levels' iterate double buffer; 3D: out-of-place buffer
    // of the fused red-black sweep
    const bool alt = (nd == 2 && l + 1 < P->L) ||
                     (nd == 3 && l + 1 < P->L &&
                      (((int64_t)cells >= sweep_min_cells() &&
                        gs_sweep3d_ok(P->g[l])) ||
                       ((int64_t)cells > kLevelLdsCells &&
                        gs_tile3d_ok(P->g[l]))));
    if (alt) {
      P->alt[l] = take(cells * (mixed ? 4 : 8));
      if (pre64) P->alt64[l] = take(cells * 8);
    }
    if (own_rows(*p)) P->sd64[l] = take(cells * 8);
    if (p->held_cells && l > 0) P->held[l] = take(cells);
  }
  P->bcopy = take((size_t)P->g[0].N * 8);
  if (nd == 3) P->dscr = take((size_t)P->g[0].N * 8);
  int64_t nparts = blocks_for(P->g[0].N);
  if (p->ndim == 3)  // one partial per block of the 3D launch grid
    nparts = std::max<int64_t>(nparts, blocks3(P->g[0]));
  if (coef2d_ok(P->g[0]))  // |b|^2 and |r0|^2 partials of the 2D stage
    nparts = std::max<int64_t>(nparts, 2 * (int64_t)coef2d_blocks(P->g[0]));
  if (p->ndim == 2)
    for (int nu = 1; nu <= 3; ++nu)
      for (int v = 0; v < kTileVariants; ++v) {
        const int64_t t = tile2d_blocks(P->g[0], nu, true, v);
        if (t > nparts) nparts = t;
      }
  if (p->krylov)  // (p, q) and (p, r) partials of the flexible-CG passes
    nparts = std::max<int64_t>(nparts, 2 * (int64_t)krylov_blocks(P->g[0]));
  P->n_partials = nparts + 64;
  P->partials = take((size_t)P->n_partials * 8);
  P->tmp = take((size_t)P->g[P->L - 1].N * 8);
  P->ctrl = take(sizeof(Control));
  if (p->ndim >= 2)
    P->mean = take((size_t)(p->n[2] + nn::mean_log_scratch(p->n[0] * p->n[1],
                                                           (int)p->n[2])) * 8);
  if (p->guess == FLD_GUESS_LEARNED) {
    P->net_bytes = nn::workspace_bytes((int)p->n[2], (int)p->n[1],
                                       (int)p->n[0], 0);
    P->net = take(P->net_bytes);
    P->guess = take((size_t)P->g[0].N * 8);
  }
  if (p->krylov) {
    const size_t n0 = (size_t)P->g[0].N * 8;
    P->kr_r = take(n0);
    P->kr_p[0] = take(n0);
    P->kr_p[1] = take(n0);
    P->kr_q = take(n0);
    // FP64 preconditioner output (FP32_IR: the FP32 level-0 iterate, and
    // this one after a fallback to FP64 V-cycles)
    P->kr_z = take(n0);
  }
  P->total = o;
}

template <typename T>
LevelView<T> view(const fld_ctx* c, const Levels<T>& H, int l) {
  LevelView<T> v;
  v.g = c->geom[l];
  v.x = H.x[l];
  v.b = H.b[l];
  for (int d = 0; d < 3; ++d) v.a[d] = H.a[l][d];
  v.sd = H.sd[l];
  v.held = H.held[l];
  return v;
}

// The timing events only timestamp launches; their intervals are read after
// the step's stream synchronisation, so they skip the system-scope cache
// writeback a default event performs when it completes (that writeback cost
// about 6.5 us per timed launch and slowed the work after it).
hipEvent_t next_event(fld_ctx* c) {
  if (c->ev_used == c->ev.size()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
      return nullptr;
    c->ev.push_back(e);
  }
  return c->ev[c->ev_used++];
}

// Event pair recorded by one launch of the timed kernel itself
// (hipExtLaunchKernelGGL): the interval is the kernel's own execution.
struct TimedLaunch {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  fld_status st = FLD_OK;
  TimedLaunch(fld_ctx* c, bool on, double bytes, const char* name) {
    if (!on || !c->timing) return;
    e0 = next_event(c);
    e1 = next_event(c);
    if (!e0 || !e1) {
      st = fail(c, FLD_ERR_DEVICE, "hipEventCreate failed");
      e0 = e1 = nullptr;
      return;
    }
    c->ev_bytes.push_back(bytes);
    c->t_name = name;
  }
};

bool tile_path(const fld_ctx* c) {
  auto ok = [](int nu) { return nu >= 1 && nu <= 3; };
  return c->fast && c->p.ndim == 2 && ok(c->p.pre_smooth) &&
         ok(c->p.post_smooth) && ok(nu_pre(c->p, 1)) && ok(nu_post(c->p, 1));
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

// How level l smooths in 3D: 0 colour passes only; pairs of one-launch
// sweeps where it has the alternate buffer and some pre or post count of at
// least two: 1 z-marching sweeps (large levels), 2 tiled sweeps.
constexpr int kFusedNone = 0, kFusedMarch = 1, kFusedTile = 2;
template <typename T>
int fused_level(const fld_ctx* c, const Levels<T>& H, int l) {
  const Geom& g = c->geom[l];
  if (!c->sweep3d || g.ndim != 3 || !H.alt[l] ||
      (nu_pre(c->p, l) < 2 && nu_post(c->p, l) < 2))
    return kFusedNone;
  if (c->tile3d_all && gs_tile3d_ok(g)) return kFusedTile;
  if (g.N >= sweep_min_cells() && gs_sweep3d_ok(g)) return kFusedMarch;
  if (c->tile3d && gs_tile3d_ok(g)) return kFusedTile;
  return kFusedNone;
}

// Simple path: one launch per colour pass, or, on a 3D level with an
// alternate buffer, pairs of fused red-black sweeps (x -> alt -> x) after
// one sweep of colour passes when the count is odd.  With `timed` (the
// finest level's smoothing in 3D), the first fused launch of the call
// records its own duration for the kernel timing, or, on a level without
// fused sweeps, the first colour pass of the pre-smoothing.  A colour pass
// updates half the cells, reading b of those, all three face arrays and the
// iterate, and writing its half: 4.5 N elements touched once; a fused sweep
// reads b, the three face arrays and the iterate and writes the whole
// iterate: 6 N.
// a coarse 3D level small enough for one workgroup (fld_level.hip), above
// the tail
bool level_lds(const fld_ctx* c, int l) {
  return c->level_lds && l >= 1 && l < c->tail_l0 &&
         level_lds_ok(c->geom[l], c->geom[l + 1]);
}

template <typename T>
fld_status smooth_simple(fld_ctx* c, const Levels<T>& H, int l, int sweeps,
                         bool timed_fused, bool timed_colour) {
  LevelView<T> v = view(c, H, l);
  T* alt = H.alt[l];
  const int mode = fused_level(c, H, l);
  const bool fused = mode != kFusedNone;
  const int pairs = fused ? sweeps / 2 : 0;
  // only the context's own precision is timed (an FP32_IR solve whose
  // flexible CG fell back to FP64 V-cycles runs both)
  if ((sizeof(T) == 4) != c->mixed) timed_fused = timed_colour = false;
  const int plain = sweeps - 2 * pairs;
  for (int s = 0; s < plain; ++s)
    for (int color = 0; color < gs_colors(v.g); ++color) {
      TimedLaunch tl(c, timed_colour && !fused && s == 0 && color == 0,
                     4.5 * (double)v.g.N * sizeof(T),
                     sizeof(T) == 8 ? "k_gs_color_3d<double>"
                                    : "k_gs_color_3d<float>");
      FLD_TRY(tl.st);
      HIP_TRY(c, launch_gs_color<T>(v, color, c->ctrl, c->stream, tl.e0,
                                    tl.e1));
    }
  LevelView<T> va = v;
  va.x = alt;
  for (int s = 0; s < pairs; ++s) {
    const bool march = mode == kFusedMarch;
    const char* name =
        march ? (sizeof(T) == 8 ? "k_gs_sweep_3d<double>" : "k_gs_sweep_3d<float>")
              : (sizeof(T) == 8 ? "k_gs_tile_3d<double>" : "k_gs_tile_3d<float>");
    TimedLaunch tl(c, timed_fused && s == 0, 6.0 * (double)v.g.N * sizeof(T),
                   name);
    FLD_TRY(tl.st);
    if (march) {
      HIP_TRY(c, launch_gs_sweep3d<T>(v, alt, c->sweep_zc, c->ctrl, c->stream,
                                      tl.e0, tl.e1));
      HIP_TRY(c, launch_gs_sweep3d<T>(va, v.x, c->sweep_zc, c->ctrl, c->stream));
    } else {
      HIP_TRY(c, launch_gs_tile3d<T>(v, alt, c->ctrl, c->stream, tl.e0, tl.e1));
      HIP_TRY(c, launch_gs_tile3d<T>(va, v.x, c->ctrl, c->stream));
    }
  }
  return FLD_OK;
}

// Down pass on level l (above the tail): pre-smoothing, residual,
// restriction.  `zero_init`: x starts at zero.  On the finest FP64 level
// the residual norm feeds the stop test.
template <typename T>
fld_status down(fld_ctx* c, const Levels<T>& H, int l, bool zero_init) {
  const bool norm = (sizeof(T) == 8) && l == 0 && !c->precond;
  int nb = 0;
  if (level_lds(c, l)) {  // (l >= 1: its x was zeroed by the restriction)
    HIP_TRY(c, launch_level_down<T>(view(c, H, l), view(c, H, l + 1),
                                    nu_pre(c->p, l), c->ctrl, c->stream));
    return FLD_OK;
  }
  if (tile_path(c)) {
    Tile2DArgs<T> a{};
    a.g = c->geom[l];
    a.spec = l == 0;
    a.x = H.x[l];
    a.xo = H.alt[l];
    a.b = H.b[l];
    a.ax = H.a[l][0];
    a.ay = H.a[l][1];
    a.gc = c->geom[l + 1];
    a.cb = H.b[l + 1];
    a.ce = nullptr;
    a.partials = norm ? c->partials : nullptr;
    a.zero_init = zero_init;
    a.ctrl = c->ctrl;
    if (sizeof(T) == 8 && l == 1 && c->pending_fin > 0) {
      a.fin_partials = c->partials;
      a.fin_count = c->pending_fin;
      a.fin_cycle = c->fin_cycle;
      a.fin_ctrl = c->ctrl;
      c->pending_fin = 0;
    }
    // x (unless zero), b, two face arrays read; x and the coarse rhs written
    const double w = sizeof(T);
    const double bytes = (double)c->geom[l].N *
                         (w * (zero_init ? 4.0 : 5.0) + w / 4.0);
    TimedLaunch t(c, l == 0, bytes,
                  sizeof(T) == 8 ? "k_tile2d<double,down>" : "k_tile2d<float,down>");
    FLD_TRY(t.st);
    HIP_TRY(c, launch_tile2d<T>(a, nu_pre(c->p, l), true, c->tile_var[l][0],
                                c->stream, &nb, t.e0, t.e1));
  } else {
    if (zero_init && l == 0) FLD_TRY(fill_zero<T>(c, H.x[0], c->geom[0].N));
    // level 0 of a 3D solve times one launch per V-cycle: the first fused
    // sweep (pre-smoothing if it has one, else post), or the first colour
    // pass of the pre-smoothing on a level without fused sweeps
    const bool t0 = l == 0 && c->geom[0].ndim == 3;
    FLD_TRY(smooth_simple<T>(c, H, l, nu_pre(c->p, l),
                             t0 && nu_pre(c->p, l) >= 2, t0));
    HIP_TRY(c, launch_resid_restrict<T>(view(c, H, l), view(c, H, l + 1),
                                        norm ? c->partials : nullptr, &nb,
                                        c->ctrl, c->stream));
  }
  if (norm) {
    // a tiled level 1 takes the stop test itself (its blocks reduce the
    // partials), saving a launch per V-cycle
    if (tile_path(c) && c->tail_l0 >= 2 && c->fin_cycle >= 0)
      c->pending_fin = nb;
    else
      HIP_TRY(c, launch_finalize(kFinCycle, c->partials, nb, c->ctrl,
                                 c->stream));
  }
  return FLD_OK;
}

// Up pass on level l: prolongation of level l+1 and post-smoothing.
template <typename T>
fld_status up(fld_ctx* c, const Levels<T>& H, int l) {
  if (tile_path(c)) {
    Tile2DArgs<T> a{};
    a.g = c->geom[l];
    a.x = H.alt[l];  // the down pass's output
    a.xo = H.x[l];
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
    HIP_TRY(c, launch_tile2d<T>(a, nu_post(c->p, l), false, c->tile_var[l][1],
                                c->stream, &nb));
    return FLD_OK;
  }
  if (level_lds(c, l)) {
    HIP_TRY(c, launch_level_up<T>(view(c, H, l), view(c, H, l + 1),
                                  nu_post(c->p, l), c->ctrl, c->stream));
    return FLD_OK;
  }
  HIP_TRY(c, launch_prolong<T>(view(c, H, l + 1), view(c, H, l), c->ctrl,
                               c->stream));
  const bool t0 = l == 0 && c->geom[0].ndim == 3 && nu_pre(c->p, l) < 2;
  return smooth_simple<T>(c, H, l, nu_post(c->p, l), t0, false);
}

template <typename T>
TailArgs<T> tail_args(fld_ctx* c, const Levels<T>& H, int l0, bool whole) {
  TailArgs<T> t;
  t.l0 = l0;
  t.L = c->L;
  t.pre = nu_pre(c->p, l0);  // one count for every tail level
  t.post = nu_post(c->p, l0);
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

// An FP64 V-cycle split at its stop test (multi-level fast path): `head`
// is the finest down pass with the test itself (a finalize launch where a
// tiled level 1 would otherwise take it), `tail` the rest of the cycle.
fld_status vcycle_head(fld_ctx* c, const Levels<double>& H) {
  FLD_TRY(down<double>(c, H, 0, false));
  if (c->pending_fin > 0) {
    HIP_TRY(c, launch_finalize(kFinCycle, c->partials, c->pending_fin, c->ctrl,
                               c->stream));
    c->pending_fin = 0;
  }
  return FLD_OK;
}

fld_status vcycle_tail(fld_ctx* c, const Levels<double>& H) {
  const int l0 = c->tail_l0;
  for (int l = 1; l < l0; ++l) FLD_TRY(down<double>(c, H, l, true));
  TailArgs<double> ta = tail_args<double>(c, H, l0, false);
  ta.zero = l0 > 0;
  HIP_TRY(c, launch_tail<double>(ta, c->stream));
  for (int l = l0 - 1; l >= 0; --l) FLD_TRY(up<double>(c, H, l));
  return FLD_OK;
}

// Launches after the stop flag was set return at once; the first `cycles`
// timed launches of the solve are the ones that did the work.
fld_status collect_timing(fld_ctx* c) {
  if (!c->timing) return FLD_OK;
  const size_t real = (size_t)std::max(0, c->host_ctrl->cycles);
  for (size_t i = 0; i + 1 < c->ev_used && i / 2 < real; i += 2) {
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
  if (c->net_clock) {
    HIP_TRY(c, hipEventRecord(c->net_ev[2], c->stream));
    c->net_ev_end = true;
  }
  if (c->ctrl_by_copy)
    HIP_TRY(c, hipMemcpyAsync(c->host_ctrl, c->ctrl, sizeof(Control),
                              hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return FLD_OK;
}

// FP64 V-cycles until the device stop flag is set.  Cycles are enqueued in
// batches between reads of the control block; a batch ends with the finest
// down pass and stop test of the cycle predicted to stop (the last step's
// count), so the rest of that cycle is not enqueued behind the test that
// ends the solve (its launches would return at once, but still cost their
// issue); when the test says to go on, the cycle is finished first.
fld_status solve_fp64(fld_ctx* c) {
  int nb = 0;
  if (!c->init_fused) {
    HIP_TRY(c, launch_resid_norm<double>(view(c, c->h64, 0), c->partials, &nb,
                                         c->ctrl, c->stream));
    HIP_TRY(c, launch_finalize(kFinInitial, c->partials, nb, c->ctrl,
                               c->stream));
  }
  if (c->fast && c->tail_l0 == 0) {
    // the whole problem fits one workgroup: one launch runs every cycle
    HIP_TRY(c, launch_tail<double>(tail_args<double>(c, c->h64, 0, true),
                                   c->stream));
    return read_control(c);
  }
  const bool split = c->fast && c->tail_l0 > 0;
  int enqueued = 0;
  bool open_cycle = false;  // the last batch stopped after a cycle's head
  int batch = c->last_batch < 1 ? 1 : c->last_batch;
  for (;;) {
    if (open_cycle) {
      FLD_TRY(vcycle_tail(c, c->h64));
      open_cycle = false;
    }
    if (batch > c->p.max_cycles - enqueued) batch = c->p.max_cycles - enqueued;
    for (int k = 0; k < batch; ++k) {
      c->fin_cycle = enqueued + k;
      const bool head_only = split && k == batch - 1;
      const fld_status st = head_only ? vcycle_head(c, c->h64)
                                      : vcycle<double>(c, c->h64, false);
      c->fin_cycle = -1;
      c->pending_fin = 0;
      FLD_TRY(st);
      open_cycle = head_only;
    }
    // a stop right after the finest down pass leaves the iterate in the
    // alternate buffer of the tiled path (the copy checks the device flag)
    if (tile_path(c))
      HIP_TRY(c, launch_take_alt(c->geom[0].N, c->h64.alt[0], c->h64.x[0],
                                 c->ctrl, c->stream));
    enqueued += batch;
    FLD_TRY(read_control(c));
    if (c->host_ctrl->done != kRunning || enqueued >= c->p.max_cycles) break;
    batch = 2;
  }
  if (c->host_ctrl->done == kConverged) c->last_batch = c->host_ctrl->cycles;
  return FLD_OK;
}

// FP32 V-cycles inside an FP64 iterative refinement.  The FP64 residual
// (with its FP32 copy and the stop test) is taken once up front and then at
// the end of every correction, so a batch is exactly the corrections the
// last step needed: no correction's V-cycles are enqueued behind the test
// that ends the solve (they would return at once, but still cost their
// launches).
fld_status solve_mixed(fld_ctx* c) {
  const Geom& g0 = c->geom[0];
  auto check = [&]() -> fld_status {
    int nb = 0;
    HIP_TRY(c, launch_resid_to32(view(c, c->h64, 0), c->h32.b[0], c->partials,
                                 &nb, c->ctrl, c->stream));
    HIP_TRY(c, launch_finalize(kFinOuter, c->partials, nb, c->ctrl, c->stream));
    return FLD_OK;
  };
  int enqueued = 0;
  int batch = c->last_batch < 1 ? 1 : c->last_batch;
  const int max_outer = c->p.max_cycles / c->inner + 2;
  FLD_TRY(check());
  for (;;) {
    for (int k = 0; k < batch; ++k) {
      for (int i = 0; i < c->inner; ++i)
        FLD_TRY(vcycle<float>(c, c->h32, i == 0));
      HIP_TRY(c, launch_correct(g0.N, c->h64.x[0], c->h32.x[0], c->ctrl,
                                c->stream));
      FLD_TRY(check());
    }
    enqueued += batch;
    FLD_TRY(read_control(c));
    if (c->host_ctrl->done != kRunning || enqueued >= max_outer) break;
    batch = 1;
  }
  if (c->host_ctrl->done == kRunning) c->host_ctrl->done = kCapped;
  if (c->host_ctrl->done == kConverged) c->last_batch = c->host_ctrl->outer;
  return FLD_OK;
}

// Face coefficients of every coarse level from the finest one's.
template <typename T>
fld_status coarsen_levels(fld_ctx* c, Levels<T>& H) {
  if constexpr (sizeof(T) == sizeof(double)) {
    if (H.sd[0])  // the Dirichlet walls' diagonal term on every level
      for (int l = 0; l + 1 < c->L; ++l)
        HIP_TRY(c, launch_coarsen_sd(c->geom[l], c->geom[l + 1], H.sd[l],
                                     H.sd[l + 1], c->stream));
    if (c->p.held_cells)  // held points: a coarse cell with a held child
      for (int l = 0; l + 1 < c->L; ++l)
        HIP_TRY(c, launch_coarsen_held(c->geom[l], c->geom[l + 1],
                                       l == 0 ? c->held_mask : H.held[l],
                                       H.held[l + 1], c->stream));
  }
  if (c->coarsen_multi && c->geom[0].ndim == 2) {
    HIP_TRY(c, launch_coarsen2d<T>(c->geom, c->L, H.a, c->stream));
    return FLD_OK;
  }
  for (int l = 0; l + 1 < c->L; ++l) {
    const T* fa[3] = {H.a[l][0], H.a[l][1], H.a[l][2]};
    T* ca[3] = {H.a[l + 1][0], H.a[l + 1][1], H.a[l + 1][2]};
    HIP_TRY(c, launch_coarsen<T>(c->geom[l], c->geom[l + 1], fa, ca,
                                 c->stream));
  }
  return FLD_OK;
}

// Flexible conjugate gradients preconditioned by V-cycles (FP64 V-cycles,
// or `inner` FP32 V-cycles in FP32_IR) until the device stop flag is set.
// The FP64 residual is carried by the recurrence r -= alpha A p; its norm
// is the stop test.  Iterations are enqueued in batches like the V-cycles
// of solve_fp64 (launches after the stop return at once).
//
// FP32 V-cycles cannot resolve a correction whose right-hand side is below
// their rounding of the large face terms (face coefficients many decades
// above 1): there the FP32-preconditioned iteration stops contracting.  The
// host watches the FP64 residual at every read of the control block; when it
// has fallen by less than kStallDrop over kStallIters iterations, the solve
// continues from its current iterate with FP64 V-cycles (FP64 coarse levels
// built then), and the next steps start with them (2, 4, 8, ... up to
// kMaxPre64Pause steps while the stall recurs).
constexpr int kStallIters = 4;
constexpr double kStallDrop = 0.25;
constexpr int kMaxPre64Pause = 32;

fld_status solve_krylov(fld_ctx* c) {
  const Geom& g0 = c->geom[0];
  KrylovArgs K{};
  K.g = g0;
  for (int d = 0; d < g0.ndim; ++d) K.a[d] = c->h64.a[0][d];
  K.r = c->kr_r;
  K.q = c->kr_q;
  K.partials = c->partials;
  K.ctrl = c->ctrl;
  // FP64 preconditioner: level 0 of the hierarchy solves A z = r from zero
  Levels<double> pre = c->h64;
  pre.x[0] = c->kr_z;
  pre.b[0] = c->kr_r;
  const int nb = krylov_blocks(g0);
  bool fp32 = c->mixed && c->pre64_skip == 0;
  if (c->mixed && !fp32) {  // step_impl initialised the control with inner 1
    --c->pre64_skip;
    FLD_TRY(coarsen_levels<double>(c, c->h64));
  }
  c->pre64_used = c->mixed && !fp32;
  K.r32 = fp32 ? c->h32.b[0] : nullptr;
  HIP_TRY(c, launch_fcg_init(K, c->h64.x[0], c->h64.b[0], c->stream));
  HIP_TRY(c, launch_finalize(kFinInitial, c->partials, nb, c->ctrl,
                             c->stream));
  const int max_iter = c->p.max_cycles + 1;
  int k = 0, k_first = 0;  // iteration count; first iteration of this run
  int k_mark = -1;         // stall watch: iteration and residual at a mark
  double res_mark = 0.0;
  int batch = c->last_batch < 1 ? 1 : c->last_batch;
  // an FP32 retry after a pause: the first batch (sized by the last, FP64,
  // step) is cut so that a stall shows after a few iterations
  if (fp32 && c->pre64_span > 0) batch = std::min(batch, 2 * kStallIters);
  c->precond = true;
  fld_status st = FLD_OK;
  for (;;) {
    for (int j = 0; j < batch && k < max_iter && st == FLD_OK; ++j, ++k) {
      K.p_old = c->kr_p[(k + 1) & 1];
      K.p_new = c->kr_p[k & 1];
      if (fp32) {
        for (int i = 0; i < c->inner && st == FLD_OK; ++i)
          st = vcycle<float>(c, c->h32, i == 0);
      } else {
        st = vcycle<double>(c, pre, true);
      }
      if (st != FLD_OK) break;
      const int first = k == k_first;
      hipError_t e = hipSuccess;
      if (!first) {
        e = fp32 ? launch_fcg_zq<float>(K, c->h32.x[0], c->stream)
                 : launch_fcg_zq<double>(K, c->kr_z, c->stream);
        if (e == hipSuccess) e = launch_fcg_scalar(0, K, c->stream);
      }
      if (e == hipSuccess)
        e = fp32 ? launch_fcg_dir<float>(K, c->h32.x[0], first, c->stream)
                 : launch_fcg_dir<double>(K, c->kr_z, first, c->stream);
      if (e == hipSuccess) e = launch_fcg_scalar(1, K, c->stream);
      if (e == hipSuccess) e = launch_fcg_update(K, c->h64.x[0], c->stream);
      if (e == hipSuccess)
        e = launch_finalize(kFinKrylov, c->partials, nb, c->ctrl, c->stream);
      if (e != hipSuccess)
        st = fail(c, FLD_ERR_DEVICE, "flexible CG launch: %s",
                  hipGetErrorString(e));
    }
    if (st != FLD_OK) break;
    st = read_control(c);
    if (st != FLD_OK || c->host_ctrl->done != kRunning || k >= max_iter) break;
    batch = 2;
    if (!fp32) continue;
    if (k_mark < 0 || k - k_mark < kStallIters) {
      if (k_mark < 0) {
        k_mark = k;
        res_mark = c->host_ctrl->res;
      }
      continue;
    }
    if (c->host_ctrl->res > kStallDrop * res_mark) {
      // FP32 V-cycles stalled: FP64 V-cycles from the current iterate
      fp32 = false;
      c->pre64_used = true;
      c->pre64_span = std::min(std::max(2, 2 * c->pre64_span), kMaxPre64Pause);
      c->pre64_skip = c->pre64_span;
      st = coarsen_levels<double>(c, c->h64);
      if (st != FLD_OK) break;
      K.r32 = nullptr;
      hipError_t e = launch_fcg_init(K, c->h64.x[0], c->h64.b[0], c->stream);
      if (e == hipSuccess)
        e = launch_finalize(kFinRestart, c->partials, nb, c->ctrl, c->stream);
      if (e != hipSuccess) {
        st = fail(c, FLD_ERR_DEVICE, "flexible CG restart: %s",
                  hipGetErrorString(e));
        break;
      }
      k_first = k;
    } else {
      k_mark = k;
      res_mark = c->host_ctrl->res;
    }
  }
  c->precond = false;
  FLD_TRY(st);
  if (c->host_ctrl->done == kRunning) c->host_ctrl->done = kCapped;
  if (c->host_ctrl->done == kConverged) {
    c->last_batch = c->host_ctrl->outer;
    // an FP32 run that converged ends the pause
    if (c->mixed && fp32 && !c->pre64_used) c->pre64_span = 0;
  }
  return FLD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Batched solve: many independent 2D grids per launch
// ---------------------------------------------------------------------------
//
// Each grid keeps an ordinary sub-context (its own slice of the workspace,
// its own control block and stop flag).  Every phase of a step is one launch
// over all grids: the per-grid arguments are laid out in a device table
// (rebuilt on the host each step and uploaded only when it changed), and
// blocks are mapped onto grids by prefix sums.  Grids that have converged
// skip their blocks.  Optionally the sequence of one batch of refinement
// iterations is captured once into a hipGraph and replayed.

namespace {

struct Image {
  std::vector<char> buf;
  template <typename X>
  size_t put(const std::vector<X>& v) {
    const size_t o = align_up(buf.size());
    buf.resize(o + v.size() * sizeof(X));
    if (!v.empty()) memcpy(buf.data() + o, v.data(), v.size() * sizeof(X));
    return o;
  }
};

struct Phase {  // one batched launch: table offset, block starts, counts
  size_t tab = 0, start = 0;
  int ng = 0, nblocks = 0;
};

}  // namespace

struct BatchState {
  int ng = 0;
  // kernel timing: the first finest-level down pass of the step (every grid
  // still running) is timed, without graph replay
  bool time_next = false;
  int tile_var[kMaxLevels][2] = {};  // tile shape per level index: down, up
  std::vector<fld_ctx*> sub;
  char* dev_tab = nullptr;  // device table area (end of the workspace)
  size_t tab_cap = 0;
  char* host_tab = nullptr;  // pinned staging of the table image
  std::vector<char> last;    // last image uploaded
  char* dev_aux = nullptr;   // tables of the pointwise calls
  char* host_aux = nullptr;
  size_t aux_cap = 0;
  // layout of the step image
  Phase ctrl, coef, fin_b, resid, fin_r, correct, fin_c, take;
  std::vector<Phase> coarsen, down[2], up;
  Phase tail[2];
  size_t tail_lds = 0;
  bool tail2d[2] = {false, false};  // every grid's tail fits the 2D register tail
  int maxL = 0, maxl0 = 0;
  bool graph_on = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_iters = 0;
  int last_batch = 3;
};

namespace {

template <typename X>
void add_phase(Image& im, Phase& ph, const std::vector<X>& jobs,
               const std::vector<int>& blocks) {
  ph.ng = (int)jobs.size();
  ph.tab = im.put(jobs);
  std::vector<int> start(jobs.size() + 1, 0);
  for (size_t g = 0; g < jobs.size(); ++g) start[g + 1] = start[g] + blocks[g];
  ph.nblocks = start.back();
  ph.start = im.put(start);
}

template <typename T>
Levels<T>& hier(fld_ctx* c);
template <>
Levels<double>& hier<double>(fld_ctx* c) { return c->h64; }
template <>
Levels<float>& hier<float>(fld_ctx* c) { return c->h32; }

template <typename T>
Tile2DArgs<T> tile_job(fld_ctx* c, int l, bool down, bool zero_init,
                       double* partials, int variant) {
  Levels<T>& H = hier<T>(c);
  Tile2DArgs<T> a{};
  a.g = c->geom[l];
  a.x = down ? H.x[l] : H.alt[l];
  a.xo = down ? H.alt[l] : H.x[l];
  a.b = H.b[l];
  a.ax = H.a[l][0];
  a.ay = H.a[l][1];
  a.gc = c->geom[l + 1];
  a.cb = down ? H.b[l + 1] : nullptr;
  a.ce = down ? nullptr : H.x[l + 1];
  a.partials = partials;
  a.zero_init = zero_init;
  a.ctrl = c->ctrl;
  tile2d_grid(a.g, down ? nu_pre(c->p, l) : nu_post(c->p, l), down, variant,
              &a.tiles_x, &a.tiles_y);
  a.vec = tile2d_vec_ok(a);
  return a;
}

// Build the step image for the current field pointers (levels of
// precision T carry the V-cycles).
template <typename T>
void build_image(fld_ctx* bc, Image& im, const double* dt,
                 const double* const* rho, const double* const* kappa,
                 const double* const* E_in, double* const* E_out) {
  BatchState* B = bc->batch;
  const int ng = B->ng;
  std::vector<JobCtrl> jc(ng);
  std::vector<JobCoef> jf(ng);
  std::vector<JobFinalize> fb(ng), fr(ng), fcy(ng);
  std::vector<JobResid> jr(ng);
  std::vector<JobCorrect> jx(ng);
  std::vector<JobTake> jt(ng);
  std::vector<int> bcoef(ng), bres(ng), one(ng, 1);
  for (int g = 0; g < ng; ++g) {
    fld_ctx* c = B->sub[g];
    const bool aliased = E_in[g] == E_out[g];
    c->h64.x[0] = E_out[g];
    c->h64.b[0] = aliased ? c->bcopy : const_cast<double*>(E_in[g]);
    jc[g] = {c->ctrl, c->p.rtol, c->p.max_cycles, c->inner, c->host_ctrl_dev};
    JobCoef& J = jf[g];
    J.A.g = c->geom[0];
    for (int d = 0; d < 3; ++d) {
      J.A.dx[d] = c->p.dx[d];
      J.A.gscale[d] = 1.0 / (12.0 * c->p.dx[d]);
    }
    J.A.dt = dt[g];
    J.A.c = c->p.c;
    J.A.limiter = c->p.limiter;
    J.A.face_mean = c->p.face_mean;
    J.E = E_in[g];
    J.rho = rho[g];
    J.kappa = kappa[g];
    for (int d = 0; d < 3; ++d) {
      J.O.a64[d] = c->h64.a[0][d];
      J.O.a32[d] = c->mixed ? c->h32.a[0][d] : nullptr;
    }
    J.O.copy_dst = aliased ? c->bcopy : E_out[g];
    // batched grids have no Dirichlet walls and no held cells
    J.O.sd = J.O.rhs = nullptr;
    J.O.held = nullptr;
    J.O.hold = nullptr;
    J.O.partials = c->partials;
    J.O.ctrl = c->ctrl;
    bcoef[g] = blocks_for(c->geom[0].N);
    fb[g] = {c->partials, bcoef[g], c->ctrl};
    LevelView<double> v0;
    v0.g = c->geom[0];
    v0.x = c->h64.x[0];
    v0.b = c->h64.b[0];
    for (int d = 0; d < 3; ++d) v0.a[d] = c->h64.a[0][d];
    v0.sd = nullptr;
    jr[g] = {v0, c->mixed ? c->h32.b[0] : nullptr, c->partials, c->ctrl};
    bres[g] = blocks_for(c->geom[0].N);
    fr[g] = {c->partials, bres[g], c->ctrl};
    jx[g] = {c->geom[0].N, c->h64.x[0], c->mixed ? c->h32.x[0] : nullptr,
             c->ctrl};
    jt[g] = {c->geom[0].N, c->h64.alt[0], c->h64.x[0], c->ctrl};
    fcy[g] = {c->partials,
              tile2d_blocks(c->geom[0], c->p.pre_smooth, true, B->tile_var[0][0]),
              c->ctrl};
  }
  add_phase(im, B->ctrl, jc, one);
  add_phase(im, B->coef, jf, bcoef);
  add_phase(im, B->fin_b, fb, one);
  add_phase(im, B->resid, jr, bres);
  add_phase(im, B->fin_r, fr, one);
  add_phase(im, B->correct, jx, bres);
  add_phase(im, B->take, jt, bres);
  add_phase(im, B->fin_c, fcy, one);
  // coarse face coefficients of precision T, per level index
  B->coarsen.assign(B->maxL > 1 ? B->maxL - 1 : 0, Phase());
  for (int l = 0; l + 1 < B->maxL; ++l) {
    std::vector<CoarsenArgs<T>> jobs;
    std::vector<int> blocks;
    for (int g = 0; g < ng; ++g) {
      fld_ctx* c = B->sub[g];
      if (l + 1 >= c->L) continue;
      Levels<T>& H = hier<T>(c);
      CoarsenArgs<T> a;
      a.f = c->geom[l];
      a.c = c->geom[l + 1];
      for (int d = 0; d < 3; ++d) {
        a.fa[d] = H.a[l][d];
        a.ca[d] = H.a[l + 1][d];
      }
      jobs.push_back(a);
      blocks.push_back(blocks_for(c->geom[l + 1].N));
    }
    add_phase(im, B->coarsen[l], jobs, blocks);
  }
  // multigrid tile passes per level index; variant 0 starts the finest
  // iterate at zero (first FP32 cycle of a refinement iteration)
  const bool mixed = B->sub[0]->mixed;
  for (int v = 0; v < 2; ++v) {
    B->down[v].assign(B->maxl0, Phase());
    for (int l = 0; l < B->maxl0; ++l) {
      std::vector<Tile2DArgs<T>> jobs;
      std::vector<int> blocks;
      for (int g = 0; g < ng; ++g) {
        fld_ctx* c = B->sub[g];
        if (l >= c->tail_l0) continue;
        const bool zero = l > 0 || (mixed && v == 0);
        double* parts = (!mixed && l == 0) ? c->partials : nullptr;
        jobs.push_back(tile_job<T>(c, l, true, zero, parts, B->tile_var[l][0]));
        blocks.push_back(tile2d_blocks(c->geom[l], nu_pre(c->p, l), true,
                                       B->tile_var[l][0]));
      }
      add_phase(im, B->down[v][l], jobs, blocks);
    }
    std::vector<TailArgs<T>> tails(ng);
    std::vector<int> ones(ng, 1);
    size_t lds = 0;
    for (int g = 0; g < ng; ++g) {
      fld_ctx* c = B->sub[g];
      TailArgs<T> t = tail_args<T>(c, hier<T>(c), c->tail_l0, false);
      t.zero = c->tail_l0 > 0 || (mixed && v == 0);
      tails[g] = t;
      lds = std::max(lds, tail_lds_bytes<T>(t));
    }
    add_phase(im, B->tail[v], tails, ones);
    B->tail_lds = lds;
    bool t2 = true;
    for (int g = 0; g < ng; ++g) t2 = t2 && tail2d_ok(tails[g]);
    B->tail2d[v] = t2;
  }
  B->up.assign(B->maxl0, Phase());
  for (int l = 0; l < B->maxl0; ++l) {
    std::vector<Tile2DArgs<T>> jobs;
    std::vector<int> blocks;
    for (int g = 0; g < ng; ++g) {
      fld_ctx* c = B->sub[g];
      if (l >= c->tail_l0) continue;
      jobs.push_back(tile_job<T>(c, l, false, false, nullptr, B->tile_var[l][1]));
      blocks.push_back(tile2d_blocks(c->geom[l], nu_post(c->p, l), false,
                                     B->tile_var[l][1]));
    }
    add_phase(im, B->up[l], jobs, blocks);
  }
}

template <typename X>
const X* tab_ptr(BatchState* B, const Phase& ph) {
  return (const X*)(B->dev_tab + ph.tab);
}
inline const int* start_ptr(BatchState* B, const Phase& ph) {
  return (const int*)(B->dev_tab + ph.start);
}

// One V-cycle of precision T over all grids.  `var`: 0 = the finest iterate
// starts at zero.
template <typename T>
fld_status batch_vcycle(fld_ctx* bc, int var) {
  BatchState* B = bc->batch;
  hipStream_t s = bc->stream;
  const fld_params& p = B->sub[0]->p;
  for (int l = 0; l < B->maxl0; ++l) {
    const Phase& ph = B->down[var][l];
    // x (unless zero), b, two face arrays read; x and the coarse rhs written
    double bytes = 0.0;
    const bool timed = l == 0 && B->time_next;
    if (timed) {
      const double w = sizeof(T);
      for (fld_ctx* c : B->sub)
        bytes += (double)c->geom[0].N * (w * (var == 0 ? 4.0 : 5.0) + w / 4.0);
      B->time_next = false;
    }
    TimedLaunch t(bc, timed, bytes,
                  sizeof(T) == 8 ? "k_tile2d_batch<double,down>"
                                 : "k_tile2d_batch<float,down>");
    FLD_TRY(t.st);
    HIP_TRY(bc, launch_tile2d_batch<T>(tab_ptr<Tile2DArgs<T>>(B, ph),
                                       start_ptr(B, ph), ph.ng, ph.nblocks,
                                       nu_pre(p, l), true, B->tile_var[l][0],
                                       s, t.e0, t.e1));
    if (sizeof(T) == 8 && l == 0)
      HIP_TRY(bc, launch_finalize_batch(kFinCycle,
                                        tab_ptr<JobFinalize>(B, B->fin_c),
                                        B->fin_c.ng, s));
  }
  if (B->tail2d[var])
    HIP_TRY(bc, launch_tail2d_batch<T>(tab_ptr<TailArgs<T>>(B, B->tail[var]),
                                       B->tail[var].ng, s));
  else
    HIP_TRY(bc, launch_tail_lds_batch<T>(tab_ptr<TailArgs<T>>(B, B->tail[var]),
                                         B->tail[var].ng, 2, B->tail_lds, s));
  for (int l = B->maxl0 - 1; l >= 0; --l) {
    const Phase& ph = B->up[l];
    HIP_TRY(bc, launch_tile2d_batch<T>(tab_ptr<Tile2DArgs<T>>(B, ph),
                                       start_ptr(B, ph), ph.ng, ph.nblocks,
                                       nu_post(p, l), false, B->tile_var[l][1],
                                       s));
  }
  return FLD_OK;
}

// FP64 residual, its FP32 copy and the refinement stop test of every grid.
fld_status batch_check(fld_ctx* bc) {
  BatchState* B = bc->batch;
  hipStream_t s = bc->stream;
  HIP_TRY(bc, launch_resid_batch(tab_ptr<JobResid>(B, B->resid),
                                 start_ptr(B, B->resid), B->resid.ng,
                                 B->resid.nblocks, s));
  HIP_TRY(bc, launch_finalize_batch(kFinOuter, tab_ptr<JobFinalize>(B, B->fin_r),
                                    B->fin_r.ng, s));
  return FLD_OK;
}

// One refinement correction followed by its check (mixed; the first check
// comes before the iterations), or one V-cycle (FP64), over all grids.
fld_status batch_iteration(fld_ctx* bc) {
  BatchState* B = bc->batch;
  hipStream_t s = bc->stream;
  if (!B->sub[0]->mixed) return batch_vcycle<double>(bc, 1);
  const int inner = B->sub[0]->inner;
  for (int i = 0; i < inner; ++i) FLD_TRY(batch_vcycle<float>(bc, i == 0 ? 0 : 1));
  HIP_TRY(bc, launch_correct_batch(tab_ptr<JobCorrect>(B, B->correct),
                                   start_ptr(B, B->correct), B->correct.ng,
                                   B->correct.nblocks, s));
  return batch_check(bc);
}

// `iters` iterations, replayed from a captured graph when enabled.
fld_status batch_iterations(fld_ctx* bc, int iters) {
  BatchState* B = bc->batch;
  if (!B->graph_on) {
    for (int k = 0; k < iters; ++k) FLD_TRY(batch_iteration(bc));
    return FLD_OK;
  }
  if (!B->gexec || B->graph_iters != iters) {
    if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->gexec = nullptr;
    B->graph = nullptr;
    HIP_TRY(bc, hipStreamBeginCapture(bc->stream, hipStreamCaptureModeRelaxed));
    fld_status st = FLD_OK;
    for (int k = 0; k < iters && st == FLD_OK; ++k) st = batch_iteration(bc);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(bc->stream, &g);
    if (st != FLD_OK) return st;
    if (e != hipSuccess)
      return fail(bc, FLD_ERR_DEVICE, "hipStreamEndCapture: %s",
                  hipGetErrorString(e));
    B->graph = g;
    HIP_TRY(bc, hipGraphInstantiate(&B->gexec, g, nullptr, nullptr, 0));
    B->graph_iters = iters;
  }
  HIP_TRY(bc, hipGraphLaunch(B->gexec, bc->stream));
  return FLD_OK;
}

bool all_stopped(BatchState* B) {
  for (fld_ctx* c : B->sub)
    if (c->host_ctrl->done == kRunning) return false;
  return true;
}

template <typename T>
fld_status batch_step_impl(fld_ctx* bc, const double* dt,
                           const double* const* rho, const double* const* kappa,
                           const double* const* E_in, double* const* E_out) {
  BatchState* B = bc->batch;
  hipStream_t s = bc->stream;
  Image im;
  build_image<T>(bc, im, dt, rho, kappa, E_in, E_out);
  if (im.buf.size() > B->tab_cap)
    return fail(bc, FLD_ERR_WORKSPACE, "batch table needs %zu bytes, has %zu",
                im.buf.size(), B->tab_cap);
  if (im.buf != B->last) {
    memcpy(B->host_tab, im.buf.data(), im.buf.size());
    HIP_TRY(bc, hipMemcpyAsync(B->dev_tab, B->host_tab, im.buf.size(),
                               hipMemcpyHostToDevice, s));
    B->last = im.buf;
  }
  HIP_TRY(bc, launch_ctrl_init_batch(tab_ptr<JobCtrl>(B, B->ctrl), B->ctrl.ng, s));
  HIP_TRY(bc, launch_coef_batch(tab_ptr<JobCoef>(B, B->coef),
                                start_ptr(B, B->coef), B->coef.ng,
                                B->coef.nblocks, s));
  HIP_TRY(bc, launch_finalize_batch(kFinBnorm, tab_ptr<JobFinalize>(B, B->fin_b),
                                    B->fin_b.ng, s));
  for (size_t l = 0; l < B->coarsen.size(); ++l) {
    const Phase& ph = B->coarsen[l];
    HIP_TRY(bc, launch_coarsen_batch<T>(tab_ptr<CoarsenArgs<T>>(B, ph),
                                        start_ptr(B, ph), ph.ng, ph.nblocks, s));
  }
  if (sizeof(T) == 8) {
    HIP_TRY(bc, launch_resid_batch(tab_ptr<JobResid>(B, B->resid),
                                   start_ptr(B, B->resid), B->resid.ng,
                                   B->resid.nblocks, s));
    HIP_TRY(bc, launch_finalize_batch(kFinInitial,
                                      tab_ptr<JobFinalize>(B, B->fin_r),
                                      B->fin_r.ng, s));
  }
  int maxc = 0;
  for (fld_ctx* c : B->sub) maxc = std::max(maxc, c->p.max_cycles);
  const int max_iters =
      B->sub[0]->mixed ? maxc / B->sub[0]->inner + 2 : maxc;
  int done_iters = 0;
  int batch = B->last_batch < 1 ? 1 : B->last_batch;
  B->time_next = bc->timing && !B->graph_on;
  if (B->sub[0]->mixed) FLD_TRY(batch_check(bc));
  for (;;) {
    if (batch > max_iters - done_iters) batch = max_iters - done_iters;
    if (batch < 1) break;
    FLD_TRY(batch_iterations(bc, batch));
    if (!B->sub[0]->mixed)  // FP64: a grid may stop after its down pass
      HIP_TRY(bc, launch_take_batch(tab_ptr<JobTake>(B, B->take),
                                    start_ptr(B, B->take), B->take.ng,
                                    B->take.nblocks, s));
    done_iters += batch;
    FLD_TRY(read_control(bc));
    if (all_stopped(B) || done_iters >= max_iters) break;
    batch = 1;
  }
  if (all_stopped(B)) B->last_batch = done_iters;
  // the timed launches ran while every grid was running: all count
  for (size_t i = 0; i + 1 < bc->ev_used; i += 2) {
    float ms = 0.f;
    HIP_TRY(bc, hipEventElapsedTime(&ms, bc->ev[i], bc->ev[i + 1]));
    bc->t_ms += ms;
    bc->t_launches += 1;
    bc->t_bytes += bc->ev_bytes[i / 2];
  }
  bc->ev_used = 0;
  bc->ev_bytes.clear();
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
  p->coarse_pre_smooth = 0;
  p->coarse_post_smooth = 0;
}

size_t fld_workspace_bytes(const fld_params* p) {
  if (!validate(p).empty()) return 0;
  Plan P;
  make_plan(p, &P);
  return P.total;
}

}  // extern "C"

namespace {

// Validate the parameters and the workspace and plan the levels.
fld_status check_setup(const fld_params* p, const void* workspace,
                       size_t ws_bytes, Plan& P) {
  std::string why = validate(p);
  if (!why.empty()) return fail(nullptr, FLD_ERR_INVALID_ARG, "%s", why.c_str());
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
  return FLD_OK;
}

// First level of the single-workgroup tail: the first of at most 1024
// cells, or the level above it where the 2D tail from a level of up to
// 4096 cells fits (c->tail_big).
void choose_tail(fld_ctx* c) {
  c->tail_l0 = c->L - 1;
  for (int l = 0; l < c->L; ++l)
    if (c->geom[l].N <= kTailLdsCells) {
      c->tail_l0 = l;
      break;
    }
  if (c->fast && c->tail_big && c->tail_l0 >= 2 &&
      tail2d_big_fits(c->geom + c->tail_l0 - 1, c->L - c->tail_l0 + 1))
    c->tail_l0 -= 1;
}

// Point a context's level buffers into the workspace and apply the
// environment switches of the tests (kernel path, coarsening form, fused
// 3D sweeps, tiled 3D sweeps, 2D tail start, fixed tile shape).  Allocates
// nothing.
void fill_ctx(fld_ctx* c, const fld_params* p, const Plan& P, void* workspace,
              size_t ws_bytes, void* hip_stream) {
  c->p = *p;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace;
  c->ws_bytes = ws_bytes;
  c->L = P.L;
  c->mixed = p->precision == FLD_PREC_FP32_IR;
  c->inner = p->ir_inner > 0 ? p->ir_inner : 2;
  char* w = c->ws;
  for (int l = 0; l < P.L; ++l) {
    c->geom[l] = P.g[l];
    const bool has64 = l == 0 || !c->mixed || p->krylov;
    for (int d = 0; d < p->ndim; ++d) {
      c->h64.a[l][d] = has64 ? (double*)(w + P.a64[l][d]) : nullptr;
      c->h32.a[l][d] = c->mixed ? (float*)(w + P.a32[l][d]) : nullptr;
    }
    c->h64.x[l] = (has64 && l > 0) ? (double*)(w + P.x64[l]) : nullptr;
    c->h64.b[l] = (has64 && l > 0) ? (double*)(w + P.b64[l]) : nullptr;
    c->h32.x[l] = c->mixed ? (float*)(w + P.x32[l]) : nullptr;
    c->h32.b[l] = c->mixed ? (float*)(w + P.b32[l]) : nullptr;
    if (P.alt[l]) {
      if (c->mixed)
        c->h32.alt[l] = (float*)(w + P.alt[l]);
      else
        c->h64.alt[l] = (double*)(w + P.alt[l]);
    }
    if (P.alt64[l]) c->h64.alt[l] = (double*)(w + P.alt64[l]);
    c->h64.sd[l] = P.sd64[l] ? (double*)(w + P.sd64[l]) : nullptr;
    c->h64.held[l] = P.held[l] ? (uint8_t*)(w + P.held[l]) : nullptr;
  }
  const char* path = getenv("FLD_KERNEL_PATH");
  // Dirichlet walls and held cells: the one-launch-per-pass kernels (the
  // only ones with the extra diagonal term)
  c->fast = !(path && strcmp(path, "simple") == 0) && !own_rows(*p);
  // one coarsening launch per level (tests that both forms agree bitwise)
  c->coarsen_multi = c->fast && !getenv("FLD_COARSEN_PER_LEVEL");
  // 3D smoothing by colour passes only ("0"; tests that both forms agree),
  // or fused sweeps with a fixed number of z planes per block (a number > 1)
  if (const char* sw = getenv("FLD_SWEEP3D")) {
    const int v = atoi(sw);
    c->sweep3d = v != 0;
    if (v > 1) c->sweep_zc = v;
  }
  c->sweep3d = c->sweep3d && c->fast;
  // small 3D coarse levels by colour-pass launches ("0"; tests that both
  // forms agree bitwise)
  if (const char* lv = getenv("FLD_LEVEL_LDS")) c->level_lds = atoi(lv) != 0;
  // 3D levels below the marching sweeps by colour passes ("0"; tests that
  // both forms agree bitwise), or tiled sweeps on every level ("2")
  if (const char* tv = getenv("FLD_TILE3D")) {
    c->tile3d = atoi(tv) != 0;
    c->tile3d_all = atoi(tv) == 2;
  }
  c->level_lds = c->level_lds && c->fast;
  // fixed tile shape for every level (tests of shape independence)
  if (const char* tv = getenv("FLD_TILE_VARIANT")) {
    const int v = atoi(tv);
    if (v >= 0 && v < kTileVariants)
      for (int l = 0; l < kMaxLevels; ++l) c->tile_var[l][0] = c->tile_var[l][1] = v;
  }
  // a 2D tail starts one level higher where that level (not the finest)
  // has at most 4096 cells: two launches fewer per V-cycle ("0": the tail
  // from the first level of at most 1024 cells; tests that both forms
  // agree bitwise)
  if (const char* tb = getenv("FLD_TAIL_BIG")) c->tail_big = atoi(tb) != 0;
  choose_tail(c);
  c->bcopy = (double*)(w + P.bcopy);
  c->dscr = P.dscr ? (double*)(w + P.dscr) : nullptr;
  c->partials = (double*)(w + P.partials);
  c->h64.tmp = (double*)(w + P.tmp);
  c->h32.tmp = (float*)(w + P.tmp);
  c->ctrl = (Control*)(w + P.ctrl);
  if (p->ndim >= 2) c->mean = (double*)(w + P.mean);
  if (p->guess == FLD_GUESS_LEARNED) {
    c->net_ws = w + P.net;
    c->net_bytes = P.net_bytes;
    c->guess = (double*)(w + P.guess);
  }
  c->krylov = p->krylov != 0;
  if (c->krylov) {
    c->kr_r = (double*)(w + P.kr_r);
    c->kr_p[0] = (double*)(w + P.kr_p[0]);
    c->kr_p[1] = (double*)(w + P.kr_p[1]);
    c->kr_q = (double*)(w + P.kr_q);
    c->kr_z = P.kr_z ? (double*)(w + P.kr_z) : nullptr;
  }
}

}  // namespace

extern "C" {

fld_status fld_setup(const fld_params* p, void* workspace, size_t ws_bytes,
                     void* hip_stream, fld_ctx** out) {
  if (!out) return fail(nullptr, FLD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  Plan P;
  FLD_TRY(check_setup(p, workspace, ws_bytes, P));
  fld_ctx* c = new fld_ctx();
  fill_ctx(c, p, P, workspace, ws_bytes, hip_stream);
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

namespace {

// Learned guess, entirely on the device.  Both candidates, E^n (already in
// x) and the network's E^n (1 + delta), get the finest level's
// pre-smoothing of a V-cycle; the one with the smaller FP64 residual
// becomes the iterate the solve starts from (the decision lands in
// ctrl->guess_rejected).  Judging after smoothing ignores the
// high-frequency part of the network's error, which one smoothing pass
// removes, and keeps the smooth part that decides the number of cycles.
fld_status learned_guess(fld_ctx* c, const double* rho, const double* kappa) {
  const LevelView<double> v0 = view(c, c->h64, 0);
  LevelView<double> vg = v0;
  vg.x = c->guess;
  const Geom& g = c->geom[0];
  const int64_t slice = (int64_t)g.n[0] * g.n[1];
  HIP_TRY(c, nn::launch_mean_log(v0.b, slice, g.n[2], c->mean,
                                     c->mean + g.n[2], c->stream));
  HIP_TRY(c, nn::launch_features(v0.b, rho, kappa, c->h64.a[0][0],
                                 c->h64.a[0][1], c->p.dx[0], c->mean, g.N,
                                 slice, nn::input_ptr(c->net), nullptr,
                                 c->stream));
  HIP_TRY(c, nn::forward_x(c->net));
  HIP_TRY(c, nn::launch_apply_guess(v0.b, nn::delta_ptr(c->net), g.N, vg.x,
                                    c->stream));
  const int sweeps = c->p.pre_smooth > 0 ? c->p.pre_smooth : 1;
  int nb = 0;
  for (int mode = 0; mode < 2; ++mode) {
    const LevelView<double>& v = mode == 0 ? v0 : vg;
    for (int k = 0; k < sweeps; ++k)
      for (int color = 0; color < gs_colors(v.g); ++color)
        HIP_TRY(c, launch_gs_color<double>(v, color, c->ctrl, c->stream));
    HIP_TRY(c, launch_resid_norm<double>(v, c->partials, &nb, c->ctrl,
                                         c->stream));
    HIP_TRY(c, launch_guess_judge(mode, c->partials, nb, c->judge_q2, c->ctrl,
                                  c->stream));
  }
  HIP_TRY(c, launch_guess_take(g.N, vg.x, v0.x, c->ctrl, c->stream));
  return FLD_OK;
}

}  // namespace

}  // extern "C"

// ---- hooks for the block-adaptive step (fld_hooks.h) ----

fld_status fld::precond_begin(fld_ctx* c, double dt, const double* E,
                              const double* rho, const double* kappa) {
  if (c->mixed || c->batch || c->p.guess == FLD_GUESS_LEARNED)
    return fail(c, FLD_ERR_INVALID_ARG, "preconditioner: an FP64 single grid");
  const Geom& g0 = c->geom[0];
  // no stop test: the kernels only need the control block to say running
  HIP_TRY(c, launch_ctrl_init(c->ctrl, c->p.rtol, INT_MAX / 2, 1,
                             c->host_ctrl_dev, c->stream));
  CoefArgs A;
  A.g = g0;
  for (int d = 0; d < 3; ++d) {
    A.dx[d] = c->p.dx[d];
    A.gscale[d] = 1.0 / (12.0 * c->p.dx[d]);
    A.wall[d][0] = A.wall[d][1] = 0.0;
  }
  A.dt = dt;
  A.c = c->p.c;
  A.limiter = c->p.limiter;
  A.face_mean = c->p.face_mean;
  c->init_fused = false;
  if (coef2d_ok(g0)) {
    HIP_TRY(c, launch_coef2d(A, E, rho, kappa, c->h64.a[0], c->h32.a[0],
                             nullptr, c->partials, c->ctrl, false, c->stream));
  } else {
    int nb = 0;
    HIP_TRY(c, launch_coef(A, E, rho, kappa, c->h64.a[0], c->h32.a[0],
                           nullptr, c->partials, c->ctrl, c->stream, &nb,
                           c->dscr));
  }
  FLD_TRY(coarsen_levels<double>(c, c->h64));
  c->precond = true;
  return FLD_OK;
}

fld_status fld::precond_vcycle(fld_ctx* c, const double* rhs, double* z) {
  Levels<double> pre = c->h64;
  pre.x[0] = z;
  pre.b[0] = const_cast<double*>(rhs);
  return vcycle<double>(c, pre, true);
}

void fld::base_faces(const fld_ctx* c, const double** ax, const double** ay) {
  *ax = c->h64.a[0][0];
  *ay = c->h64.a[0][1];
}

void fld::precond_end(fld_ctx* c) { c->precond = false; }

hipStream_t fld::ctx_stream(const fld_ctx* c) { return c->stream; }

const char* fld::ctx_error(const fld_ctx* c) { return c->err.c_str(); }

extern "C" {

static fld_status step_impl(fld_ctx* c, double dt, const double* rho,
                            const double* kappa, const double* E_in,
                            double* E_out, fld_stats* stats) {
  if (!c) return fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (!rho || !kappa || !E_in || !E_out)
    return fail(c, FLD_ERR_INVALID_ARG, "NULL field pointer");
  if (!(dt > 0.0) || !std::isfinite(dt))
    return fail(c, FLD_ERR_INVALID_ARG, "dt must be positive and finite");
  if (c->p.guess == FLD_GUESS_LEARNED && !c->net)
    return fail(c, FLD_ERR_MODEL, "no model: call fld_set_model first");
  if (c->p.held_cells && !c->held_mask)
    return fail(c, FLD_ERR_INVALID_ARG,
                "held_cells: give the mask and values by fld_set_held first");
  const bool aliased = (E_in == E_out);
  const Geom& g0 = c->geom[0];
  const bool learned = c->p.guess == FLD_GUESS_LEARNED;
  const bool use_net = learned && (c->p.guess_policy == FLD_GUESS_EVERY_STEP ||
                                   c->net_skip == 0);
  // a learned-guess step without its network is a step with guess E^n
  const bool prev_guess = c->p.guess == FLD_GUESS_PREV || (learned && !use_net);
  // level 0: x = E_out, b = E_in (or its copy when E_out overwrites it);
  // with Dirichlet walls or held cells b is always the copy, which the
  // coefficient stage writes: E^n + sum alpha_w E_w beside the walls'
  // diagonal term, the prescribed values in the held cells, and in a free
  // cell next to held ones their values times its faces to them
  const bool own_b = own_rows(c->p);
  const bool held = c->p.held_cells != 0;
  c->h64.x[0] = E_out;
  c->h64.b[0] = (aliased || own_b) ? c->bcopy : const_cast<double*>(E_in);
  double* copy_dst =
      (aliased && !own_b) ? c->bcopy
      : (aliased || c->p.guess == FLD_GUESS_ZERO) ? nullptr
                                                  : E_out;
  // V-cycles per iteration: flexible CG with FP64 V-cycles runs one
  const bool one_inner =
      c->krylov && (!c->mixed || c->pre64_skip > 0);
  HIP_TRY(c, launch_ctrl_init(c->ctrl, c->p.rtol, c->p.max_cycles,
                             one_inner ? 1 : c->inner, c->host_ctrl_dev,
                             c->stream));
  CoefArgs A;
  A.g = g0;
  for (int d = 0; d < 3; ++d) {
    A.dx[d] = c->p.dx[d];
    A.gscale[d] = 1.0 / (12.0 * c->p.dx[d]);
  }
  A.dt = dt;
  A.c = c->p.c;
  A.limiter = c->p.limiter;
  A.face_mean = c->p.face_mean;
  for (int d = 0; d < 3; ++d) {
    A.wall[d][0] = c->p.bc_value_lo[d];
    A.wall[d][1] = c->p.bc_value_hi[d];
  }
  // 2D grids: the LDS-tiled coefficient stage; with x0 = E^n in FP64 it also
  // forms the initial residual, so the solve needs no separate first pass
  // (Dirichlet walls, held cells: the one-pass kernels, which write b)
  const bool tiled_coef = coef2d_ok(g0) && !own_b;
  c->init_fused = tiled_coef && !c->mixed && prev_guess && !c->krylov;
  if (tiled_coef) {
    HIP_TRY(c, launch_coef2d(A, E_in, rho, kappa, c->h64.a[0], c->h32.a[0],
                             copy_dst, c->partials, c->ctrl, c->init_fused,
                             c->stream));
    HIP_TRY(c, launch_finalize(c->init_fused ? kFinCoef : kFinBnorm,
                               c->partials, coef2d_blocks(g0), c->ctrl,
                               c->stream));
  } else {
    int nb = 0;
    HIP_TRY(c, launch_coef(A, E_in, rho, kappa, c->h64.a[0], c->h32.a[0],
                           copy_dst, c->partials, c->ctrl, c->stream, &nb,
                           c->dscr, c->h64.sd[0], own_b ? c->bcopy : nullptr,
                           held ? c->held_mask : nullptr,
                           held ? c->held_vals : nullptr));
    if (!held)
      HIP_TRY(c, launch_finalize(kFinBnorm, c->partials, nb, c->ctrl,
                                 c->stream));
  }
  FLD_TRY(c->mixed ? coarsen_levels<float>(c, c->h32)
                   : coarsen_levels<double>(c, c->h64));
  if (held) {
    // with the coarse levels built from the uncut faces, the held cells
    // leave the finest level's free rows (their faces become diagonal and
    // right-hand-side terms) and their faces are cut: a held row is
    // x = E_hold, the free block is symmetric
    int nb = 0;
    HIP_TRY(c, launch_held_fold(g0, c->h64.a[0], c->held_mask, c->held_vals,
                                c->h64.sd[0], c->bcopy, c->partials, &nb,
                                c->stream));
    HIP_TRY(c, launch_held_cut(g0, c->h64.a[0], c->held_mask, c->stream));
    HIP_TRY(c, launch_finalize(kFinBnorm, c->partials, nb, c->ctrl,
                               c->stream));
  }
  if (c->p.guess == FLD_GUESS_ZERO)
    HIP_TRY(c, launch_fill(E_out, g0.N, 0.0, c->stream));
  // the adaptive policy times the network and the solve on the stream
  const bool adaptive = learned && c->p.guess_policy == FLD_GUESS_ADAPTIVE;
  if (adaptive) {
    // the two events inside the step skip the system-scope fence (a default
    // event writes back and invalidates the caches where it is recorded);
    // the one before the solve's synchronisation keeps it, as the last
    // command the host waits for
    for (int k = 0; k < 2; ++k)
      if (!c->net_ev[k])
        HIP_TRY(c, hipEventCreateWithFlags(&c->net_ev[k],
                                           hipEventDisableSystemFence));
    if (!c->net_ev[2]) HIP_TRY(c, hipEventCreate(&c->net_ev[2]));
  }
  c->net_clock = adaptive;
  c->net_ev_end = false;
  if (use_net) {
    if (adaptive) HIP_TRY(c, hipEventRecord(c->net_ev[0], c->stream));
    FLD_TRY(learned_guess(c, rho, kappa));
  }
  if (adaptive) HIP_TRY(c, hipEventRecord(c->net_ev[1], c->stream));
  const fld_status solved = c->krylov ? solve_krylov(c)
                                      : (c->mixed ? solve_mixed(c)
                                                  : solve_fp64(c));
  c->net_clock = false;
  FLD_TRY(solved);
  FLD_TRY(collect_timing(c));
  const Control& h = *c->host_ctrl;
  if (adaptive && h.done == kConverged) {
    // the solve's last control read recorded net_ev[2] and synchronised
    float solve_ms = 0.f, net_ms = 0.f;
    bool timed = c->net_ev_end &&
                 hipEventElapsedTime(&solve_ms, c->net_ev[1], c->net_ev[2]) ==
                     hipSuccess;
    if (timed && use_net)
      timed = hipEventElapsedTime(&net_ms, c->net_ev[0], c->net_ev[1]) ==
              hipSuccess;
    if (!timed) (void)hipGetLastError();  // no stale error for later launches
    const int units = c->mixed ? h.outer : h.cycles;
    if (!use_net) {
      c->plain_units = units;
      if (units > 0 && timed) c->unit_ms = solve_ms / units;
      if (c->net_skip > 0) --c->net_skip;
      if (units > 0 && h.res_initial > 0.0 && h.res > 0.0) {
        const double rho = std::pow(h.res / h.res_initial, 1.0 / units);
        const double r = std::min(std::max(rho, 1e-3), 1.0);
        c->judge_q2 = r * r;
      }
    } else {
      // the guess pays when the work it saved took longer than the
      // network; a solve still runs at least one cycle or iteration (its
      // stop test follows one), so when the network costs more than all
      // the others of a solve without it, no guess can repay it, and the
      // next try waits the longest
      const bool known = timed && c->plain_units >= 0 && c->unit_ms > 0.0;
      const double saved_ms =
          known ? (c->plain_units - units) * c->unit_ms : 0.0;
      const bool pays = !h.guess_rejected && known && saved_ms > net_ms;
      if (known && net_ms >= (c->plain_units - 1) * c->unit_ms) {
        c->net_span = kMaxNetPause;
        c->net_skip = kMaxNetPause;
      } else if (!pays) {
        c->net_span = std::min(std::max(2, 2 * c->net_span), kMaxNetPause);
        c->net_skip = c->net_span;
      } else {
        c->net_span = 0;
      }
    }
  }
  if (stats) {
    memset(stats, 0, sizeof *stats);
    stats->cycles = h.cycles;
    stats->guess_rejected = use_net ? h.guess_rejected : 0;
    stats->guess_skipped = learned && !use_net;
    stats->outer_iters = (c->mixed || c->krylov) ? h.outer : 0;
    stats->precond_fp64 = c->krylov && c->mixed && c->pre64_used;
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

fld_status fld_step(fld_ctx* c, double dt, const double* rho,
                    const double* kappa, const double* E_in, double* E_out,
                    fld_stats* stats) {
  return step_impl(c, dt, rho, kappa, E_in, E_out, stats);
}

fld_status fld_step_noalloc(const fld_params* p, double dt, const double* rho,
                            const double* kappa, const double* E_in,
                            double* E_out, fld_stats* stats,
                            void* hip_stream) {
  if (!p) return fail(nullptr, FLD_ERR_INVALID_ARG, "params is NULL");
  if (p->guess == FLD_GUESS_LEARNED)
    return fail(nullptr, FLD_ERR_INVALID_ARG,
                "fld_step_noalloc takes guess E^n or zero (the learned guess "
                "needs a context with a model)");
  if (p->held_cells)
    return fail(nullptr, FLD_ERR_INVALID_ARG,
                "fld_step_noalloc has no held cells (they are given to a "
                "context by fld_set_held)");
  void* ws = nullptr;
  FLD_TRY(static_scratch(&ws));
  Plan P;
  if (validate(p).empty()) {
    make_plan(p, &P);
    if (P.total > kScratchBytes)
      return fail(nullptr, FLD_ERR_WORKSPACE,
                  "fld_step_noalloc: this grid needs %zu bytes of workspace, "
                  "the static scratch holds %zu",
                  P.total, (size_t)kScratchBytes);
  }
  FLD_TRY(check_setup(p, ws, kScratchBytes, P));
  fld_ctx c;  // host-side state only, on this call's stack
  fill_ctx(&c, p, P, ws, kScratchBytes, hip_stream);
  c.host_ctrl = &c.host_copy;  // no mapped mirror: read_control copies
  c.host_ctrl_dev = nullptr;
  c.ctrl_by_copy = true;
  const fld_status st = step_impl(&c, dt, rho, kappa, E_in, E_out, stats);
  if (st != FLD_OK) g_err = c.err;
  // the step has synchronised with the stream (its stop test reads the
  // control block), so nothing of this call is still in flight
  return st;
}

fld_status fld_set_held(fld_ctx* c, const uint8_t* mask,
                        const double* E_hold) {
  if (!c) return fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (c->batch)
    return fail(c, FLD_ERR_INVALID_ARG, "batched contexts have no held cells");
  if (!c->p.held_cells)
    return fail(c, FLD_ERR_INVALID_ARG,
                "the context was set up with held_cells = 0");
  if ((mask == nullptr) != (E_hold == nullptr))
    return fail(c, FLD_ERR_INVALID_ARG, "give both mask and E_hold, or neither");
  c->held_mask = mask;
  c->held_vals = E_hold;
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

fld_status fld_explicit_sources(fld_ctx* c, const double* rho,
                                const double* kappa, const double* E,
                                const double* const* v, double* const* f_r,
                                double* work, double* tiring, double* fedd) {
  if (!c) return fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (c->batch)
    return fail(c, FLD_ERR_INVALID_ARG, "batched contexts have no explicit "
                                        "source call");
  if (has_dirichlet(c->p))
    return fail(c, FLD_ERR_INVALID_ARG, "explicit sources take periodic or "
                                        "Neumann walls");
  if (!rho || !kappa || !E)
    return fail(c, FLD_ERR_INVALID_ARG, "NULL field pointer");
  const Geom& g = c->geom[0];
  ExplicitArgs a{};
  a.g = g;
  a.limiter = c->p.limiter;
  a.E = E;
  a.rho = rho;
  a.kappa = kappa;
  for (int d = 0; d < g.ndim; ++d) a.gscale[d] = 1.0 / (12.0 * c->p.dx[d]);
  if ((work || tiring) && !v)
    return fail(c, FLD_ERR_INVALID_ARG, "work and tiring need the velocity");
  for (int d = 0; d < g.ndim; ++d) {
    if (v) {
      if (!v[d]) return fail(c, FLD_ERR_INVALID_ARG, "NULL velocity component");
      a.v[d] = v[d];
    }
    if (f_r) a.fr[d] = f_r[d];
  }
  a.work = work;
  a.tiring = tiring;
  a.fedd = fedd;
  HIP_TRY(c, launch_explicit(a, c->stream));
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

}  // extern "C"

namespace {

// Time every tile shape of the down and up passes on each tiled level of c
// (zeroed level buffers of the context: the kernels' speed does not depend
// on the values) and keep the fastest.  choice[l][0 / 1]: down / up.
template <typename T>
fld_status tune_levels(fld_ctx* c, Levels<T>& H, int choice[kMaxLevels][2],
                       int nvar) {
  hipStream_t s = c->stream;
  // Level-0 buffers: the FP32 iterate and rhs of a mixed context belong to
  // the workspace; the FP64 ones are the caller's arrays during a step (the
  // pointers of the last step are stale here), so the rhs copy stands in
  // for both.
  const bool own0 = sizeof(T) == sizeof(float);
  T* x0 = own0 ? H.x[0] : (T*)c->bcopy;
  T* b0 = own0 ? H.b[0] : (T*)c->bcopy;
  FLD_TRY(fill_zero<T>(c, (T*)c->bcopy, c->geom[0].N * (int64_t)sizeof(double) /
                                            (int64_t)sizeof(T)));
  for (int l = 0; l <= c->tail_l0 && l < c->L; ++l) {
    if (l > 0 || own0) {
      FLD_TRY(fill_zero<T>(c, H.x[l], c->geom[l].N));
      FLD_TRY(fill_zero<T>(c, H.b[l], c->geom[l].N));
    }
    for (int d = 0; d < 2; ++d) FLD_TRY(fill_zero<T>(c, H.a[l][d], c->geom[l].N));
  }
  HIP_TRY(c, launch_ctrl_init(c->ctrl, c->p.rtol, c->p.max_cycles, c->inner,
                             nullptr, s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, FLD_ERR_DEVICE, "hipEventCreate failed");
  }
  fld_status st = FLD_OK;
  constexpr int kReps = 6;
  for (int l = 0; l < c->tail_l0 && st == FLD_OK; ++l)
    for (int dir = 0; dir < 2 && st == FLD_OK; ++dir) {
      Tile2DArgs<T> a{};
      a.g = c->geom[l];
      a.spec = l == 0 && dir == 0;
      T* xl = l == 0 ? x0 : H.x[l];
      a.x = dir == 0 ? xl : H.alt[l];
      a.xo = dir == 0 ? H.alt[l] : xl;
      a.b = l == 0 ? b0 : H.b[l];
      a.ax = H.a[l][0];
      a.ay = H.a[l][1];
      a.gc = c->geom[l + 1];
      a.cb = dir == 0 ? H.b[l + 1] : nullptr;
      a.ce = dir == 0 ? nullptr : H.x[l + 1];
      a.partials = (dir == 0 && l == 0) ? c->partials : nullptr;
      a.zero_init = 0;
      a.ctrl = c->ctrl;
      const int nu = dir == 0 ? nu_pre(c->p, l) : nu_post(c->p, l);
      // best of 3 rounds per shape; shapes are tried from 32x32/256 (the
      // usual winner) and another replaces the current choice only when it
      // is more than 5% faster, so that timing noise (or a profiler's
      // per-dispatch overhead) rarely changes the pick between runs
      float best = 1e30f;
      for (int k = 0; k < nvar && st == FLD_OK; ++k) {
        const int v = kTilePreferred < nvar ? (k + kTilePreferred) % nvar : k;
        float vbest = 1e30f;
        for (int round = 0; round < 3 && st == FLD_OK; ++round) {
          int nb = 0;
          hipError_t e = launch_tile2d<T>(a, nu, dir == 0, v, s, &nb);  // warm-up
          if (e == hipSuccess) e = hipEventRecord(e0, s);
          for (int r = 0; r < kReps && e == hipSuccess; ++r)
            e = launch_tile2d<T>(a, nu, dir == 0, v, s, &nb);
          if (e == hipSuccess) e = hipEventRecord(e1, s);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (e != hipSuccess) {
            st = fail(c, FLD_ERR_DEVICE, "autotune: %s", hipGetErrorString(e));
            break;
          }
          vbest = ms < vbest ? ms : vbest;
        }
        if (vbest < 0.95f * best) {
          best = vbest;
          choice[l][dir] = v;
        }
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

fld_status tune_ctx(fld_ctx* c, int choice[kMaxLevels][2], int nvar) {
  for (int l = 0; l < kMaxLevels; ++l) choice[l][0] = choice[l][1] = 0;
  if (!tile_path(c)) return FLD_OK;
  return c->mixed ? tune_levels<float>(c, c->h32, choice, nvar)
                  : tune_levels<double>(c, c->h64, choice, nvar);
}

}  // namespace

extern "C" {

fld_status fld_autotune(fld_ctx* c, int32_t* choices, int32_t max_levels) {
  if (!c) return fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (choices && max_levels < 0)
    return fail(c, FLD_ERR_INVALID_ARG, "max_levels must be >= 0");
  int choice[kMaxLevels][2];
  if (c->batch) {
    // tune on the largest grid; one shape per level index for all grids
    BatchState* B = c->batch;
    fld_ctx* big = B->sub[0];
    for (fld_ctx* sub : B->sub)
      if (sub->geom[0].N > big->geom[0].N) big = sub;
    const fld_status st = tune_ctx(big, choice, kTileVariantsBatch);
    if (st != FLD_OK) return fail(c, st, "%s", big->err.c_str());
    for (int l = 0; l < kMaxLevels; ++l)
      for (int d = 0; d < 2; ++d) B->tile_var[l][d] = choice[l][d];
    // the captured graph holds the old launch shapes
    if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->gexec = nullptr;
    B->graph = nullptr;
    B->last.clear();
  } else {
    FLD_TRY(tune_ctx(c, choice, kTileVariants));
    for (int l = 0; l < kMaxLevels; ++l)
      for (int d = 0; d < 2; ++d) c->tile_var[l][d] = choice[l][d];
  }
  if (choices)
    for (int l = 0; l < max_levels && l < kMaxLevels; ++l) {
      choices[2 * l] = choice[l][0];
      choices[2 * l + 1] = choice[l][1];
    }
  return FLD_OK;
}

const char* fld_tile_shape_name(int32_t variant) {
  return (variant >= 0 && variant < kTileVariants) ? tile2d_variant_name(variant)
                                                   : "invalid";
}

fld_status fld_set_model(fld_ctx* c, const float* host, size_t count) {
  if (!c) return fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (!host) return fail(c, FLD_ERR_INVALID_ARG, "weights pointer is NULL");
  if (c->p.guess != FLD_GUESS_LEARNED || !c->net_ws)
    return fail(c, FLD_ERR_INVALID_ARG,
                "the context was not set up with FLD_GUESS_LEARNED");
  if (count != nn::param_count())
    return fail(c, FLD_ERR_MODEL, "%zu parameters given, the network has %zu",
                count, nn::param_count());
  if (!c->net) {
    std::string err;
    const Geom& g = c->geom[0];
    c->net = nn::create(g.n[2], g.n[1], g.n[0], 0, c->net_ws, c->net_bytes,
                        c->stream, &err);
    if (!c->net) return fail(c, FLD_ERR_DEVICE, "%s", err.c_str());
  }
  if (!nn::set_params(c->net, host, count))
    return fail(c, FLD_ERR_MODEL, "non-finite parameter or device error");
  // a new network is tried at the next step once a reference step exists
  c->net_span = 0;
  if (c->plain_units >= 0) c->net_skip = 0;
  return FLD_OK;
}

fld_status fld_features(fld_ctx* c, double dt, const double* rho,
                        const double* kappa, const double* E, float* out) {
  if (!c) return fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (c->batch) return fail(c, FLD_ERR_INVALID_ARG, "batched context");
  if (c->p.ndim < 2) return fail(c, FLD_ERR_INVALID_ARG, "needs ndim >= 2");
  if (c->p.n[2] > 65535)
    return fail(c, FLD_ERR_INVALID_ARG, "at most 65535 z-slices");
  if (!rho || !kappa || !E || !out)
    return fail(c, FLD_ERR_INVALID_ARG, "NULL field pointer");
  if (!(dt > 0.0) || !std::isfinite(dt))
    return fail(c, FLD_ERR_INVALID_ARG, "dt must be positive and finite");
  const Geom& g0 = c->geom[0];
  HIP_TRY(c, launch_ctrl_init(c->ctrl, c->p.rtol, c->p.max_cycles, c->inner,
                             nullptr, c->stream));
  CoefArgs A;
  A.g = g0;
  for (int d = 0; d < 3; ++d) {
    A.dx[d] = c->p.dx[d];
    A.gscale[d] = 1.0 / (12.0 * c->p.dx[d]);
  }
  A.dt = dt;
  A.c = c->p.c;
  A.limiter = c->p.limiter;
  A.face_mean = c->p.face_mean;
  HIP_TRY(c, launch_coef(A, E, rho, kappa, c->h64.a[0], c->h32.a[0], nullptr,
                         c->partials, c->ctrl, c->stream));
  const int64_t slice = (int64_t)g0.n[0] * g0.n[1];
  HIP_TRY(c, nn::launch_mean_log(E, slice, g0.n[2], c->mean,
                                     c->mean + g0.n[2], c->stream));
  HIP_TRY(c, nn::launch_features(E, rho, kappa, c->h64.a[0][0], c->h64.a[0][1],
                                 c->p.dx[0], c->mean, g0.N, slice, nullptr, out,
                                 c->stream));
  return FLD_OK;
}

void fld_destroy(fld_ctx* c) {
  if (!c) return;
  if (c->net) {
    nn::destroy(c->net);
    c->net = nullptr;
  }
  if (c->batch) {
    BatchState* B = c->batch;
    for (fld_ctx* s : B->sub) fld_destroy(s);
    if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    if (B->host_tab) (void)hipHostFree(B->host_tab);
    if (B->host_aux) (void)hipHostFree(B->host_aux);
    delete B;
    c->batch = nullptr;
  }
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->net_ev)
    if (e) (void)hipEventDestroy(e);
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

// ---- batched entry points --------------------------------------------------

static std::string validate_batch(int32_t count, const fld_params* each) {
  if (count < 1) return "count must be >= 1";
  if (!each) return "params array is NULL";
  for (int g = 0; g < count; ++g) {
    std::string why = validate(&each[g]);
    if (!why.empty()) return "grid " + std::to_string(g) + ": " + why;
    const fld_params& p = each[g];
    if (p.ndim != 2) return "batched grids must be 2D";
    if (p.precision != each[0].precision)
      return "batched grids must share the precision";
    if (p.pre_smooth < 1 || p.pre_smooth > 3 || p.post_smooth < 1 ||
        p.post_smooth > 3 || p.pre_smooth != each[0].pre_smooth ||
        p.post_smooth != each[0].post_smooth || nu_pre(p, 1) > 3 ||
        nu_post(p, 1) > 3 || nu_pre(p, 1) != nu_pre(each[0], 1) ||
        nu_post(p, 1) != nu_post(each[0], 1))
      return "batched grids need equal pre/post smoothing in 1..3";
    if (p.guess != FLD_GUESS_PREV) return "batched grids use guess E^n";
    if (has_dirichlet(p)) return "batched grids take periodic or Neumann walls";
    if (p.held_cells) return "batched grids have no held cells";
    if (p.krylov) return "batched grids iterate V-cycles (krylov = 0)";
    if (p.ir_inner != each[0].ir_inner)
      return "batched grids must share ir_inner";
    Plan P;
    make_plan(&p, &P);
    int l0 = P.L - 1;
    for (int l = 0; l < P.L; ++l)
      if (P.g[l].N <= kTailLdsCells) {
        l0 = l;
        break;
      }
    if (l0 == 0 || P.g[l0].N > kTailLdsCells || P.L - l0 > 10)
      return "grid " + std::to_string(g) +
             ": too small (<= 1024 cells) or not coarsenable to 1024 cells";
  }
  return "";
}

static size_t batch_sub_bytes(int32_t count, const fld_params* each,
                              std::vector<size_t>* offs) {
  size_t o = 0;
  for (int g = 0; g < count; ++g) {
    Plan P;
    make_plan(&each[g], &P);
    if (offs) offs->push_back(o);
    o = align_up(o + P.total);
  }
  return o;
}

static size_t batch_aux_bytes(int32_t count) {
  return 2 * (align_up(sizeof(JobOpacity) * count) +
              align_up(sizeof(int) * (count + 1))) + 4 * kAlign;
}

extern "C" {

size_t fld_workspace_bytes_batch(int32_t count, const fld_params* each) {
  if (!validate_batch(count, each).empty()) return 0;
  // table image size: build one with the real level structure
  std::vector<size_t> offs;
  const size_t subs = batch_sub_bytes(count, each, &offs);
  fld_ctx tmp_batch;
  BatchState B;
  tmp_batch.batch = &B;
  B.ng = count;
  std::vector<fld_ctx> subs_ctx(count);
  char* fake = (char*)kAlign;  // layout only: no memory is touched
  for (int g = 0; g < count; ++g) {
    Plan P;
    make_plan(&each[g], &P);
    fld_ctx* c = &subs_ctx[g];
    c->p = each[g];
    c->L = P.L;
    c->mixed = each[g].precision == FLD_PREC_FP32_IR;
    for (int l = 0; l < P.L; ++l) c->geom[l] = P.g[l];
    c->tail_l0 = P.L - 1;
    for (int l = 0; l < P.L; ++l)
      if (P.g[l].N <= kTailLdsCells) {
        c->tail_l0 = l;
        break;
      }
    B.sub.push_back(c);
    B.maxL = std::max(B.maxL, c->L);
    B.maxl0 = std::max(B.maxl0, c->tail_l0);
  }
  std::vector<const double*> pc(count, (const double*)fake);
  std::vector<double*> pm(count, (double*)fake);
  std::vector<double> dts(count, 1.0);
  Image im;
  if (each[0].precision == FLD_PREC_FP32_IR)
    build_image<float>(&tmp_batch, im, dts.data(), pc.data(), pc.data(),
                       pc.data(), pm.data());
  else
    build_image<double>(&tmp_batch, im, dts.data(), pc.data(), pc.data(),
                        pc.data(), pm.data());
  tmp_batch.batch = nullptr;
  return subs + align_up(im.buf.size() + kAlign) + batch_aux_bytes(count);
}

fld_status fld_setup_batch(int32_t count, const fld_params* each,
                           void* workspace, size_t ws_bytes, void* hip_stream,
                           fld_ctx** out) {
  if (!out) return fail(nullptr, FLD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  std::string why = validate_batch(count, each);
  if (!why.empty()) return fail(nullptr, FLD_ERR_INVALID_ARG, "%s", why.c_str());
  const size_t need = fld_workspace_bytes_batch(count, each);
  if (!workspace) return fail(nullptr, FLD_ERR_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)workspace % kAlign)
    return fail(nullptr, FLD_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < need)
    return fail(nullptr, FLD_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu",
                ws_bytes, need);
  std::vector<size_t> offs;
  const size_t subs = batch_sub_bytes(count, each, &offs);
  fld_ctx* bc = new fld_ctx();
  bc->p = each[0];
  bc->stream = (hipStream_t)hip_stream;
  bc->ws = (char*)workspace;
  bc->ws_bytes = ws_bytes;
  BatchState* B = new BatchState();
  bc->batch = B;
  B->ng = count;
  if (const char* tv = getenv("FLD_TILE_VARIANT")) {  // as in fld_setup
    const int v = atoi(tv);
    if (v >= 0 && v < kTileVariantsBatch)
      for (int l = 0; l < kMaxLevels; ++l) B->tile_var[l][0] = B->tile_var[l][1] = v;
  }
  for (int g = 0; g < count; ++g) {
    Plan P;
    make_plan(&each[g], &P);
    fld_ctx* c = nullptr;
    fld_status st = fld_setup(&each[g], bc->ws + offs[g], P.total, hip_stream, &c);
    if (st != FLD_OK) {
      std::string msg = g_err;
      fld_destroy(bc);
      return fail(nullptr, st, "grid %d: %s", g, msg.c_str());
    }
    // the batched tails start at the first level of at most 1024 cells
    c->tail_big = false;
    choose_tail(c);
    B->sub.push_back(c);
    B->maxL = std::max(B->maxL, c->L);
    B->maxl0 = std::max(B->maxl0, c->tail_l0);
  }
  B->aux_cap = batch_aux_bytes(count);
  B->tab_cap = need - subs - B->aux_cap;
  B->dev_tab = bc->ws + subs;
  B->dev_aux = B->dev_tab + B->tab_cap;
  hipError_t he = hipHostMalloc((void**)&B->host_tab, B->tab_cap, hipHostMallocDefault);
  if (he == hipSuccess)
    he = hipHostMalloc((void**)&B->host_aux, B->aux_cap, hipHostMallocDefault);
  if (he != hipSuccess) {
    fld_destroy(bc);
    return fail(nullptr, FLD_ERR_DEVICE, "hipHostMalloc of the batch tables: %s",
                hipGetErrorString(he));
  }
  *out = bc;
  return FLD_OK;
}

fld_status fld_step_batch(fld_ctx* bc, const double* dt,
                          const double* const* rho, const double* const* kappa,
                          const double* const* E_in, double* const* E_out,
                          fld_stats* stats) {
  if (!bc || !bc->batch)
    return fail(bc, FLD_ERR_INVALID_ARG, "not a batched context");
  BatchState* B = bc->batch;
  if (!dt || !rho || !kappa || !E_in || !E_out)
    return fail(bc, FLD_ERR_INVALID_ARG, "NULL array");
  for (int g = 0; g < B->ng; ++g) {
    if (!(dt[g] > 0.0) || !std::isfinite(dt[g]))
      return fail(bc, FLD_ERR_INVALID_ARG, "grid %d: dt must be positive", g);
    if (!rho[g] || !kappa[g] || !E_in[g] || !E_out[g])
      return fail(bc, FLD_ERR_INVALID_ARG, "grid %d: NULL field pointer", g);
  }
  if (B->sub[0]->mixed)
    FLD_TRY((batch_step_impl<float>(bc, dt, rho, kappa, E_in, E_out)));
  else
    FLD_TRY((batch_step_impl<double>(bc, dt, rho, kappa, E_in, E_out)));
  fld_status worst = FLD_OK;
  int worst_g = -1;
  for (int g = 0; g < B->ng; ++g) {
    const Control& h = *B->sub[g]->host_ctrl;
    if (stats) {
      memset(&stats[g], 0, sizeof(fld_stats));
      stats[g].cycles = h.cycles;
      stats[g].outer_iters = B->sub[g]->mixed ? h.outer : 0;
      stats[g].flagged_cells = h.flagged;
      stats[g].rel_res_initial = h.res_initial;
      stats[g].rel_res_final = h.res;
    }
    fld_status st = h.done == kConverged     ? FLD_OK
                    : h.done == kNonPhysical ? FLD_ERR_NONPHYSICAL
                                             : FLD_ERR_NOT_CONVERGED;
    if (st != FLD_OK && (worst == FLD_OK || st == FLD_ERR_NONPHYSICAL)) {
      worst = st;
      worst_g = g;
    }
  }
  if (worst != FLD_OK)
    return fail(bc, worst, "grid %d: %s", worst_g,
                worst == FLD_ERR_NONPHYSICAL ? "non-physical input"
                                             : "not converged");
  return FLD_OK;
}

}  // extern "C"

// Tables of the pointwise batched calls: staged and uploaded per call
// (after the previous use of the staging buffer has finished).
template <typename X>
static fld_status aux_upload(fld_ctx* bc, const std::vector<X>& jobs,
                             const std::vector<int>& blocks, Phase* ph) {
  BatchState* B = bc->batch;
  Image im;
  add_phase(im, *ph, jobs, blocks);
  if (im.buf.size() > B->aux_cap)
    return fail(bc, FLD_ERR_WORKSPACE, "aux table too large");
  HIP_TRY(bc, hipStreamSynchronize(bc->stream));
  memcpy(B->host_aux, im.buf.data(), im.buf.size());
  HIP_TRY(bc, hipMemcpyAsync(B->dev_aux, B->host_aux, im.buf.size(),
                             hipMemcpyHostToDevice, bc->stream));
  return FLD_OK;
}

extern "C" {

fld_status fld_exchange_batch(fld_ctx* bc, const double* dt,
                              const double* const* rho,
                              const double* const* kappa, double* const* E,
                              double* const* e_int) {
  if (!bc || !bc->batch)
    return fail(bc, FLD_ERR_INVALID_ARG, "not a batched context");
  BatchState* B = bc->batch;
  if (!dt || !rho || !kappa || !E || !e_int)
    return fail(bc, FLD_ERR_INVALID_ARG, "NULL array");
  std::vector<JobExchange> jobs(B->ng);
  std::vector<int> blocks(B->ng);
  for (int g = 0; g < B->ng; ++g) {
    if (!(dt[g] > 0.0) || !std::isfinite(dt[g]))
      return fail(bc, FLD_ERR_INVALID_ARG, "grid %d: dt must be positive", g);
    if (!rho[g] || !kappa[g] || !E[g] || !e_int[g])
      return fail(bc, FLD_ERR_INVALID_ARG, "grid %d: NULL field pointer", g);
    const fld_params& p = B->sub[g]->p;
    jobs[g] = {B->sub[g]->geom[0].N, dt[g], p.c, p.a_rad, p.gamma - 1.0,
               p.gas_const, rho[g], kappa[g], E[g], e_int[g]};
    blocks[g] = blocks_for(B->sub[g]->geom[0].N);
  }
  Phase ph;
  FLD_TRY(aux_upload(bc, jobs, blocks, &ph));
  HIP_TRY(bc, launch_exchange_batch((const JobExchange*)(B->dev_aux + ph.tab),
                                    (const int*)(B->dev_aux + ph.start), ph.ng,
                                    ph.nblocks, bc->stream));
  return FLD_OK;
}

fld_status fld_opacity_powerlaw_batch(fld_ctx* bc, const double* const* rho,
                                      const double* const* e_int, double k0,
                                      double a, double b, double kmin,
                                      double kmax, double* const* kappa) {
  if (!bc || !bc->batch)
    return fail(bc, FLD_ERR_INVALID_ARG, "not a batched context");
  BatchState* B = bc->batch;
  if (!rho || !e_int || !kappa) return fail(bc, FLD_ERR_INVALID_ARG, "NULL array");
  if (!(k0 > 0.0) || !(kmin > 0.0) || !(kmax >= kmin) || !std::isfinite(a) ||
      !std::isfinite(b) || !std::isfinite(kmax))
    return fail(bc, FLD_ERR_INVALID_ARG,
                "need k0 > 0, 0 < kmin <= kmax, finite exponents");
  int ha = INT_MIN, hb = INT_MIN;
  if (2.0 * a == std::floor(2.0 * a) && 2.0 * b == std::floor(2.0 * b) &&
      std::fabs(a) <= 16.0 && std::fabs(b) <= 16.0) {
    ha = (int)(2.0 * a);
    hb = (int)(2.0 * b);
  }
  std::vector<JobOpacity> jobs(B->ng);
  std::vector<int> blocks(B->ng);
  for (int g = 0; g < B->ng; ++g) {
    if (!rho[g] || !e_int[g] || !kappa[g])
      return fail(bc, FLD_ERR_INVALID_ARG, "grid %d: NULL field pointer", g);
    const fld_params& p = B->sub[g]->p;
    jobs[g] = {B->sub[g]->geom[0].N, p.gamma - 1.0, p.gas_const, rho[g],
               e_int[g], k0, a, b, ha, hb, kmin, kmax, kappa[g]};
    blocks[g] = blocks_for(B->sub[g]->geom[0].N);
  }
  Phase ph;
  FLD_TRY(aux_upload(bc, jobs, blocks, &ph));
  HIP_TRY(bc, launch_opacity_batch((const JobOpacity*)(B->dev_aux + ph.tab),
                                   (const int*)(B->dev_aux + ph.start), ph.ng,
                                   ph.nblocks, bc->stream));
  return FLD_OK;
}

fld_status fld_batch_set_graph(fld_ctx* bc, int32_t on) {
  if (!bc || !bc->batch)
    return fail(bc, FLD_ERR_INVALID_ARG, "not a batched context");
  if (on && bc->stream == nullptr)
    return fail(bc, FLD_ERR_INVALID_ARG,
                "graph capture needs a non-default stream (fld_setup_batch "
                "was given the null stream)");
  bc->batch->graph_on = on != 0;
  return FLD_OK;
}

}  // extern "C"
