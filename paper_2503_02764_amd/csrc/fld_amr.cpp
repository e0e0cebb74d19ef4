// Block-adaptive 2D step (include/fld.h, fld_amr_*): a base grid and up
// to four levels of nested refined blocks, the backward-Euler diffusion of
// eq. mhd_r_e on the leaf cells (Sect. 3 solves it by multigrid on
// MPI-AMRVAC's block-adaptive grids).
//
// The composite operator (fld_amr.hip) is symmetric in the volume-weighted
// inner product, so the solve is conjugate gradients in that product,
// flexible (one previous direction) because its preconditioner is a
// multigrid cycle over the levels:
//   1. down, from the finest level: red-black Gauss-Seidel sweeps over
//      every cell of the level (those under finer blocks included) for the
//      level's own correction problem, whose right-hand side is r on leaf
//      cells and the restricted residual of the finer level under finer
//      blocks; then the level's residual restricted to the next coarser
//      level, whose leaf cells next to this level also take the flux of
//      its correction;
//   2. one V-cycle of the base grid's own multigrid (a single-grid context,
//      its faces from the base view of E) for the base correction;
//   3. up, from level 1: each level's correction += the coarser one
//      prolonged (bilinear), then the sweeps again in reverse colour order;
//   4. each leaf cell takes its level's correction.
// The stop test is the volume-weighted relative residual |r|_V / |b|_V.
// The scalars of an iteration stay on the device: the operator and update
// kernels leave block sums, one-block reductions turn them into the
// scalars the next kernels read, and the host reads (r, r) once an
// iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fld.h"
#include "fld_amr.h"
#include "fld_hooks.h"
#include "fld_internal.h"

using namespace fld;

struct fld_amr_ctx {
  AmrGeom G{};
  AmrPhys P{};
  fld_params p{};
  fld_ctx* base = nullptr;
  hipStream_t stream = nullptr;
  double *Ev = nullptr, *rv = nullptr, *kv = nullptr;
  double *Evf = nullptr, *rvf = nullptr, *kvf = nullptr;  // fine views
  double* t = nullptr;  // preconditioner: level residuals
  double* g = nullptr;  // preconditioner: right-hand sides per level
  double *Db = nullptr, *Df = nullptr, *cf = nullptr, *rhs = nullptr;
  double *x = nullptr, *b = nullptr, *r = nullptr, *z = nullptr;
  double *p2[2] = {}, *q2[2] = {};
  double* partials = nullptr;
  double* sc = nullptr;  // Krylov scalars on the device (amr_reduce)
  int* bad = nullptr;
  std::vector<double> host_part;
  std::string err;
  // kernel timing: every level-1 half-sweep of a step, each between a pair
  // of events from this pool (ev_used pairs taken in the current step)
  bool timing = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  double t_ms = 0.0, t_bytes = 0.0;
  int64_t t_launches = 0;
};

namespace {

thread_local std::string g_amr_err;

fld_status amr_fail(fld_amr_ctx* c, fld_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  g_amr_err = buf;
  return st;
}

#define AMR_HIP(c, expr)                                                    \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return amr_fail(c, FLD_ERR_DEVICE, "%s: %s", #expr,                  \
                      hipGetErrorString(e_));                               \
  } while (0)

#define AMR_TRY(expr)              \
  do {                             \
    fld_status s_ = (expr);        \
    if (s_ != FLD_OK) return s_;   \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// The base grid's own context: FP64 V-cycles, zero guess (it only ever
// runs as the preconditioner's base solve).
fld_params base_params(const fld_params& p) {
  fld_params q = p;
  q.guess = FLD_GUESS_ZERO;
  q.precision = FLD_PREC_FP64;
  q.krylov = 0;
  q.held_cells = 0;
  return q;
}

// Levels: nlevels entries of nblocks; blocks_xy holds the (bx, by) of
// level 1's blocks, then level 2's, ...  A level-l block refines the b x b
// patch of level-(l-1) cells with corner (bx b, by b).
std::string validate_amr(const fld_params* p, int32_t block, int32_t nlevels,
                         const int32_t* nblocks, const int32_t* blocks_xy) {
  if (!p) return "params is NULL";
  if (p->ndim != 2) return "the block-adaptive step is 2D (ndim = 2)";
  if (p->precision != FLD_PREC_FP64) return "precision must be FP64";
  if (p->guess != FLD_GUESS_PREV && p->guess != FLD_GUESS_ZERO)
    return "guess must be E^n or zero";
  if (p->krylov) return "krylov must be 0 (the step is a Krylov solve)";
  if (p->held_cells) return "no held cells on a block-adaptive grid";
  for (int d = 0; d < 2; ++d)
    if (p->bc_lo[d] == FLD_BC_DIRICHLET || p->bc_hi[d] == FLD_BC_DIRICHLET)
      return "walls must be periodic or zero-gradient";
  if (block < 2) return "block must be >= 2 base cells";
  if (p->n[0] < 4 || p->n[1] < 4) return "the base grid needs >= 4 x 4 cells";
  if (p->n[0] % block || p->n[1] % block)
    return "the base grid's sides must be multiples of block";
  if (nlevels < 0 || nlevels > kAmrMaxLevels) return "nlevels must be in [0, 4]";
  if (nlevels > 0 && !nblocks) return "nblocks is NULL";
  int64_t total = 0;
  for (int l = 0; l < nlevels; ++l) {
    if (nblocks[l] < 0) return "nblocks must be >= 0";
    if (l > 0 && nblocks[l] > 0 && nblocks[l - 1] == 0)
      return "a level follows an empty one";
    total += nblocks[l];
  }
  if (total > 0 && !blocks_xy) return "blocks_xy is NULL";
  const bool per[2] = {p->bc_lo[0] == FLD_BC_PERIODIC,
                       p->bc_lo[1] == FLD_BC_PERIODIC};
  // units (b cells) of each level's lattice, and which hold a block
  std::vector<std::vector<char>> has(nlevels + 1);
  const int32_t* xy = blocks_xy;
  for (int l = 1; l <= nlevels; ++l) {
    const int64_t ux = (p->n[0] << (l - 1)) / block;
    const int64_t uy = (p->n[1] << (l - 1)) / block;
    has[l].assign((size_t)(ux * uy), 0);
    for (int32_t k = 0; k < nblocks[l - 1]; ++k, xy += 2) {
      const int32_t bx = xy[0], by = xy[1];
      if (bx < 0 || by < 0 || bx >= ux || by >= uy)
        return "a refined block lies outside its level's lattice";
      char& sl = has[l][(size_t)(by * ux + bx)];
      if (sl) return "a block is listed twice";
      sl = 1;
      if (l == 1) continue;
      // nested: inside a level-(l-1) block (whose corner unit is (bx/2,
      // by/2) of level l-2); 2:1: so are the four face-adjacent patches
      const int64_t pux = (p->n[0] << (l - 2)) / block;
      auto inside = [&](int64_t x, int64_t y) {
        if (x < 0 || x >= ux) {
          if (!per[0]) return true;  // a wall
          x = (x + ux) % ux;
        }
        if (y < 0 || y >= uy) {
          if (!per[1]) return true;
          y = (y + uy) % uy;
        }
        return has[l - 1][(size_t)((y / 2) * pux + x / 2)] != 0;
      };
      if (!inside(bx, by)) return "a block lies outside the coarser level";
      if (!inside(bx - 1, by) || !inside(bx + 1, by) || !inside(bx, by - 1) ||
          !inside(bx, by + 1))
        return "levels not 2:1 nested: a block's face neighbour is two "
               "levels coarser";
    }
  }
  return "";
}

struct AmrPlan {
  size_t base_ws = 0, bmap[kAmrMaxLevels] = {}, bxy[kAmrMaxLevels] = {};
  size_t views = 0, fviews = 0, Db = 0, Df = 0, cf = 0;
  size_t rhs = 0, vec = 0, partials = 0, sc = 0, bad = 0, total = 0;
  int64_t Nb = 0, Nf = 0, nvec = 0;
  int dot_blocks = 0;
};

AmrPlan make_amr_plan(const fld_params& p, int32_t block, int32_t nlevels,
                      const int32_t* nblocks) {
  AmrPlan P;
  P.Nb = p.n[0] * p.n[1];
  for (int l = 0; l < nlevels; ++l)
    P.Nf += (int64_t)nblocks[l] * 4 * block * block;
  P.nvec = P.Nb + P.Nf;
  P.dot_blocks = (int)((P.nvec + 255) / 256);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return r;
  };
  const fld_params bp = base_params(p);
  P.base_ws = take(fld_workspace_bytes(&bp));
  for (int l = 1; l <= nlevels; ++l) {
    const int64_t units = ((p.n[0] << (l - 1)) / block) *
                          ((p.n[1] << (l - 1)) / block);
    P.bmap[l - 1] = take((size_t)units * 4);
    P.bxy[l - 1] = take((size_t)nblocks[l - 1] * 8);
  }
  P.views = take((size_t)P.Nb * 8 * 3);
  P.fviews = take((size_t)P.Nf * 8 * 3);
  P.Db = take((size_t)P.Nb * 8);
  P.Df = take((size_t)P.Nf * 8);
  P.cf = take((size_t)P.Nf * 8 * 4);
  P.rhs = take((size_t)P.Nb * 8);
  P.vec = take((size_t)P.nvec * 8 * 10);  // x, b, r, z, p[2], q[2], t, g
  P.partials = take((size_t)P.dot_blocks * 3 * 8);
  P.sc = take(8 * 8);
  P.bad = take(8);
  P.total = o;
  return P;
}

fld_status dots(fld_amr_ctx* c, int n, const double* u0, const double* v0,
                const double* u1, const double* v1, double out[2]) {
  AmrDots D{};
  D.n = n;
  D.u[0] = u0;
  D.v[0] = v0;
  D.u[1] = u1;
  D.v[1] = v1;
  const int nb = amr_dot_blocks(c->G);
  AMR_HIP(c, amr_dots(c->G, D, c->partials, c->stream));
  c->host_part.resize((size_t)nb * n);
  AMR_HIP(c, hipMemcpyAsync(c->host_part.data(), c->partials,
                            sizeof(double) * nb * n, hipMemcpyDeviceToHost,
                            c->stream));
  AMR_HIP(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < n; ++k) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += c->host_part[(size_t)k * nb + i];
    out[k] = s;
  }
  return FLD_OK;
}

// the next pair of timing events of this step (created on first use)
fld_status timing_pair(fld_amr_ctx* c, hipEvent_t* e0, hipEvent_t* e1) {
  while (c->ev.size() < 2 * (c->ev_used + 1)) {
    hipEvent_t e = nullptr;
    AMR_HIP(c, hipEventCreate(&e));
    c->ev.push_back(e);
  }
  *e0 = c->ev[2 * c->ev_used];
  *e1 = c->ev[2 * c->ev_used + 1];
  ++c->ev_used;
  return FLD_OK;
}

// z = M r (the cycle of the file comment); z holds each level's correction
// e on every cell of the level (cells under finer blocks included) until
// the end, where those cells are zeroed
fld_status precondition(fld_amr_ctx* c, const double* r, double* z) {
  const AmrGeom& G = c->G;
  hipStream_t s = c->stream;
  const int64_t n = G.Nb + G.Nf;
  AMR_HIP(c, hipMemsetAsync(z, 0, sizeof(double) * n, s));
  AMR_HIP(c, hipMemcpyAsync(c->g, r, sizeof(double) * n,
                            hipMemcpyDeviceToDevice, s));
  const int pre = std::max(c->p.pre_smooth, 1);
  const int post = std::max(c->p.post_smooth, 1);
  for (int l = G.L; l >= 1; --l) {  // down: the finest level first
    for (int k = 0; k < pre; ++k)
      for (int colour = 0; colour < 2; ++colour) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing && l == 1) AMR_TRY(timing_pair(c, &e0, &e1));
        AMR_HIP(c, amr_smooth_level(G, l, c->cf, c->g, z, colour, s, e0, e1));
      }
    AMR_HIP(c, amr_resid_level(G, l, c->cf, c->g, z, c->t, s));
    AMR_HIP(c, amr_coarse_rhs(G, l - 1, c->cf, z, c->t, c->g, s));
  }
  const fld_status st = precond_vcycle(c->base, c->g, z);
  if (st != FLD_OK)
    return amr_fail(c, st, "base V-cycle: %s", ctx_error(c->base));
  for (int l = 1; l <= G.L; ++l) {  // up: prolong, then sweep again
    AMR_HIP(c, amr_prolong_level(G, l, z, s));
    for (int k = 0; k < post; ++k)
      for (int colour = 1; colour >= 0; --colour) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing && l == 1) AMR_TRY(timing_pair(c, &e0, &e1));
        AMR_HIP(c, amr_smooth_level(G, l, c->cf, c->g, z, colour, s, e0, e1));
      }
  }
  AMR_HIP(c, amr_zero_covered(G, z, s));
  return FLD_OK;
}

fld_status amr_solve(fld_amr_ctx* c, double dt, const double* rho_b,
                     const double* kap_b, const double* E_b,
                     double* E_b_out, const double* rho_f,
                     const double* kap_f, const double* E_f,
                     double* E_f_out, fld_stats* stats) {
  const AmrGeom& G = c->G;
  hipStream_t s = c->stream;
  const int64_t n = G.Nb + G.Nf;
  c->ev_used = 0;
  // coefficients: views, D on both levels, fine faces, base faces
  AMR_HIP(c, amr_views(G, E_b, rho_b, kap_b, E_f, rho_f, kap_f, c->Ev, c->rv,
                       c->kv, c->Evf, c->rvf, c->kvf, s));
  AMR_HIP(c, hipMemsetAsync(c->bad, 0, sizeof(int), s));
  AMR_HIP(c, amr_coefficients(G, c->P, dt, c->Ev, c->rv, c->kv, c->Evf,
                              c->rvf, c->kvf, c->Db, c->Df, c->cf, c->bad, s));
  int bad = 0;
  AMR_HIP(c, hipMemcpyAsync(&bad, c->bad, sizeof(int), hipMemcpyDeviceToHost,
                            s));
  AMR_HIP(c, hipStreamSynchronize(s));
  if (stats) stats->flagged_cells = bad;
  if (bad > 0)
    return amr_fail(c, FLD_ERR_NONPHYSICAL,
                    "%d cells with E <= 0, rho kappa <= 0 or non-finite", bad);
  fld_status st = precond_begin(c->base, dt, c->Ev, c->rv, c->kv);
  if (st != FLD_OK) return amr_fail(c, st, "base grid: %s", ctx_error(c->base));
  const double* ax = nullptr;
  const double* ay = nullptr;
  base_faces(c->base, &ax, &ay);
  // b = E^n on the leaf cells, x0 = E^n or 0, r = b - A x0
  AMR_HIP(c, amr_pack(G, E_b, E_f, c->b, s));
  if (c->p.guess == FLD_GUESS_ZERO) {
    AMR_HIP(c, hipMemsetAsync(c->x, 0, sizeof(double) * n, s));
    AMR_HIP(c, hipMemcpyAsync(c->r, c->b, sizeof(double) * n,
                              hipMemcpyDeviceToDevice, s));
  } else {
    AMR_HIP(c, hipMemcpyAsync(c->x, c->b, sizeof(double) * n,
                              hipMemcpyDeviceToDevice, s));
    AMR_HIP(c, amr_apply(G, ax, ay, c->cf, c->x, c->q2[0], s));
    AMR_HIP(c, amr_axpy(n, -1.0, c->q2[0], c->b, c->r, s));
  }
  double d2[2];
  AMR_TRY(dots(c, 2, c->b, c->b, c->r, c->r, d2));
  const double bb = d2[0];
  double res = bb > 0.0 ? std::sqrt(d2[1] / bb) : 0.0;
  const double res0 = res;
  // the iteration's scalars stay on the device (amr_reduce); the host
  // reads (r, r) once per iteration for the stop test
  int k = 0;
  bool converged = !(res > c->p.rtol);
  const int nbd = amr_dot_blocks(G);
  double rr = 0.0;
  while (!converged && k < c->p.max_cycles) {
    double* p = c->p2[k & 1];
    double* p_old = c->p2[(k + 1) & 1];
    double* q = c->q2[k & 1];
    double* q_old = c->q2[(k + 1) & 1];
    AMR_TRY(precondition(c, c->r, c->z));
    if (k > 0) {
      AmrDots D{};
      D.n = 1;
      D.u[0] = c->z;
      D.v[0] = q_old;
      AMR_HIP(c, amr_dots(G, D, c->partials, s));
      AMR_HIP(c, amr_reduce(c->partials, nbd, 1, c->sc, 0, 0, s));
    }
    AMR_HIP(c, amr_dir(n, c->z, p_old, p, c->sc, k == 0, s));
    AMR_HIP(c, amr_apply(G, ax, ay, c->cf, p, q, s, c->r, c->partials));
    AMR_HIP(c, amr_reduce(c->partials, nbd, 2, c->sc, 2, 0, s));
    AMR_HIP(c, amr_update(G, p, q, c->x, c->r, c->sc, c->partials, s));
    AMR_HIP(c, amr_reduce(c->partials, nbd, 1, c->sc, 4, 1, s));
    AMR_HIP(c, hipMemcpyAsync(&rr, c->sc + 4, sizeof(double),
                              hipMemcpyDeviceToHost, s));
    AMR_HIP(c, hipStreamSynchronize(s));
    res = std::sqrt(rr / bb);
    ++k;
    converged = !(res > c->p.rtol);
    if (!std::isfinite(res)) break;
  }
  precond_end(c->base);
  AMR_HIP(c, amr_unpack(G, c->x, E_b_out, E_f_out, s));
  AMR_HIP(c, hipStreamSynchronize(s));
  for (size_t k = 0; k < c->ev_used; ++k) {
    float ms = 0.0f;
    AMR_HIP(c, hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
    c->t_ms += ms;
    c->t_launches += 1;
    // one colour: g and the four faces of half the level-1 cells read, e
    // of every level-1 cell read once, half of e written
    c->t_bytes += 8.0 * (double)(G.off[1] - G.off[0]) *
                  (0.5 + 2.0 + 1.0 + 0.5);
  }
  c->ev_used = 0;
  if (stats) {
    stats->cycles = k;
    stats->outer_iters = k;
    stats->guess_rejected = 0;
    stats->guess_skipped = 0;
    stats->precond_fp64 = 1;
    stats->rel_res_initial = res0;
    stats->rel_res_final = res;
  }
  if (!converged)
    return amr_fail(c, FLD_ERR_NOT_CONVERGED,
                    "relative residual %.3e > rtol %.3e after %d iterations",
                    res, c->p.rtol, k);
  return FLD_OK;
}

}  // namespace

extern "C" {

size_t fld_amr_workspace_bytes_levels(const fld_params* p, int32_t block,
                                      int32_t nlevels, const int32_t* nblocks,
                                      const int32_t* blocks_xy) {
  if (!validate_amr(p, block, nlevels, nblocks, blocks_xy).empty()) return 0;
  const fld_params bp = base_params(*p);
  if (fld_workspace_bytes(&bp) == 0) return 0;
  return make_amr_plan(*p, block, nlevels, nblocks).total;
}

size_t fld_amr_workspace_bytes(const fld_params* p, int32_t block,
                               const int32_t* blocks_xy, int32_t nblocks) {
  return fld_amr_workspace_bytes_levels(p, block, 1, &nblocks, blocks_xy);
}

fld_status fld_amr_setup_levels(const fld_params* p, int32_t block,
                                int32_t nlevels, const int32_t* nblocks,
                                const int32_t* blocks_xy, void* workspace,
                                size_t ws_bytes, void* hip_stream,
                                fld_amr_ctx** out) {
  if (!out) return amr_fail(nullptr, FLD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  const std::string why = validate_amr(p, block, nlevels, nblocks, blocks_xy);
  if (!why.empty()) return amr_fail(nullptr, FLD_ERR_INVALID_ARG, "%s", why.c_str());
  const AmrPlan P = make_amr_plan(*p, block, nlevels, nblocks);
  if (!workspace || ws_bytes < P.total)
    return amr_fail(nullptr, FLD_ERR_WORKSPACE,
                    "workspace of %zu bytes needed", P.total);
  if ((uintptr_t)workspace % kAlign)
    return amr_fail(nullptr, FLD_ERR_WORKSPACE, "workspace not 256-aligned");
  char* w = (char*)workspace;
  fld_amr_ctx* c = new fld_amr_ctx();
  c->p = *p;
  c->stream = (hipStream_t)hip_stream;
  const fld_params bp = base_params(*p);
  fld_status st = fld_setup(&bp, w + P.base_ws, fld_workspace_bytes(&bp),
                            hip_stream, &c->base);
  if (st != FLD_OK) {
    delete c;
    return amr_fail(nullptr, st, "base grid set-up: %s",
                    fld_last_error(nullptr));
  }
  AmrGeom& G = c->G;
  G.nx = (int)p->n[0];
  G.ny = (int)p->n[1];
  G.b = block;
  G.S = 2 * block;
  G.nbx = G.nx / block;
  G.nby = G.ny / block;
  for (int d = 0; d < 2; ++d) G.per[d] = p->bc_lo[d] == FLD_BC_PERIODIC;
  G.Nb = P.Nb;
  G.Nf = P.Nf;
  G.dx = p->dx[0];
  G.dy = p->dx[1];
  G.vb = G.dx * G.dy;
  G.L = 0;
  G.off[0] = 0;
  for (int l = 1; l <= nlevels; ++l)
    if (nblocks[l - 1] > 0) G.L = l;
  // tables: the block of every unit of each level's parent lattice, each
  // block's corner
  std::vector<std::vector<int>> maps(nlevels), corners(nlevels);
  const int32_t* xy = blocks_xy;
  for (int l = 1; l <= nlevels; ++l) {
    const int ux = (G.nx << (l - 1)) / block, uy = (G.ny << (l - 1)) / block;
    G.units_x[l - 1] = ux;
    G.nblk[l - 1] = nblocks[l - 1];
    G.off[l] = G.off[l - 1] + (int64_t)nblocks[l - 1] * G.S * G.S;
    maps[l - 1].assign((size_t)ux * uy, -1);
    corners[l - 1].resize((size_t)2 * nblocks[l - 1]);
    for (int32_t k = 0; k < nblocks[l - 1]; ++k, xy += 2) {
      corners[l - 1][2 * k] = xy[0];
      corners[l - 1][2 * k + 1] = xy[1];
      maps[l - 1][(size_t)xy[1] * ux + xy[0]] = k;
    }
    G.bmap[l - 1] = (int*)(w + P.bmap[l - 1]);
    G.bxy[l - 1] = (int*)(w + P.bxy[l - 1]);
  }
  c->P.c = p->c;
  c->P.limiter = p->limiter;
  c->P.face_mean = p->face_mean;
  c->Ev = (double*)(w + P.views);
  c->rv = c->Ev + P.Nb;
  c->kv = c->rv + P.Nb;
  c->Evf = (double*)(w + P.fviews);
  c->rvf = c->Evf + P.Nf;
  c->kvf = c->rvf + P.Nf;
  c->Db = (double*)(w + P.Db);
  c->Df = (double*)(w + P.Df);
  c->cf = (double*)(w + P.cf);
  c->rhs = (double*)(w + P.rhs);
  double* v = (double*)(w + P.vec);
  double** vecs[10] = {&c->x, &c->b, &c->r, &c->z, &c->p2[0],
                       &c->p2[1], &c->q2[0], &c->q2[1], &c->t, &c->g};
  for (int k = 0; k < 10; ++k) *vecs[k] = v + (size_t)k * P.nvec;
  c->partials = (double*)(w + P.partials);
  c->sc = (double*)(w + P.sc);
  c->bad = (int*)(w + P.bad);
  hipError_t e = hipSuccess;
  for (int l = 0; l < nlevels && e == hipSuccess; ++l) {
    e = hipMemcpyAsync((void*)G.bmap[l], maps[l].data(), maps[l].size() * 4,
                       hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && !corners[l].empty())
      e = hipMemcpyAsync((void*)G.bxy[l], corners[l].data(),
                         corners[l].size() * 4, hipMemcpyHostToDevice,
                         c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    fld_destroy(c->base);
    delete c;
    return amr_fail(nullptr, FLD_ERR_DEVICE, "table upload: %s",
                    hipGetErrorString(e));
  }
  *out = c;
  return FLD_OK;
}

fld_status fld_amr_setup(const fld_params* p, int32_t block,
                         const int32_t* blocks_xy, int32_t nblocks,
                         void* workspace, size_t ws_bytes, void* hip_stream,
                         fld_amr_ctx** out) {
  return fld_amr_setup_levels(p, block, 1, &nblocks, blocks_xy, workspace,
                              ws_bytes, hip_stream, out);
}

fld_status fld_amr_step(fld_amr_ctx* c, double dt, const double* rho_base,
                        const double* kappa_base, const double* E_base_in,
                        double* E_base_out, const double* rho_fine,
                        const double* kappa_fine, const double* E_fine_in,
                        double* E_fine_out, fld_stats* stats) {
  if (!c) return amr_fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (!rho_base || !kappa_base || !E_base_in || !E_base_out)
    return amr_fail(c, FLD_ERR_INVALID_ARG, "NULL base field pointer");
  if (c->G.Nf > 0 && (!rho_fine || !kappa_fine || !E_fine_in || !E_fine_out))
    return amr_fail(c, FLD_ERR_INVALID_ARG, "NULL fine field pointer");
  if (!(dt > 0.0) || !std::isfinite(dt))
    return amr_fail(c, FLD_ERR_INVALID_ARG, "dt must be positive and finite");
  // in place is allowed: the inputs are read before the outputs are written
  return amr_solve(c, dt, rho_base, kappa_base, E_base_in, E_base_out,
                   rho_fine, kappa_fine, E_fine_in, E_fine_out, stats);
}

fld_status fld_amr_exchange(fld_amr_ctx* c, double dt, const double* rho_base,
                            const double* kappa_base, double* E_base,
                            double* e_base, const double* rho_fine,
                            const double* kappa_fine, double* E_fine,
                            double* e_fine) {
  if (!c) return amr_fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (!rho_base || !kappa_base || !E_base || !e_base)
    return amr_fail(c, FLD_ERR_INVALID_ARG, "NULL base field pointer");
  if (c->G.Nf > 0 && (!rho_fine || !kappa_fine || !E_fine || !e_fine))
    return amr_fail(c, FLD_ERR_INVALID_ARG, "NULL fine field pointer");
  if (!(dt > 0.0) || !std::isfinite(dt))
    return amr_fail(c, FLD_ERR_INVALID_ARG, "dt must be positive and finite");
  const fld_params& p = c->p;
  AMR_HIP(c, launch_exchange(c->G.Nb, dt, p.c, p.a_rad, p.gamma, p.gas_const,
                             rho_base, kappa_base, E_base, e_base, c->stream));
  if (c->G.Nf > 0)
    AMR_HIP(c, launch_exchange(c->G.Nf, dt, p.c, p.a_rad, p.gamma,
                               p.gas_const, rho_fine, kappa_fine, E_fine,
                               e_fine, c->stream));
  return FLD_OK;
}

fld_status fld_amr_opacity_powerlaw(fld_amr_ctx* c, const double* rho_base,
                                    const double* e_base,
                                    const double* rho_fine,
                                    const double* e_fine, double k0, double a,
                                    double b, double kmin, double kmax,
                                    double* kappa_base, double* kappa_fine) {
  if (!c) return amr_fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (!rho_base || !e_base || !kappa_base)
    return amr_fail(c, FLD_ERR_INVALID_ARG, "NULL base field pointer");
  if (c->G.Nf > 0 && (!rho_fine || !e_fine || !kappa_fine))
    return amr_fail(c, FLD_ERR_INVALID_ARG, "NULL fine field pointer");
  if (!(k0 > 0.0) || !(kmin > 0.0) || !(kmax >= kmin) || !std::isfinite(a) ||
      !std::isfinite(b) || !std::isfinite(kmax))
    return amr_fail(c, FLD_ERR_INVALID_ARG,
                    "need k0 > 0, 0 < kmin <= kmax, finite exponents");
  const fld_params& p = c->p;
  AMR_HIP(c, launch_opacity(c->G.Nb, p.gamma, p.gas_const, rho_base, e_base,
                            k0, a, b, kmin, kmax, kappa_base, c->stream));
  if (c->G.Nf > 0)
    AMR_HIP(c, launch_opacity(c->G.Nf, p.gamma, p.gas_const, rho_fine, e_fine,
                              k0, a, b, kmin, kmax, kappa_fine, c->stream));
  return FLD_OK;
}

fld_status fld_amr_kernel_timing_enable(fld_amr_ctx* c, int32_t on) {
  if (!c) return amr_fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  c->timing = on != 0;
  c->ev_used = 0;
  return FLD_OK;
}

fld_status fld_amr_kernel_timing_read(fld_amr_ctx* c, double* ms_total,
                                      int64_t* launches, double* bytes_total,
                                      const char** kernel_name) {
  if (!c) return amr_fail(nullptr, FLD_ERR_INVALID_ARG, "ctx is NULL");
  if (ms_total) *ms_total = c->t_ms;
  if (launches) *launches = c->t_launches;
  if (bytes_total) *bytes_total = c->t_bytes;
  if (kernel_name) *kernel_name = "k_amr_smooth_level";
  c->t_ms = c->t_bytes = 0.0;
  c->t_launches = 0;
  return FLD_OK;
}

const char* fld_amr_last_error(const fld_amr_ctx* c) {
  return c ? c->err.c_str() : g_amr_err.c_str();
}

void fld_amr_destroy(fld_amr_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  fld_destroy(c->base);
  delete c;
}

}  // extern "C"
