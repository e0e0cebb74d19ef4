// Internal declarations of the FLD library: grid geometry, per-level views,
// the device-side control block and the kernel launch wrappers.
//
// Layout: every field is a contiguous array, x fastest
// (idx = i + nx * (j + ny * k)).  A face coefficient alpha_d[idx] belongs to
// the face between cell idx and its +d neighbour; along a Neumann dimension
// the last cell's +d face is a wall and holds 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fld {

constexpr int kMaxLevels = 24;
constexpr int kBlock = 256;        // threads per block of the grid kernels
constexpr int kReduceBlock = 1024; // threads of the single-block reductions

struct Geom {
  int ndim;
  int n[3];    // cells per dimension (unused = 1)
  int per[3];  // 1 if periodic along that dimension
  int dirw[3]; // Dirichlet walls along that dimension: bit 0 lower, 1 upper
  int64_t N;   // cells
};

template <typename T>
struct LevelView {
  Geom g;
  T* x;          // iterate (correction on coarse levels)
  T* b;          // right-hand side (restricted residual on coarse levels)
  const T* a[3]; // face coefficients, one array per dimension
  // Dirichlet walls' diagonal term per cell (null without such walls): the
  // operator is (1 + sd) x + sum_f alpha_f (x - x_f)
  const T* sd;
  // coarse levels with held cells below them (null otherwise): nonzero
  // where some child is held; such a cell's correction stays 0
  const uint8_t* held;
};

// Device control block of one solve: norms, counters and the stop flag
// that every multigrid kernel reads before doing any work.
struct Control {
  double bnorm2;      // |b|^2 of the finest level
  double res_initial; // |b - A x0| / |b|
  double res;         // relative residual of the returned iterate
  double rtol;
  double guess_ref;   // |b - A E^n|^2, the learned guess's benchmark
  int32_t done;       // 0 running, 1 converged, 2 cycle cap, 3 non-physical
  int32_t cycles;
  int32_t max_cycles;
  int32_t flagged;    // non-physical cells seen by the coefficient kernel
  int32_t outer;      // refinement iterations (corrections applied)
  int32_t inner;      // FP32 V-cycles per refinement iteration
  int32_t guess_rejected;  // 1 when the learned guess lost to E^n
  int32_t stop_in_down;    // the stop test fired after a finest down pass
                           // (tiled path: the iterate is in the alternate
                           // buffer)
  double fcg_beta;    // flexible CG: the current direction's beta,
  double fcg_alpha;   // step length,
  double fcg_pq;      // and (p, A p) of the last direction
  Control* mirror;    // device address of the host-visible copy (or null)
};

enum DoneCode { kRunning = 0, kConverged = 1, kCapped = 2, kNonPhysical = 3 };

struct CoefArgs {
  Geom g;
  double dx[3];
  double gscale[3];  // 1 / (12 dx): the five-point gradient's scale
  double dt, c;
  int limiter;   // 0 LP, 1 diffusion, 2 Minerbo
  int face_mean; // 0 arithmetic, 1 harmonic
  double wall[3][2];  // E held on the Dirichlet walls (g.dirw), lower, upper
};

// Explicit source terms of one grid (fld_explicit_sources): inputs E, rho,
// kappa and ndim velocity components; every output pointer may be null.
struct ExplicitArgs {
  Geom g;
  double gscale[3];  // 1 / (12 dx): the five-point gradient's scale
  int limiter;
  const double* E;
  const double* rho;
  const double* kappa;
  const double* v[3];
  double* fr[3];
  double* work;
  double* tiring;
  double* fedd;
};

// ---- launch wrappers (kernels live in the .hip files) ----------------------
// *nblocks (if given) receives the number of block partial sums of |E|^2.
hipError_t launch_coef(const CoefArgs& a, const double* E, const double* rho,
                       const double* kappa, double* const a64[3],
                       float* const a32[3], double* copy_dst, double* partials,
                       Control* ctrl, hipStream_t s, int* nblocks = nullptr,
                       double* dscr = nullptr, double* sd = nullptr,
                       double* rhs = nullptr, const uint8_t* held = nullptr,
                       const double* hold = nullptr);
// With rhs the coefficient stage also writes the finest level's own
// right-hand side (one-pass kernels): with sd each cell's Dirichlet-wall
// diagonal term (0 off the walls of a.g.dirw) and E^n + sum alpha_w E_w;
// with held cells (mask `held`) the prescribed value `hold` in them.
// launch_coarsen_sd carries the diagonal term to a coarse level.
hipError_t launch_coarsen_sd(const Geom& fine, const Geom& coarse,
                             const double* sdf, double* sdc, hipStream_t s);
// Held cells eliminated from the free cells' rows, after the coefficient
// stage: launch_held_fold moves each free cell's faces to held neighbours
// onto its diagonal (sd) and their held values times alpha onto its
// right-hand side (rhs), and leaves the per-block sums of rhs^2 in
// partials (*nblocks of them); launch_held_cut then zeroes every face
// that touches a held cell, so a held row is x = b = E_hold.
hipError_t launch_held_fold(const Geom& g, double* const a[3],
                            const uint8_t* held, const double* hold,
                            double* sd, double* rhs, double* partials,
                            int* nblocks, hipStream_t s);
hipError_t launch_held_cut(const Geom& g, double* const a[3],
                           const uint8_t* held, hipStream_t s);
// Coarse held mask: nonzero where some child is held.
hipError_t launch_coarsen_held(const Geom& fine, const Geom& coarse,
                               const uint8_t* hf, uint8_t* hc, hipStream_t s);
hipError_t launch_finalize(int mode, const double* partials, int count,
                           Control* ctrl, hipStream_t s);
hipError_t launch_exchange(int64_t N, double dt, double c, double a_rad,
                           double gamma, double gas_const, const double* rho,
                           const double* kappa, double* E, double* e,
                           hipStream_t s);
hipError_t launch_opacity(int64_t N, double gamma, double gas_const,
                          const double* rho, const double* e, double k0,
                          double pa, double pb, double kmin, double kmax,
                          double* kappa, hipStream_t s);
hipError_t launch_resid_to32(const LevelView<double>& L, float* r32,
                             double* partials, int* nblocks,
                             const Control* ctrl, hipStream_t s);
hipError_t launch_correct(int64_t N, double* x, const float* e,
                          const Control* ctrl, hipStream_t s);

// Fused red-black sweep of a 3D level, out of place: xo = one Gauss-Seidel
// sweep (red, then black) of L.x.  Levels of nx % 64 == 0, ny % 16 == 0 and
// two colours; zc = z planes per block (0: chosen from the shape).
bool gs_sweep3d_ok(const Geom& g);
template <typename T>
hipError_t launch_gs_sweep3d(const LevelView<T>& L, T* xo, int zc,
                             const Control* ctrl, hipStream_t s,
                             hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// The same sweep by 32 x 8 x 4 tiles in one launch (fld_tile3d.hip), for
// levels too small for the z-marching sweep: nx % 32 == 0, ny % 8 == 0,
// nz % 4 == 0 and two colours.
bool gs_tile3d_ok(const Geom& g);
template <typename T>
hipError_t launch_gs_tile3d(const LevelView<T>& L, T* xo, const Control* ctrl,
                            hipStream_t s, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr);

template <typename T>
hipError_t launch_coarsen(const Geom& fine, const Geom& coarse,
                          const T* const fa[3], T* const ca[3], hipStream_t s);
// Coefficients of levels 1 .. L-1 of a 2D hierarchy from those of level 0,
// several levels per launch; a[l][d] holds level l's faces along d.
template <typename T>
hipError_t launch_coarsen2d(const Geom* g, int L, T* const (*a)[3],
                            hipStream_t s);
template <typename T>
hipError_t launch_resid_norm(const LevelView<T>& L, double* partials,
                             int* nblocks, const Control* ctrl, hipStream_t s);
// With ev0/ev1 given (3D levels), the launch itself records them.
template <typename T>
hipError_t launch_gs_color(const LevelView<T>& L, int color,
                           const Control* ctrl, hipStream_t s,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename T>
hipError_t launch_resid_restrict(const LevelView<T>& fine,
                                 const LevelView<T>& coarse, double* partials,
                                 int* nblocks, const Control* ctrl,
                                 hipStream_t s);
template <typename T>
hipError_t launch_prolong(const LevelView<T>& coarse, const LevelView<T>& fine,
                          const Control* ctrl, hipStream_t s);
template <typename T>
hipError_t launch_coarsest(const LevelView<T>& L, T* tmp, const Control* ctrl,
                           hipStream_t s);

// Single-workgroup V-cycle tail: levels l0 .. L-1 (see k_tail).
template <typename T>
struct TailArgs {
  int l0, L, pre, post;
  int whole;  // run the cycle loop and the stop test (FP64, l0 == 0)
  int zero;   // x(l0) starts at zero (else it is read)
  LevelView<T> lv[kMaxLevels];
  T* tmp;
  Control* ctrl;
};
template <typename T>
hipError_t launch_tail(const TailArgs<T>& a, hipStream_t s);
// LDS variant (fld_tail.hip); *used = false when the levels do not fit.
template <typename T>
hipError_t launch_tail_lds(const TailArgs<T>& a, hipStream_t s, bool* used);
// Blocks of the 3D launch grid of the one-pass kernels over level g (their
// partial sums: one per block).
int64_t blocks3(const Geom& g);
// LDS-tiled coefficient stage of a 2D grid (fld_coef2d.hip), for grids of at
// least 4 x 4 cells (coef2d_ok): k_coef's coefficients, and with `resid` the
// initial residual of x0 = E^n as well (finalize with kFinCoef).
bool coef2d_ok(const Geom& g);
int coef2d_blocks(const Geom& g);
hipError_t launch_coef2d(const CoefArgs& a, const double* E, const double* rho,
                         const double* kappa, double* const a64[3],
                         float* const a32[3], double* copy_dst,
                         double* partials, Control* ctrl, bool resid,
                         hipStream_t s);
// Two-dimensional register tail (fld_tail2d.hip) for sub-V-cycles whose
// levels fit it (tail2d_ok); launched by launch_tail_lds when they do.
template <typename T>
bool tail2d_ok(const TailArgs<T>& a);
template <typename T>
hipError_t launch_tail2d(const TailArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_tail2d_batch(const TailArgs<T>* tab, int ng, hipStream_t s);
// The same for tails whose first level has 1025..4096 cells (one block of
// 1024 threads); tail2d_big_fits checks the level geometries g[0..nt).
bool tail2d_big_fits(const Geom* g, int nt);
template <typename T>
bool tail2d_big_ok(const TailArgs<T>& a);
template <typename T>
hipError_t launch_tail2d_big(const TailArgs<T>& a, hipStream_t s);
// LDS bytes the LDS tail needs (0 when the levels do not fit).
template <typename T>
size_t tail_lds_bytes(const TailArgs<T>& a);
// Batched LDS tail: block g runs tab[g] (device memory); lds = max bytes.
template <typename T>
hipError_t launch_tail_lds_batch(const TailArgs<T>* tab, int ng, int nd,
                                 size_t lds, hipStream_t s);

hipError_t launch_ctrl_init(Control* ctrl, double rtol, int max_cycles,
                            int inner, Control* mirror, hipStream_t s);
hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s);
hipError_t launch_explicit(const ExplicitArgs& a, hipStream_t s);
// Learned guess judge: mode 0 stores the summed partials as the benchmark
// |b - A x_prev|^2; mode 1 rejects the guess unless its |b - A x|^2 is below
// q2 times that benchmark (q2 = 1: any smaller residual; q2 = rho^2, rho a
// V-cycle's contraction: the guess must be worth at least one cycle), or
// when it is not finite.  launch_guess_take then copies the guess into the
// iterate where it was accepted.
hipError_t launch_guess_judge(int mode, const double* partials, int count,
                              double q2, Control* ctrl, hipStream_t s);
hipError_t launch_guess_take(int64_t n, const double* guess, double* x,
                             const Control* ctrl, hipStream_t s);
// x = alt where the solve stopped right after a finest down pass
hipError_t launch_take_alt(int64_t n, const double* alt, double* x,
                           const Control* ctrl, hipStream_t s);
hipError_t launch_fill32(float* x, int64_t n, hipStream_t s);

// Levels up to this many cells run in the single-workgroup tail, in LDS.
constexpr int64_t kTailLdsCells = 1024;
// 3D coarse levels of at most this many cells above the tail run their down
// and up passes in one workgroup each (fld_level.hip)
constexpr int kLevelLdsCells = 4096;
bool level_lds_ok(const Geom& g, const Geom& coarse);
template <typename T>
hipError_t launch_level_down(const LevelView<T>& F, const LevelView<T>& C,
                             int sweeps, const Control* ctrl, hipStream_t s);
template <typename T>
hipError_t launch_level_up(const LevelView<T>& F, const LevelView<T>& C,
                           int sweeps, const Control* ctrl, hipStream_t s);

// finalize modes
// kFinOuter: FP64 residual of a refinement iteration (first call also sets
// the initial residual); counts outer iterations.
enum FinalizeMode {
  kFinBnorm = 0,
  kFinInitial = 1,
  kFinCycle = 2,
  kFinOuter = 3,
  kFinCoef = 4,  // |b|^2 in partials[0, count), |b - A x0|^2 in [count, 2 count)
  kFinKrylov = 5,  // |r|^2 after a flexible-CG iteration (counts iterations)
  kFinRestart = 6  // |r|^2 of a flexible-CG restart with FP64 V-cycles
                   // (one V-cycle per iteration from then on)
};

// Flexible CG around the V-cycle (fld_krylov.hip): level-0 geometry and
// face coefficients, the FP64 residual r (and its FP32 copy for FP32
// V-cycles, or null), the previous and new directions p, q = A p, block
// partials and the control block (scalars beta, alpha, (p, q)).
struct KrylovArgs {
  Geom g;
  const double* a[3];
  double* r;
  float* r32;
  const double* p_old;
  double* p_new;
  double* q;
  double* partials;
  Control* ctrl;
};
constexpr int kKrylovBlocks = 2048;
int krylov_blocks(const Geom& g);  // blocks (and partials) of each pass
hipError_t launch_fcg_init(const KrylovArgs& K, const double* x,
                           const double* b, hipStream_t s);
template <typename TZ>
hipError_t launch_fcg_zq(const KrylovArgs& K, const TZ* z, hipStream_t s);
template <typename TZ>
hipError_t launch_fcg_dir(const KrylovArgs& K, const TZ* z, int first,
                          hipStream_t s);
hipError_t launch_fcg_update(const KrylovArgs& K, double* x, hipStream_t s);
hipError_t launch_fcg_scalar(int mode, const KrylovArgs& K, hipStream_t s);

// Colour classes of the Gauss-Seidel sweeps.  Red-black by (x + y + z) & 1
// is a proper colouring unless a periodic dimension has odd length: there
// cells n-1 and 0 are neighbours of the same parity.  Cells on the last
// slab of such a dimension therefore get passes of their own: the class of a
// cell is (set of odd periodic dimensions on whose last slab it lies, parity
// of its other coordinates), numbered 2 * set + parity.  Two neighbours
// differ in one coordinate: either the set differs, or the parity does.
// Without odd periodic dimensions the classes are the two usual colours.
template <class G>
__host__ __device__ inline bool gs_odd_periodic(const G& g, int d) {
  return g.per[d] && (g.n[d] & 1) && g.n[d] > 1;
}

template <class G>
__host__ __device__ inline int gs_colors(const G& g) {
  int k = 0;
  for (int d = 0; d < 3; ++d) k += gs_odd_periodic(g, d) ? 1 : 0;
  return 2 << k;
}

template <class G>
__host__ __device__ inline int gs_color(const G& g, const int c[3]) {
  int set = 0, bit = 0, par = 0;
  for (int d = 0; d < 3; ++d) {
    const bool odd = gs_odd_periodic(g, d);
    if (odd && c[d] == g.n[d] - 1)
      set |= 1 << bit;
    else
      par += c[d];
    bit += odd ? 1 : 0;
  }
  return 2 * set + (par & 1);
}

inline int blocks_for(int64_t n, int bs = kBlock) {
  return (int)((n + bs - 1) / bs);
}

}  // namespace fld
