/*
 * fld.h - implicit flux-limited-diffusion (FLD) radiation-energy update on
 * one AMD Instinct MI355X (gfx950).
 *
 * The update is the stiff part of a split radiation-MHD step (Narechania et
 * al., "Radiation-magnetohydrodynamics with MPI-AMRVAC using flux-limited
 * diffusion", arXiv:2503.02764):
 *
 *   fld_step      diffusion: dE/dt = -div F with F = -D grad E (eq. fld_F),
 *                 D = c lambda / (rho kappa), lambda the flux limiter of
 *                 eq. fld_lambda with R of eq. fld_R, the gradient by the
 *                 five-point central stencil of Sect. 3, advanced by one
 *                 backward-Euler step and solved by geometric multigrid
 *                 (Sect. 3 solves div F with multigrid).
 *   fld_exchange  gas-radiation energy exchange qdot of eqs. heating/qdot,
 *                 implicit in both the gas and the radiation energy, which
 *                 leaves one quartic per cell (Sect. 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Fields are DEVICE pointers to contiguous float64 arrays of
 *   nx*ny*nz cells, x fastest: index i + nx*(j + ny*k).  The caller owns
 *   them; the library never keeps a pointer past the call.
 * - All work is enqueued on the HIP stream given to fld_setup, in stream
 *   order.  The context is not thread-safe: one context per stream.
 * - Code units are the caller's: c, a_rad, gamma and gas_const
 *   (= k_B / (mu m_p), so that p = rho gas_const T, eq. ideal_gas_law) are
 *   parameters.  e_int is the gas internal energy density p / (gamma - 1)
 *   (eq. energy_density with v = B = 0).
 * - Errors: host validation fails fast with FLD_ERR_INVALID_ARG and
 *   launches nothing.  A HIP runtime failure gives FLD_ERR_DEVICE.  Every
 *   failing call stores a message readable with fld_last_error.
 */
#ifndef FLD_H
#define FLD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fld_ctx fld_ctx;

typedef enum {
  FLD_OK = 0,
  FLD_ERR_INVALID_ARG = 1,   /* bad argument; nothing was launched          */
  FLD_ERR_WORKSPACE = 2,     /* workspace missing, too small or misaligned  */
  FLD_ERR_DEVICE = 3,        /* a HIP call failed                           */
  FLD_ERR_NONPHYSICAL = 4,   /* E <= 0, rho*kappa <= 0 or a non-finite input */
  FLD_ERR_NOT_CONVERGED = 5, /* max_cycles reached; last iterate returned   */
  FLD_ERR_MODEL = 6          /* learned-guess weights rejected              */
} fld_status;

/* Boundary condition of one side of one dimension.  Periodic must be set on
 * both sides of a dimension.  Neumann is the paper's zero-gradient boundary
 * (Sect. 4.1, 4.4): mirror ghost cells for the gradient (E[-1] = E[0],
 * E[-2] = E[1]) and no flux through the boundary face.  Dirichlet holds E
 * at bc_value_lo/hi on the boundary face (the radiation temperature tied to
 * the gas temperature on the walls of the magnetoconvection case, Sect.
 * 4.5): the gradient's ghosts are the mirror ghosts reflected about that
 * value (2 E_w - E[0], 2 E_w - E[1]), and the boundary face, half a cell
 * from the centre with the boundary cell's D, adds alpha_w = 2 dt D / dx^2
 * to the cell's diagonal and alpha_w E_w to its right-hand side.  Contexts
 * with a Dirichlet wall solve in FP64 with V-cycles alone (precision FP64,
 * krylov 0, guess E^n or zero, not batched) on the one-launch-per-pass
 * kernels; fld_explicit_sources rejects them. */
typedef enum {
  FLD_BC_PERIODIC = 0,
  FLD_BC_NEUMANN = 1,
  FLD_BC_DIRICHLET = 2
} fld_bc;

/* eq. fld_lambda (Levermore-Pomraning), the diffusion value 1/3 used by
 * the paper for its stationary shocks (Sect. 4.1), or Minerbo's limiter
 * (named in Sect. 2 as an alternative; the paper gives no formula, so its
 * published piecewise form is used: lambda = 2 / (3 + sqrt(9 + 12 R^2)) for
 * R <= 3/2 and 1 / (1 + R + sqrt(1 + 2 R)) above). */
typedef enum { FLD_LIMITER_LP = 0, FLD_LIMITER_DIFFUSION = 1,
               FLD_LIMITER_MINERBO = 2 } fld_limiter;

/* Mean of the two cell-centred D on a face. */
typedef enum { FLD_FACE_ARITH = 0, FLD_FACE_HARMONIC = 1 } fld_face_mean;

/* FP64 multigrid, or FP32 V-cycles inside an FP64 iterative refinement.
 * The exchange is FP64 in both. */
typedef enum { FLD_PREC_FP64 = 0, FLD_PREC_FP32_IR = 1 } fld_precision;

/* Initial guess of the diffusion solve: E^n, zero, or a learned guess. */
typedef enum { FLD_GUESS_PREV = 0, FLD_GUESS_ZERO = 1, FLD_GUESS_LEARNED = 2 } fld_guess;

/* When the learned guess evaluates its network (FLD_GUESS_LEARNED only).
 * FLD_GUESS_ADAPTIVE: the context's first step runs without the network and
 * its count of V-cycles (FP64) or refinement iterations (FP32_IR), and the
 * solve's time per cycle or iteration (events on the stream), become the
 * reference, which every later step without the network renews.  A step
 * with the network pays when the cycles or iterations it saved took longer
 * than the network did.  One that does not pay (or whose guess the
 * residual judge rejects) makes the next 2, 4, 8, 16, then 32 steps run
 * without it before it is tried again; one where the network took longer
 * than all but one cycle or iteration of a solve without it (a solve runs
 * at least one) makes the next 32 steps run without it; a step that pays
 * keeps it on for the next step.  A step without the network
 * is exactly a step with guess E^n.  FLD_GUESS_EVERY_STEP: the network runs
 * on every step. */
typedef enum { FLD_GUESS_ADAPTIVE = 0, FLD_GUESS_EVERY_STEP = 1 } fld_guess_policy;

typedef struct {
  int32_t ndim;          /* 1, 2 or 3                                      */
  int32_t pad0;
  int64_t n[3];          /* cells per dimension; unused dimensions = 1     */
  double dx[3];          /* cell widths; unused = 1                        */
  int32_t bc_lo[3];      /* fld_bc per dimension                           */
  int32_t bc_hi[3];
  double c;              /* speed of light                                 */
  double a_rad;          /* radiation constant a_r = 4 sigma / c           */
  double gamma;          /* adiabatic index, > 1                           */
  double gas_const;      /* k_B / (mu m_p)                                 */
  int32_t limiter;       /* fld_limiter                                    */
  int32_t face_mean;     /* fld_face_mean                                  */
  int32_t precision;     /* fld_precision                                  */
  int32_t guess;         /* fld_guess                                      */
  double rtol;           /* stop when |b - A x|_2 / |b|_2 <= rtol          */
  int32_t max_cycles;    /* V-cycle cap (fine-level smoothing passes)      */
  int32_t pre_smooth;    /* red-black Gauss-Seidel sweeps before restriction */
  int32_t post_smooth;   /* sweeps after prolongation                      */
  int32_t ir_inner;      /* FP32 V-cycles per refinement iteration
                            (FP32_IR), 1..8; 0 selects 2             */
  int32_t coarse_pre_smooth;   /* sweeps before restriction on the coarse
                                  levels; 0: pre_smooth                   */
  int32_t coarse_post_smooth;  /* sweeps after prolongation on the coarse
                                  levels; 0: post_smooth                  */
  int32_t guess_policy;  /* fld_guess_policy (learned guess only)         */
  int32_t krylov;        /* 0: the V-cycle is the iteration; 1: V-cycles
                            precondition flexible conjugate gradients
                            (stays convergent where coefficient jumps make
                            a V-cycle overshoot); single grids only.
                            With FP32_IR the FP32 V-cycles give way to
                            FP64 ones (same iterate) when the FP64
                            residual falls less than 4x over 4 iterations,
                            and the next 2, 4, ... 32 steps start with
                            FP64 ones; the workspace then also holds the
                            FP64 hierarchy                                */
  double bc_value_lo[3]; /* E on a Dirichlet lower / upper wall (finite,  */
  double bc_value_hi[3]; /* > 0); unused on other walls                   */
  int32_t held_cells;    /* 1: held cells (fld_set_held) take part in every
                            step; same restrictions as Dirichlet walls    */
} fld_params;

typedef struct {
  int32_t cycles;          /* fine-level V-cycles started (the last one may
                              stop after its pre-smoothing, where it found
                              the residual below rtol)                     */
  int32_t outer_iters;     /* FP64 refinement iterations (FP32_IR) or
                              flexible-CG iterations (krylov), else 0     */
  int32_t guess_rejected;  /* 1 when a learned guess lost to E^n          */
  int32_t guess_skipped;   /* 1 when FLD_GUESS_ADAPTIVE ran this step
                              without the network (guess E^n)              */
  int32_t precond_fp64;    /* FP32_IR with krylov: 1 when this step ran
                              flexible-CG iterations with FP64 V-cycles
                              (the FP32 ones stalled on it, or on a recent
                              step), else 0                                */
  int32_t pad;
  int64_t flagged_cells;   /* cells with E <= 0, rho kappa <= 0 or NaN     */
  double rel_res_initial;  /* |b - A x0| / |b|                              */
  double rel_res_final;    /* |b - A x| / |b| of the returned E_out        */
} fld_stats;

/* Fill *p with defaults: 1D, 1 cell, periodic, c = a_rad = gas_const = 1,
 * gamma = 5/3, LP limiter, arithmetic face mean, FP64, guess E^n
 * (adaptive network policy if the learned guess is chosen), rtol 1e-8,
 * max_cycles 50, V(2,2) on every level. */
void fld_params_default(fld_params* p);

/* Bytes of device workspace fld_setup needs for these parameters, or 0 if
 * the parameters are invalid. */
size_t fld_workspace_bytes(const fld_params* p);

/* Validate the parameters, build the multigrid level list (every dimension
 * halved while all sides are even and the halves are >= 3) and carve
 * per-level buffers out of `workspace` (device memory, >= 256-byte aligned,
 * ws_bytes >= fld_workspace_bytes(p)).  `hip_stream` is a hipStream_t (NULL:
 * the default stream).  Launches nothing.  The context keeps `workspace`
 * until fld_destroy; the caller keeps it alive. */
fld_status fld_setup(const fld_params* p, void* workspace, size_t ws_bytes,
                     void* hip_stream, fld_ctx** out);

/* One backward-Euler diffusion step: E_out = A^-1 E_in, with
 * (A x)_i = x_i + sum_faces alpha_f (x_i - x_nb), alpha_f = dt D_f / dx^2,
 * D_f the face mean of D = c lambda / (rho kappa) computed from E_in
 * (eqs. fld_F, fld_lambda, fld_R; gradient by the five-point stencil).
 * Solved by V-cycles until |E_in - A E_out|_2 / |E_in|_2 <= rtol.
 * rho, kappa, E_in: device, read only.  E_out: device, written; it may
 * alias E_in.  stats: host pointer or NULL.
 * Blocks the calling thread until convergence is known, with or without
 * stats: the number of V-cycles is not known in advance, so cycles are
 * enqueued in batches (sized by the last step's count) between reads of
 * the device's stop flag, and the host decides after each read whether to
 * enqueue more (a solve entirely on the device would need a launch that
 * enqueues launches, or a persistent kernel with grid barriers, which cost
 * as much as the launches they replace on this GPU).  Returns
 * FLD_ERR_NONPHYSICAL if any cell has E <= 0, rho kappa <= 0 or a
 * non-finite input (outputs unspecified), FLD_ERR_NOT_CONVERGED after
 * max_cycles (E_out holds the last iterate, stats the residual). */
fld_status fld_step(fld_ctx* ctx, double dt, const double* rho,
                    const double* kappa, const double* E_in, double* E_out,
                    fld_stats* stats);

/* fld_step for callers that cannot allocate (code that must not call
 * hipMalloc or hipHostMalloc: inside HIP graph capture set-up, tight serving
 * loops, harnesses that forbid allocation).  Same operation, arguments and
 * results as fld_setup + fld_step with the same parameters (the same kernels
 * with the default tile shape on every level), but with no context and no
 * workspace argument: the step's workspace is a static device array of
 * 64 MiB inside the library (one per device, held until the process ends),
 * and the control block is read back by a stream copy instead of a mapped
 * host mirror.  It calls no device or pinned allocation routine.
 *   p: host parameters (guess E^n or zero; FLD_GUESS_LEARNED gives
 *      FLD_ERR_INVALID_ARG).
 *   rho, kappa, E_in, E_out, stats: as for fld_step (device fields, E_out
 *      may alias E_in; stats host or NULL).
 *   hip_stream: a hipStream_t of the current device (NULL: default stream).
 * Limit: parameters whose fld_workspace_bytes exceeds 64 MiB are rejected
 * with FLD_ERR_WORKSPACE before anything is launched (2D grids up to about
 * 1024 x 1024 in either precision, 3D up to about 96^3).  Every call on one
 * device shares that device's array and leaves its contents behind (each
 * step initialises what it reads), so calls that overlap on one device,
 * from several threads or streams, race and must be serialised by the
 * caller.  Blocks until convergence is known, like fld_step.  Errors are
 * read with fld_last_error(NULL). */
fld_status fld_step_noalloc(const fld_params* p, double dt, const double* rho,
                            const double* kappa, const double* E_in,
                            double* E_out, fld_stats* stats,
                            void* hip_stream);

/* Held cells: an interior boundary whose cells take a prescribed new E
 * (the linear-wave tests of Sect. 4.3 overwrite the first wavelength of
 * the domain with a known solution).  A held cell's row of the system
 * becomes E*_i = E_hold[i]; every other row is unchanged, so a free cell
 * next to a held one couples to the held value through the usual face
 * coefficient (interior Dirichlet data at cell centres), and D is still
 * computed from E^n in every cell.  The library solves the equivalent
 * system with the held cells eliminated: a free cell's faces to held
 * neighbours go onto its diagonal and their held values times those faces
 * onto its right-hand side, and every face touching a held cell is cut, so
 * the free cells' block is symmetric.  On the coarse levels a cell with a
 * held child is a point of zero correction, coupled to its free neighbours
 * through faces coarsened from the faces before the cut.  The stop test's
 * |b| is that of the eliminated system's right-hand side.  Held cells end
 * exactly at E_hold.
 * mask: device array of the grid's cells (layout of E), nonzero = held;
 * E_hold: device array of the same cells (read where the mask is set;
 * must not overlap the step's E_out).  Both stay owned by the caller and
 * are read by every following fld_step, so they must stay valid until the
 * next fld_set_held or fld_destroy; their contents may change between
 * steps.  NULL for both clears them, after which fld_step fails until they
 * are given again.  Needs a context set up with held_cells = 1, whose
 * steps then solve in FP64 with V-cycles alone (precision FP64, krylov 0,
 * guess E^n or zero, not batched, not fld_step_noalloc) on the
 * one-launch-per-pass kernels.  FLD_ERR_INVALID_ARG otherwise, or when
 * only one of the two pointers is NULL.  Enqueues nothing. */
fld_status fld_set_held(fld_ctx* ctx, const uint8_t* mask,
                        const double* E_hold);

/* ---- Block-adaptive 2D grids ----------------------------------------
 * The backward-Euler diffusion step (eq. mhd_r_e, the implicit part of
 * Sect. 3) on a block-adaptive grid, as MPI-AMRVAC runs it (Sect. 3, 4.1):
 * a base grid of n[0] x n[1] cells (spacing dx[0], dx[1]) tiled by
 * `block` x `block` blocks, of which the listed ones are refined into
 * 2 block x 2 block fine cells of half the spacing.  The unknowns are the
 * leaf cells (base cells outside refined blocks, all fine cells).  The
 * paper does not give the discretisation at a block edge; here:
 * - D on each level from that level's view of E, rho, kappa: the fine
 *   level sees the fine cells where refined and each base value copied to
 *   its four fine cells elsewhere; the base level sees the base cells and,
 *   where refined, the mean of the four fine children; limiter, five-point
 *   gradient and walls as on a uniform grid of the level's spacing;
 * - faces between two leaf cells of one level as on a uniform grid;
 * - a face between a fine leaf cell f and a base leaf cell c: the flux
 *   between the two centres, 3/2 fine spacings apart, beta (x_f - x_c) with
 *   beta = (2/3) dt D_face / h_f^2 on the fine row, and beta / 4 (x_c -
 *   x_f) from each of the two fine cells along the face on the base row
 *   (conservative; the system is symmetric with volume weights).
 * The solve is flexible conjugate gradients in the volume-weighted product,
 * preconditioned by a two-level multigrid cycle (fine red-black
 * Gauss-Seidel sweeps, pre_smooth before and post_smooth after, at least
 * one each, around one V-cycle of the base grid's own multigrid); it stops
 * at |b - A x|_V / |b|_V <= rtol (volume-weighted 2-norms) or after
 * max_cycles iterations.
 * params: ndim 2, precision FP64, guess E^n or zero, krylov 0, periodic or
 * zero-gradient walls, n[0] and n[1] >= 4 and multiples of block (>= 2).
 * blocks_xy: host array of nblocks (bx, by) pairs (block coordinates, x
 * first), distinct, inside the base grid; refined block k holds fine
 * cells k * (2 block)^2 ... in the fine arrays, row-major (y, x) inside.
 * Base arrays: n[0] * n[1] doubles, x fastest (the values of cells under
 * refined blocks are not read; on output they hold the mean of their four
 * fine children).  Fine arrays: nblocks * (2 block)^2 doubles.  All device
 * pointers; E_*_out may equal E_*_in.  Workspace: device memory of
 * fld_amr_workspace_bytes (0 for invalid arguments), 256-byte aligned,
 * owned by the caller.  fld_amr_step blocks until the solve ends (the
 * Krylov scalars stay on the device; the host reads the residual once per
 * iteration for the stop test); stats as fld_step's (cycles and
 * outer_iters: iterations).  Errors: FLD_ERR_INVALID_ARG, FLD_ERR_WORKSPACE,
 * FLD_ERR_NONPHYSICAL, FLD_ERR_NOT_CONVERGED (last iterate returned),
 * FLD_ERR_DEVICE; the message is read by fld_amr_last_error. */
typedef struct fld_amr_ctx fld_amr_ctx;

size_t fld_amr_workspace_bytes(const fld_params* p, int32_t block,
                               const int32_t* blocks_xy, int32_t nblocks);
fld_status fld_amr_setup(const fld_params* p, int32_t block,
                         const int32_t* blocks_xy, int32_t nblocks,
                         void* workspace, size_t ws_bytes, void* hip_stream,
                         fld_amr_ctx** out);
fld_status fld_amr_step(fld_amr_ctx* ctx, double dt, const double* rho_base,
                        const double* kappa_base, const double* E_base_in,
                        double* E_base_out, const double* rho_fine,
                        const double* kappa_fine, const double* E_fine_in,
                        double* E_fine_out, fld_stats* stats);
/* fld_exchange and fld_opacity_powerlaw on a block-adaptive grid: both are
 * per cell, so they run over the base array (every cell, covered ones
 * included) and over the fine array, with the context's constants.  Same
 * layouts as fld_amr_step; asynchronous (stream-ordered); the same
 * argument errors as the single-grid calls. */
fld_status fld_amr_exchange(fld_amr_ctx* ctx, double dt,
                            const double* rho_base, const double* kappa_base,
                            double* E_base, double* e_base,
                            const double* rho_fine, const double* kappa_fine,
                            double* E_fine, double* e_fine);
fld_status fld_amr_opacity_powerlaw(fld_amr_ctx* ctx, const double* rho_base,
                                    const double* e_base,
                                    const double* rho_fine,
                                    const double* e_fine, double k0, double a,
                                    double b, double kmin, double kmax,
                                    double* kappa_base, double* kappa_fine);
/* Kernel timing of the block-adaptive step: with `on`, every level-1
 * red-black half-sweep of a step (the step's dominant kernel) is
 * bracketed by events recorded by the launch; the read returns the summed
 * milliseconds, the launch count and the algorithmic bytes of those
 * launches (r and the four faces of half the fine cells and z of all of
 * them read, half of z written), then resets the counters. */
fld_status fld_amr_kernel_timing_enable(fld_amr_ctx* ctx, int32_t on);
fld_status fld_amr_kernel_timing_read(fld_amr_ctx* ctx, double* ms_total,
                                      int64_t* launches, double* bytes_total,
                                      const char** kernel_name);
/* Deeper hierarchies: nlevels (<= 4) refined levels.  Level l has spacing
 * dx / 2^l on a (n[0] << l) x (n[1] << l) lattice; each of its blocks
 * refines the block x block patch of level-(l-1) cells whose corner is
 * (bx block, by block) into 2 block x 2 block level-l cells.  nblocks:
 * host array of nlevels counts; blocks_xy: the (bx, by) of level 1's
 * blocks, then level 2's, ...  A level-l block (l >= 2) must lie inside a
 * level-(l-1) block, and so must the four patches sharing its faces (2:1
 * nesting: a leaf cell's face neighbour is of its own level or of the next
 * coarser one); walls end that condition.  The fine arrays hold level 1's
 * blocks, then level 2's, ..., (2 block)^2 doubles each; the cells under
 * finer blocks are not read, and on output hold the mean of their four
 * children.  Same readings and solve as one level; the preconditioner
 * cycles through the levels: from the finest down, red-black sweeps of
 * each level's own correction problem over all of its cells (the coarser
 * correction held outside its blocks), then that level's residual,
 * averaged onto the cells under its blocks, plus the fluxes of its
 * correction into the coarser leaf cells beside them, as the next coarser
 * level's right-hand side; the base V-cycle; then from level 1 up,
 * bilinear prolongation of the coarser correction added to the level's
 * own and sweeps in reverse colour order.  fld_amr_setup and
 * fld_amr_workspace_bytes are the one-level case. */
size_t fld_amr_workspace_bytes_levels(const fld_params* p, int32_t block,
                                      int32_t nlevels, const int32_t* nblocks,
                                      const int32_t* blocks_xy);
fld_status fld_amr_setup_levels(const fld_params* p, int32_t block,
                                int32_t nlevels, const int32_t* nblocks,
                                const int32_t* blocks_xy, void* workspace,
                                size_t ws_bytes, void* hip_stream,
                                fld_amr_ctx** out);
/* Last error of a context, or with NULL of the last failed set-up. */
const char* fld_amr_last_error(const fld_amr_ctx* ctx);
void fld_amr_destroy(fld_amr_ctx* ctx);

/* Implicit gas-radiation exchange (eqs. heating, qdot) for one step dt:
 * per cell, with beta = dt c kappa rho and S = E + e_int,
 *   e' solves a4 e'^4 + (1 + beta) e' = e_int + beta S,
 *   a4 = beta a_rad ((gamma - 1) / (rho gas_const))^4,
 *   E' = S - e'  (e + E conserved per cell).
 * E: in E*, out E^{n+1}.  e_int: in e^n, out e^{n+1}.  Device pointers.
 * Asynchronous (stream-ordered).  FLD_ERR_INVALID_ARG for dt <= 0. */
fld_status fld_exchange(fld_ctx* ctx, double dt, const double* rho,
                        const double* kappa, double* E, double* e_int);

/* Explicit FLD source terms at cell centres (Sect. 3 adds them explicitly,
 * around the implicit update), from E and the gas velocity v:
 *   f_r    = rho kappa F / c = -lambda grad E   (eqs. rad_force, fld_F)
 *   work   = v . f_r                            (its work on the gas)
 *   tiring = P : grad v,  P = f E,  f_ij = (1 - f)/2 delta_ij
 *            + (3 f - 1)/2 n_i n_j,  n = grad E / |grad E|  (0 where
 *            grad E = 0),  f = lambda + lambda^2 R^2
 *            (eqs. fld_P, fld_Eddington_tensor, fld_f)
 *   fedd   = f, the scalar Eddington factor.
 * grad E and grad v by the context's five-point stencil and ghost cells
 * (periodic wrap, Neumann mirror ghosts for E and every velocity component),
 * R = |grad E| / (rho kappa E) and lambda the context's limiter, as in
 * fld_step.  Only derivatives along the grid's ndim dimensions exist.
 * rho, kappa, E: device fields.  v: HOST array of ndim DEVICE pointers
 * (v_x, v_y, v_z), or NULL when neither work nor tiring is asked for.
 * f_r: HOST array of ndim DEVICE output pointers, or NULL; work, tiring,
 * fedd: DEVICE outputs, each nullable.  A caller advancing the split step
 * adds -dt tiring to E, dt f_r to the momentum and dt work to the gas
 * energy.  Outputs are unspecified for cells with E <= 0 or rho kappa <= 0.
 * Asynchronous (stream-ordered); FLD_ERR_INVALID_ARG for a NULL input, for
 * work or tiring without v, or for a batched context. */
fld_status fld_explicit_sources(fld_ctx* ctx, const double* rho,
                                const double* kappa, const double* E,
                                const double* const* v, double* const* f_r,
                                double* work, double* tiring, double* fedd);

/* Opacity power law of the synthetic workloads (not the paper's constant
 * opacity): kappa = clip(k0 rho^a T^b, kmin, kmax) with
 * T = (gamma - 1) e_int / (rho gas_const).  Device pointers; asynchronous. */
fld_status fld_opacity_powerlaw(fld_ctx* ctx, const double* rho,
                                const double* e_int, double k0, double a,
                                double b, double kmin, double kmax,
                                double* kappa);

/* Per-launch timing of the dominant kernel (the finest-level smoother).
 * When enabled, every launch of that kernel is bracketed by HIP events on
 * the context's stream; fld_kernel_timing_read returns the summed
 * milliseconds, the launch count and the algorithmic bytes those launches
 * stream (each operand read or written once), then resets the counters. */
fld_status fld_kernel_timing_enable(fld_ctx* ctx, int32_t on);
fld_status fld_kernel_timing_read(fld_ctx* ctx, double* ms_total,
                                  int64_t* launches, double* bytes_total,
                                  const char** kernel_name);

/* Autotuner of the 2D tiled multigrid kernels: times every tile shape of
 * the down (pre-smoothing, residual, restriction) and up (prolongation,
 * post-smoothing) passes on each tiled level of this context and keeps the
 * fastest per level and pass; a batched context is tuned on its largest
 * grid, one shape per level index for all grids.  Untuned contexts use
 * shape 0.  The shapes change only the speed, never the result.  Uses the
 * context's workspace as scratch: call it between steps.  Blocks.  choices
 * (host, nullable): 2 * max_levels int32, the chosen shape per level (down,
 * up).  Contexts without tiled levels (1D, 3D) tune nothing. */
fld_status fld_autotune(fld_ctx* ctx, int32_t* choices, int32_t max_levels);
/* Name of a tile shape ("64x48/256": region and threads per block). */
const char* fld_tile_shape_name(int32_t variant);

/* ---- Batched grids ---------------------------------------------------------
 * Many independent 2D grids (each with its own size, boundaries, constants
 * and dt) advanced together: every phase of the step above is one launch
 * over all grids, so the launch count does not grow with the number of
 * grids.  Each grid gets the same result as fld_step / fld_exchange /
 * fld_opacity_powerlaw on its own (same operator, same stop test on its own
 * residual); grids that have converged skip their share of later launches.
 * Restrictions (FLD_ERR_INVALID_ARG otherwise): ndim == 2, one precision and
 * one set of smoothing counts (finest and coarse, each 1..3) for all grids,
 * guess E^n, and every
 * grid coarsenable to at most 1024 cells but larger than that itself.
 * Pointer arrays (const double* const* ...) are HOST arrays of `count`
 * DEVICE pointers. */

/* Workspace bytes for fld_setup_batch (0 if the parameters are invalid). */
size_t fld_workspace_bytes_batch(int32_t count, const fld_params* each);

/* Set up `count` grids in one workspace; *out is a batched context. */
fld_status fld_setup_batch(int32_t count, const fld_params* each,
                           void* workspace, size_t ws_bytes, void* hip_stream,
                           fld_ctx** out);

/* fld_step for every grid g with dt[g] (host array).  stats: host array of
 * `count` entries, or NULL.  Blocks until every grid has stopped.  Returns
 * FLD_OK if all converged, else the worst status (NONPHYSICAL before
 * NOT_CONVERGED); fld_last_error names the grid. */
fld_status fld_step_batch(fld_ctx* ctx, const double* dt,
                          const double* const* rho, const double* const* kappa,
                          const double* const* E_in, double* const* E_out,
                          fld_stats* stats);

/* fld_exchange for every grid (one launch).  Waits for earlier work on the
 * stream before it stages its argument table. */
fld_status fld_exchange_batch(fld_ctx* ctx, const double* dt,
                              const double* const* rho,
                              const double* const* kappa, double* const* E,
                              double* const* e_int);

/* fld_opacity_powerlaw for every grid (one launch); same staging rule. */
fld_status fld_opacity_powerlaw_batch(fld_ctx* ctx, const double* const* rho,
                                      const double* const* e_int, double k0,
                                      double a, double b, double kmin,
                                      double kmax, double* const* kappa);

/* on != 0: capture the launches of one batch of iterations into a hipGraph
 * once and replay it in later steps (argument tables stay at fixed device
 * addresses, so new field pointers do not invalidate it).  Needs a
 * non-default stream (FLD_ERR_INVALID_ARG for the null stream). */
fld_status fld_batch_set_graph(fld_ctx* ctx, int32_t on);

/* Release the context (host memory only; the workspace is the caller's). */
void fld_destroy(fld_ctx* ctx);

const char* fld_status_str(int32_t status);
const char* fld_last_error(const fld_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* FLD_H */
