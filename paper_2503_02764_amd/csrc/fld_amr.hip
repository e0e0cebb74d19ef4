// Kernels of the block-adaptive 2D step (fld_amr.cpp): a base grid and up
// to kAmrMaxLevels levels of refined blocks, the backward-Euler diffusion
// of eq. mhd_r_e on the leaf cells (Sect. 3 solves it by multigrid on
// MPI-AMRVAC's block-adaptive grids).
//
// Vectors of leaf values are one array: the base grid's nx*ny cells, then
// the blocks of level 1, of level 2, ..., each S x S = 2b x 2b cells,
// row-major; the entries of cells under finer blocks are held at 0.  Level
// l's cells sit on a (nx << l) x (ny << l) lattice; a level-l value at a
// lattice point outside level l's blocks is the next coarser level's value
// at the point's parent (the level's view of the coarser grid).  The 2:1
// nesting checked on the host makes a leaf cell's face neighbour a cell of
// its own level or a leaf cell of the next coarser level.  One thread per
// cell; the tables (block of each b-cell unit of a level's parent lattice,
// corner of each block) come from the host.
#include <hip/hip_ext.h>

#include "fld_amr.h"
#include "fld_device.h"

namespace fld {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ int amr_wrap(int i, int n, int per) {
  // periodic wrap, or the mirror ghosts of a zero-gradient wall (-1 -> 0,
  // -2 -> 1); a stencil reaches at most two cells, and n >= 2
  if (i < 0) return per ? i + n : -1 - i;
  if (i >= n) return per ? i - n : 2 * n - 1 - i;
  return i;
}

// block of level l >= 1 holding lattice point (I, J) of level l, or -1
__device__ __forceinline__ int amr_blk(const AmrGeom& G, int l, int I, int J) {
  const int pi = I >> 1, pj = J >> 1;
  return G.bmap[l - 1][(pj / G.b) * G.units_x[l - 1] + pi / G.b];
}

// fine-part index of lattice point (I, J) of level l in block blk
__device__ __forceinline__ int64_t amr_fidx(const AmrGeom& G, int l, int blk,
                                            int I, int J) {
  const int bx = G.bxy[l - 1][2 * blk], by = G.bxy[l - 1][2 * blk + 1];
  return G.off[l - 1] + ((int64_t)blk * G.S + (J - G.S * by)) * G.S +
         (I - G.S * bx);
}

// level-l view of a field at lattice point (I, J) (inside the lattice)
__device__ __forceinline__ double amr_val(const AmrGeom& G, int l,
                                          const double* vb, const double* vf,
                                          int I, int J) {
  while (l > 0) {
    const int blk = amr_blk(G, l, I, J);
    if (blk >= 0) return vf[amr_fidx(G, l, blk, I, J)];
    I >>= 1;
    J >>= 1;
    --l;
  }
  return vb[(int64_t)J * G.nx + I];
}

// the value of the leaf cell of level l under lattice point (I, J), which
// 2:1 nesting places on level l itself (l = 0: the base)
__device__ __forceinline__ double amr_val_at(const AmrGeom& G, int l,
                                             const double* vb,
                                             const double* vf, int I, int J) {
  if (l == 0) return vb[(int64_t)J * G.nx + I];
  return vf[amr_fidx(G, l, amr_blk(G, l, I, J), I, J)];
}

// a cell of level l (inside l's blocks) lies under a level-(l+1) block
__device__ __forceinline__ bool amr_covered(const AmrGeom& G, int l, int I,
                                            int J) {
  if (l >= G.L) return false;
  return G.bmap[l][(J / G.b) * G.units_x[l] + I / G.b] >= 0;
}

__device__ __forceinline__ double amr_mean(double a, double b, int kind) {
  return kind == 0 ? 0.5 * (a + b) : 2.0 * a * b / (a + b);
}

// a fine cell from its fine-part index
struct AmrCell {
  int l, blk, I, J;
};

__device__ __forceinline__ AmrCell amr_cell(const AmrGeom& G, int64_t f) {
  AmrCell c;
  c.l = 1;
  while (c.l < G.L && f >= G.off[c.l]) ++c.l;
  const int64_t loc = f - G.off[c.l - 1];
  const int64_t ss = (int64_t)G.S * G.S;
  c.blk = (int)(loc / ss);
  const int in = (int)(loc % ss);
  c.I = G.S * G.bxy[c.l - 1][2 * c.blk] + in % G.S;
  c.J = G.S * G.bxy[c.l - 1][2 * c.blk + 1] + in / G.S;
  return c;
}

__device__ __forceinline__ double amr_weight(const AmrGeom& G, int64_t t) {
  if (t < G.Nb) return G.vb;
  const AmrCell c = amr_cell(G, t - G.Nb);
  return G.vb / (double)(1 << (2 * c.l));
}

// The couplings of a leaf cell (level l, lattice (I, J); fine index f, or
// -1 on the base) in direction k (0 -x, 1 +x, 2 -y, 3 +y): its row gains
// sum w (x_cell - x_nb); adds sum w to ws and sum w x_nb to wx.
//  - neighbour of the same level and a leaf: alpha (base: the base faces,
//    owned by the lower cell; fine: this cell's face k);
//  - neighbour of the same level under finer blocks: the two finer cells
//    along the face, beta / 4 each (their faces pointing back);
//  - neighbour outside the level's blocks: the coarser leaf cell, beta
//    (this cell's face k).
__device__ __forceinline__ void amr_couple(
    const AmrGeom& G, const double* __restrict__ ax,
    const double* __restrict__ ay, const double* __restrict__ cf,
    const double* __restrict__ xb, const double* __restrict__ xf, int l,
    int64_t f, int I, int J, int k, double& ws, double& wx) {
  const int d = k >> 1, s = (k & 1) ? 1 : -1;
  const int NX = G.nx << l, NY = G.ny << l;
  int II = I + (d == 0 ? s : 0), JJ = J + (d == 1 ? s : 0);
  const int cc = d == 0 ? II : JJ, n = d == 0 ? NX : NY;
  if ((cc < 0 || cc >= n) && !G.per[d]) return;  // wall
  II = amr_wrap(II, NX, 1);
  JJ = amr_wrap(JJ, NY, 1);
  const int nb = l == 0 ? 0 : amr_blk(G, l, II, JJ);
  if (nb < 0) {  // the coarser leaf cell
    const double w = cf[(int64_t)k * G.Nf + f];
    ws += w;
    wx += w * amr_val_at(G, l - 1, xb, xf, II >> 1, JJ >> 1);
    return;
  }
  if (amr_covered(G, l, II, JJ)) {  // the finer cells along the face
    const int back = k ^ 1;
    for (int q = 0; q < 2; ++q) {
      const int I2 = d == 0 ? (s > 0 ? 2 * II : 2 * II + 1) : 2 * II + q;
      const int J2 = d == 0 ? 2 * JJ + q : (s > 0 ? 2 * JJ : 2 * JJ + 1);
      const int b2 = amr_blk(G, l + 1, I2, J2);
      const int64_t f2 = amr_fidx(G, l + 1, b2, I2, J2);
      const double w = 0.25 * cf[(int64_t)back * G.Nf + f2];
      ws += w;
      wx += w * xf[f2];
    }
    return;
  }
  double w, xn;
  if (l == 0) {
    const int64_t self = (int64_t)J * G.nx + I;
    const int64_t other = (int64_t)JJ * G.nx + II;
    w = (d == 0 ? ax : ay)[s > 0 ? self : other];
    xn = xb[other];
  } else {
    w = cf[(int64_t)k * G.Nf + f];
    xn = xf[amr_fidx(G, l, nb, II, JJ)];
  }
  ws += w;
  wx += w * xn;
}

// The four directions of a fine leaf cell (level l, block-local (lx, ly)):
// a neighbour inside the same block and not under finer blocks by offset,
// the others through amr_couple.
__device__ __forceinline__ void amr_couple_fine(
    const AmrGeom& G, const double* __restrict__ cf,
    const double* __restrict__ xb, const double* __restrict__ xf,
    const AmrCell& c, int64_t f, int lx, int ly, double& ws, double& wx) {
  const bool top = c.l >= G.L;  // no finer level: no covered neighbour
  for (int k = 0; k < 4; ++k) {
    const double a = cf[(int64_t)k * G.Nf + f];
    if (a == 0.0) continue;  // a wall (faces are positive otherwise)
    const int d = k >> 1, s = (k & 1) ? 1 : -1;
    const int ln = d == 0 ? lx + s : ly + s;
    if (ln >= 0 && ln < G.S) {
      const int64_t fn = f + (d == 0 ? s : s * G.S);
      if (top || !amr_covered(G, c.l, c.I + (d == 0 ? s : 0),
                              c.J + (d == 1 ? s : 0))) {
        ws += a;
        wx += a * xf[fn];
        continue;
      }
    }
    amr_couple(G, nullptr, nullptr, cf, xb, xf, c.l, f, c.I, c.J, k, ws, wx);
  }
}

// ---- views and coefficients ----

// cells of level l: copies of the inputs, or under finer blocks the mean of
// their four children's views
__global__ void __launch_bounds__(kT)
    k_amr_fine_views(AmrGeom G, int l, const double* __restrict__ Ef,
                     const double* __restrict__ rf,
                     const double* __restrict__ kf, double* __restrict__ Evf,
                     double* __restrict__ rvf, double* __restrict__ kvf) {
  const int64_t f = G.off[l - 1] + (int64_t)blockIdx.x * kT + threadIdx.x;
  if (f >= G.off[l]) return;
  const AmrCell c = amr_cell(G, f);
  const double* src[3] = {Ef, rf, kf};
  double* dst[3] = {Evf, rvf, kvf};
  if (!amr_covered(G, l, c.I, c.J)) {
    for (int k = 0; k < 3; ++k) dst[k][f] = src[k][f];
    return;
  }
  double acc[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < 4; ++q) {
    const int I2 = 2 * c.I + (q & 1), J2 = 2 * c.J + (q >> 1);
    const int64_t f2 = amr_fidx(G, l + 1, amr_blk(G, l + 1, I2, J2), I2, J2);
    for (int k = 0; k < 3; ++k) acc[k] += dst[k][f2];
  }
  for (int k = 0; k < 3; ++k) dst[k][f] = 0.25 * acc[k];
}

__global__ void __launch_bounds__(kT)
    k_amr_base_views(AmrGeom G, const double* __restrict__ Eb,
                     const double* __restrict__ rb,
                     const double* __restrict__ kb,
                     const double* __restrict__ Evf,
                     const double* __restrict__ rvf,
                     const double* __restrict__ kvf, double* __restrict__ Ev,
                     double* __restrict__ rv, double* __restrict__ kv) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c >= G.Nb) return;
  const int i = (int)(c % G.nx), j = (int)(c / G.nx);
  if (!amr_covered(G, 0, i, j)) {
    Ev[c] = Eb[c];
    rv[c] = rb[c];
    kv[c] = kb[c];
    return;
  }
  const double* src[3] = {Evf, rvf, kvf};
  double* dst[3] = {Ev, rv, kv};
  double acc[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < 4; ++q) {
    const int I2 = 2 * i + (q & 1), J2 = 2 * j + (q >> 1);
    const int64_t f2 = amr_fidx(G, 1, amr_blk(G, 1, I2, J2), I2, J2);
    for (int k = 0; k < 3; ++k) acc[k] += src[k][f2];
  }
  for (int k = 0; k < 3; ++k) dst[k][c] = 0.25 * acc[k];
}

// D = c lambda(R) / (rho kappa), R = |grad E| / (rho kappa E), from the
// five-point gradient of four stencil values per axis
__device__ __forceinline__ double amr_D(const AmrPhys& P, double E0,
                                        double rk, const double ex[4],
                                        const double ey[4], double hx,
                                        double hy) {
  const double gx = (ex[0] - 8.0 * ex[1] + 8.0 * ex[2] - ex[3]) / (12.0 * hx);
  const double gy = (ey[0] - 8.0 * ey[1] + 8.0 * ey[2] - ey[3]) / (12.0 * hy);
  const double R = sqrt(gx * gx + gy * gy) / (rk * E0);
  return P.c * flux_limiter(P.limiter, R) / rk;
}

__device__ __forceinline__ bool amr_bad(double E0, double rk) {
  return !(E0 > 0.0) || !(rk > 0.0) || !isfinite(E0) || !isfinite(rk);
}

__global__ void __launch_bounds__(kT)
    k_amr_dbase(AmrGeom G, AmrPhys P, const double* __restrict__ Ev,
                const double* __restrict__ rv, const double* __restrict__ kv,
                double* __restrict__ Db, int* __restrict__ bad) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c >= G.Nb) return;
  const int i = (int)(c % G.nx), j = (int)(c / G.nx);
  double ex[4], ey[4];
  const int o[4] = {-2, -1, 1, 2};
  for (int k = 0; k < 4; ++k) {
    ex[k] = Ev[(int64_t)j * G.nx + amr_wrap(i + o[k], G.nx, G.per[0])];
    ey[k] = Ev[(int64_t)amr_wrap(j + o[k], G.ny, G.per[1]) * G.nx + i];
  }
  const double E0 = Ev[c], rk = rv[c] * kv[c];
  if (amr_bad(E0, rk)) atomicAdd(bad, 1);
  Db[c] = amr_D(P, E0, rk, ex, ey, G.dx, G.dy);
}

__global__ void __launch_bounds__(kT)
    k_amr_dfine(AmrGeom G, AmrPhys P, const double* __restrict__ Ev,
                const double* __restrict__ Evf, const double* __restrict__ rvf,
                const double* __restrict__ kvf, double* __restrict__ Df,
                int* __restrict__ bad) {
  const int64_t f = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (f >= G.Nf) return;
  const AmrCell c = amr_cell(G, f);
  const int NX = G.nx << c.l, NY = G.ny << c.l;
  double ex[4], ey[4];
  const int o[4] = {-2, -1, 1, 2};
  for (int k = 0; k < 4; ++k) {
    ex[k] = amr_val(G, c.l, Ev, Evf, amr_wrap(c.I + o[k], NX, G.per[0]), c.J);
    ey[k] = amr_val(G, c.l, Ev, Evf, c.I, amr_wrap(c.J + o[k], NY, G.per[1]));
  }
  const double E0 = Evf[f], rk = rvf[f] * kvf[f];
  if (amr_bad(E0, rk)) atomicAdd(bad, 1);
  const double h = 1.0 / (double)(1 << c.l);
  Df[f] = amr_D(P, E0, rk, ex, ey, G.dx * h, G.dy * h);
}

// the four faces of every fine cell (0 -x, 1 +x, 2 -y, 3 +y): to a cell of
// the same level alpha = dt D_face / h^2, to a cell of the next coarser
// level beta = (2/3) dt D_face / h^2, 0 at a wall
__global__ void __launch_bounds__(kT)
    k_amr_faces(AmrGeom G, AmrPhys P, double dt,
                const double* __restrict__ Db, const double* __restrict__ Df,
                double* __restrict__ cf) {
  const int64_t f = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (f >= G.Nf) return;
  const AmrCell c = amr_cell(G, f);
  const int NX = G.nx << c.l, NY = G.ny << c.l;
  const double h = 1.0 / (double)(1 << c.l);
  for (int k = 0; k < 4; ++k) {
    const int d = k >> 1, s = (k & 1) ? 1 : -1;
    int II = c.I + (d == 0 ? s : 0), JJ = c.J + (d == 1 ? s : 0);
    const int n = d == 0 ? NX : NY, cc = d == 0 ? II : JJ;
    double a = 0.0;
    if ((cc >= 0 && cc < n) || G.per[d]) {
      II = amr_wrap(II, NX, 1);
      JJ = amr_wrap(JJ, NY, 1);
      const double hd = (d == 0 ? G.dx : G.dy) * h;
      const int nb = amr_blk(G, c.l, II, JJ);
      if (nb >= 0) {
        a = dt * amr_mean(Df[f], Df[amr_fidx(G, c.l, nb, II, JJ)],
                          P.face_mean) / (hd * hd);
      } else {
        const double Dc = amr_val(G, c.l - 1, Db, Df, II >> 1, JJ >> 1);
        a = (2.0 / 3.0) * dt * amr_mean(Df[f], Dc, P.face_mean) / (hd * hd);
      }
    }
    cf[(int64_t)k * G.Nf + f] = a;
  }
}

// ---- operator, smoothing, transfers ----

__device__ __forceinline__ double amr_apply_cell(
    const AmrGeom& G, const double* __restrict__ ax,
    const double* __restrict__ ay, const double* __restrict__ cf,
    const double* __restrict__ x, int64_t t) {
  const double* xf = x + G.Nb;
  int l, I, J;
  int64_t f = -1;
  if (t < G.Nb) {
    l = 0;
    I = (int)(t % G.nx);
    J = (int)(t / G.nx);
  } else {
    f = t - G.Nb;
    const AmrCell c = amr_cell(G, f);
    l = c.l;
    I = c.I;
    J = c.J;
  }
  if (amr_covered(G, l, I, J)) return 0.0;
  double ws = 0.0, wx = 0.0;
  if (l == 0) {
    for (int k = 0; k < 4; ++k)
      amr_couple(G, ax, ay, cf, x, xf, 0, -1, I, J, k, ws, wx);
  } else {
    const AmrCell c = {l, 0, I, J};
    amr_couple_fine(G, cf, x, xf, c, f, I % G.S, J % G.S, ws, wx);
  }
  return x[t] * (1.0 + ws) - wx;
}

// y = A x; with `partials`, also the per-block sums of the volume-weighted
// r . x (row 0) and x . y (row 1)
__global__ void __launch_bounds__(kT)
    k_amr_apply(AmrGeom G, const double* __restrict__ ax,
                const double* __restrict__ ay, const double* __restrict__ cf,
                const double* __restrict__ x, double* __restrict__ y,
                const double* __restrict__ r, double* __restrict__ partials) {
  __shared__ double sh[kT / 64];
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  double rx = 0.0, xy = 0.0;
  if (t < G.Nb + G.Nf) {
    const double v = amr_apply_cell(G, ax, ay, cf, x, t);
    y[t] = v;
    if (partials) {
      const double w = amr_weight(G, t);
      rx = w * r[t] * x[t];
      xy = w * x[t] * v;
    }
  }
  if (!partials) return;
  const double s0 = block_sum<kT>(rx, sh);
  __syncthreads();
  const double s1 = block_sum<kT>(xy, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = s0;
    partials[gridDim.x + blockIdx.x] = s1;
  }
}

// The couplings of a cell of level l (any of its cells, under finer blocks
// or not) in the level's own operator: same-level neighbours by alpha, the
// next coarser level's cell outside the level's blocks by beta; adds sum w
// to ws and sum w e_nb to wx.
__device__ __forceinline__ void amr_couple_level(
    const AmrGeom& G, const double* __restrict__ cf,
    const double* __restrict__ eb, const double* __restrict__ ef, int l,
    int64_t f, int lx, int ly, int I, int J, double& ws, double& wx) {
  const int NX = G.nx << l, NY = G.ny << l;
  for (int k = 0; k < 4; ++k) {
    const double a = cf[(int64_t)k * G.Nf + f];
    if (a == 0.0) continue;  // a wall
    const int d = k >> 1, s = (k & 1) ? 1 : -1;
    const int ln = d == 0 ? lx + s : ly + s;
    double v;
    if (ln >= 0 && ln < G.S) {
      v = ef[f + (d == 0 ? s : s * G.S)];
    } else {
      const int II = amr_wrap(I + (d == 0 ? s : 0), NX, 1);
      const int JJ = amr_wrap(J + (d == 1 ? s : 0), NY, 1);
      const int nb = amr_blk(G, l, II, JJ);
      v = nb >= 0 ? ef[amr_fidx(G, l, nb, II, JJ)]
                  : amr_val_at(G, l - 1, eb, ef, II >> 1, JJ >> 1);
    }
    ws += a;
    wx += a * v;
  }
}

__device__ __forceinline__ AmrCell amr_level_cell(const AmrGeom& G, int l,
                                                  int64_t loc, int& lx,
                                                  int& ly) {
  const int in = (int)(loc % ((int64_t)G.S * G.S));
  lx = in % G.S;
  ly = in / G.S;
  const int blk = (int)(loc / ((int64_t)G.S * G.S));
  const AmrCell c = {l, blk, G.S * G.bxy[l - 1][2 * blk] + lx,
                     G.S * G.bxy[l - 1][2 * blk + 1] + ly};
  return c;
}

// one colour ((I + J) & 1) of a Gauss-Seidel sweep over every cell of
// level l for the level's correction e (L_l e = g), the coarser level's e
// fixed outside the level's blocks
__global__ void __launch_bounds__(kT)
    k_amr_smooth_level(AmrGeom G, int l, const double* __restrict__ cf,
                       const double* __restrict__ g, double* __restrict__ e,
                       int colour) {
  const int64_t loc = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t f = G.off[l - 1] + loc;
  if (f >= G.off[l]) return;
  int lx, ly;
  const int in = (int)(loc % ((int64_t)G.S * G.S));
  if ((((in % G.S) + (in / G.S)) & 1) != colour) return;  // S is even
  const AmrCell c = amr_level_cell(G, l, loc, lx, ly);
  double ws = 0.0, wx = 0.0;
  amr_couple_level(G, cf, e, e + G.Nb, l, f, lx, ly, c.I, c.J, ws, wx);
  e[G.Nb + f] = (g[G.Nb + f] + wx) / (1.0 + ws);
}

// t = g - L_l e on every cell of level l
__global__ void __launch_bounds__(kT)
    k_amr_resid_level(AmrGeom G, int l, const double* __restrict__ cf,
                      const double* __restrict__ g,
                      const double* __restrict__ e, double* __restrict__ t) {
  const int64_t loc = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t f = G.off[l - 1] + loc;
  if (f >= G.off[l]) return;
  int lx, ly;
  const AmrCell c = amr_level_cell(G, l, loc, lx, ly);
  double ws = 0.0, wx = 0.0;
  amr_couple_level(G, cf, e, e + G.Nb, l, f, lx, ly, c.I, c.J, ws, wx);
  t[G.Nb + f] = g[G.Nb + f] - (e[G.Nb + f] * (1.0 + ws) - wx);
}

// The right-hand side of level l (the base for l = 0) after level l + 1's
// smoothing: a cell under level-(l+1) blocks takes the mean of its
// children's residuals t; a leaf cell next to level-(l+1) cells adds the
// flux of their correction e into it (beta / 4 e_f per finer cell).
__device__ __forceinline__ void amr_coarse_rhs_cell(
    const AmrGeom& G, int l, int64_t t_idx, int I, int J,
    const double* __restrict__ cf, const double* __restrict__ e,
    const double* __restrict__ t, double* __restrict__ g) {
  const double* ef = e + G.Nb;
  if (amr_covered(G, l, I, J)) {
    double acc = 0.0;
    for (int q = 0; q < 4; ++q) {
      const int I2 = 2 * I + (q & 1), J2 = 2 * J + (q >> 1);
      acc += t[G.Nb + amr_fidx(G, l + 1, amr_blk(G, l + 1, I2, J2), I2, J2)];
    }
    g[t_idx] = 0.25 * acc;
    return;
  }
  const int NX = G.nx << l, NY = G.ny << l;
  double add = 0.0;
  for (int k = 0; k < 4; ++k) {
    const int d = k >> 1, s = (k & 1) ? 1 : -1;
    int II = I + (d == 0 ? s : 0), JJ = J + (d == 1 ? s : 0);
    const int cc = d == 0 ? II : JJ, n = d == 0 ? NX : NY;
    if ((cc < 0 || cc >= n) && !G.per[d]) continue;
    II = amr_wrap(II, NX, 1);
    JJ = amr_wrap(JJ, NY, 1);
    if (l > 0 && amr_blk(G, l, II, JJ) < 0) continue;  // coarser side
    if (!amr_covered(G, l, II, JJ)) continue;
    const int back = k ^ 1;
    for (int q = 0; q < 2; ++q) {
      const int I2 = d == 0 ? (s > 0 ? 2 * II : 2 * II + 1) : 2 * II + q;
      const int J2 = d == 0 ? 2 * JJ + q : (s > 0 ? 2 * JJ : 2 * JJ + 1);
      const int64_t f2 =
          amr_fidx(G, l + 1, amr_blk(G, l + 1, I2, J2), I2, J2);
      add += 0.25 * cf[(int64_t)back * G.Nf + f2] * ef[f2];
    }
  }
  g[t_idx] += add;
}

__global__ void __launch_bounds__(kT)
    k_amr_coarse_rhs(AmrGeom G, int l, const double* __restrict__ cf,
                     const double* __restrict__ e,
                     const double* __restrict__ t, double* __restrict__ g) {
  const int64_t loc = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (l == 0) {
    if (loc >= G.Nb) return;
    amr_coarse_rhs_cell(G, 0, loc, (int)(loc % G.nx), (int)(loc / G.nx), cf,
                        e, t, g);
    return;
  }
  const int64_t f = G.off[l - 1] + loc;
  if (f >= G.off[l]) return;
  int lx, ly;
  const AmrCell c = amr_level_cell(G, l, loc, lx, ly);
  amr_coarse_rhs_cell(G, l, G.Nb + f, c.I, c.J, cf, e, t, g);
}

// cells of level l under finer blocks: the mean of their four children
__global__ void __launch_bounds__(kT)
    k_amr_restrict_level(AmrGeom G, int l, double* __restrict__ v) {
  const int64_t f = G.off[l - 1] + (int64_t)blockIdx.x * kT + threadIdx.x;
  if (f >= G.off[l]) return;
  const AmrCell c = amr_cell(G, f);
  if (!amr_covered(G, l, c.I, c.J)) return;
  const double* vf = v + G.Nb;
  double acc = 0.0;
  for (int q = 0; q < 4; ++q) {
    const int I2 = 2 * c.I + (q & 1), J2 = 2 * c.J + (q >> 1);
    acc += vf[amr_fidx(G, l + 1, amr_blk(G, l + 1, I2, J2), I2, J2)];
  }
  v[G.Nb + f] = 0.25 * acc;
}

// e of every cell of level l += bilinear from the parent cell and its
// neighbours towards the cell (weights 9, 3, 3, 1 over 16), on the level
// below (its view of e)
__global__ void __launch_bounds__(kT)
    k_amr_prolong_level(AmrGeom G, int l, double* __restrict__ e) {
  const int64_t f = G.off[l - 1] + (int64_t)blockIdx.x * kT + threadIdx.x;
  if (f >= G.off[l]) return;
  const AmrCell c = amr_cell(G, f);
  const int NX = G.nx << (l - 1), NY = G.ny << (l - 1);
  const int i = c.I >> 1, j = c.J >> 1;
  const int i2 = amr_wrap(i + ((c.I & 1) ? 1 : -1), NX, G.per[0]);
  const int j2 = amr_wrap(j + ((c.J & 1) ? 1 : -1), NY, G.per[1]);
  const double* ef = e + G.Nb;
  const double v = (9.0 * amr_val(G, l - 1, e, ef, i, j) +
                    3.0 * amr_val(G, l - 1, e, ef, i2, j) +
                    3.0 * amr_val(G, l - 1, e, ef, i, j2) +
                    amr_val(G, l - 1, e, ef, i2, j2)) / 16.0;
  e[G.Nb + f] += v;
}

// entries of cells under finer blocks back to 0
__global__ void __launch_bounds__(kT)
    k_amr_zero_covered(AmrGeom G, double* __restrict__ v) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t >= G.Nb + G.Nf) return;
  bool cov;
  if (t < G.Nb) {
    cov = amr_covered(G, 0, (int)(t % G.nx), (int)(t / G.nx));
  } else {
    const AmrCell c = amr_cell(G, t - G.Nb);
    cov = amr_covered(G, c.l, c.I, c.J);
  }
  if (cov) v[t] = 0.0;
}

// leaf vector from (base, fine) arrays, covered entries 0
__global__ void __launch_bounds__(kT)
    k_amr_pack(AmrGeom G, const double* __restrict__ vb,
               const double* __restrict__ vf, double* __restrict__ v) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t >= G.Nb + G.Nf) return;
  if (t < G.Nb) {
    v[t] = amr_covered(G, 0, (int)(t % G.nx), (int)(t / G.nx)) ? 0.0 : vb[t];
  } else {
    const AmrCell c = amr_cell(G, t - G.Nb);
    v[t] = amr_covered(G, c.l, c.I, c.J) ? 0.0 : vf[t - G.Nb];
  }
}

// (base, fine) arrays from a vector whose covered fine entries already
// hold their children's means: a covered base cell gets the mean of its
// level-1 children
__global__ void __launch_bounds__(kT)
    k_amr_unpack(AmrGeom G, const double* __restrict__ v,
                 double* __restrict__ vb, double* __restrict__ vf) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t < G.Nb) {
    const int i = (int)(t % G.nx), j = (int)(t / G.nx);
    if (!amr_covered(G, 0, i, j)) {
      vb[t] = v[t];
    } else {
      double acc = 0.0;
      for (int q = 0; q < 4; ++q) {
        const int I2 = 2 * i + (q & 1), J2 = 2 * j + (q >> 1);
        acc += v[G.Nb + amr_fidx(G, 1, amr_blk(G, 1, I2, J2), I2, J2)];
      }
      vb[t] = 0.25 * acc;
    }
  } else if (t < G.Nb + G.Nf) {
    vf[t - G.Nb] = v[t];
  }
}

// y = x + a * p (one of x, y may alias)
__global__ void __launch_bounds__(kT)
    k_amr_axpy(int64_t n, double a, const double* __restrict__ p,
               const double* x, double* y) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t < n) y[t] = x[t] + a * p[t];
}

// per-block partial sums of the volume-weighted products u_k . v_k
// (k < D.n), partials[k * gridDim.x + block]
__global__ void __launch_bounds__(kT)
    k_amr_dots(AmrGeom G, AmrDots D, double* __restrict__ partials) {
  __shared__ double sh[kT / 64];
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  const bool in = t < G.Nb + G.Nf;
  const double w = in ? amr_weight(G, t) : 0.0;
  for (int k = 0; k < D.n; ++k) {
    const double s = in ? w * D.u[k][t] * D.v[k][t] : 0.0;
    const double tot = block_sum<kT>(s, sh);
    __syncthreads();  // sh is reused by the next sum
    if (threadIdx.x == 0) partials[(int64_t)k * gridDim.x + blockIdx.x] = tot;
  }
}

// Krylov scalars on the device: sc[0] (z, q_old), sc[1] (p_old, q_old),
// sc[2] (r, p), sc[3] (p, q), sc[4] (r, r).  One block sums rows of
// block partials in a fixed order into sc[slot ...]; with copy, sc[1] takes
// sc[3] first (this iteration's (p, q) is the next one's (p_old, q_old)).
constexpr int kRT = 1024;  // one wide block: few partials per thread
__global__ void __launch_bounds__(kRT)
    k_amr_reduce(const double* __restrict__ partials, int nb, int npair,
                 double* __restrict__ sc, int slot, int copy) {
  __shared__ double sh[kRT / 64];
  if (copy && threadIdx.x == 0) sc[1] = sc[3];
  for (int k = 0; k < npair; ++k) {
    const double* row = partials + (int64_t)k * nb;
    double v[4] = {0.0, 0.0, 0.0, 0.0};  // four loads in flight
    int i = threadIdx.x;
    for (; i + 3 * kRT < nb; i += 4 * kRT)
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] += row[i + u * kRT];
    for (; i < nb; i += kRT) v[0] += row[i];
    const double tot = block_sum<kRT>((v[0] + v[1]) + (v[2] + v[3]), sh);
    __syncthreads();
    if (threadIdx.x == 0) sc[slot + k] = tot;
  }
}

// p = z (first) or z - (sc[0] / sc[1]) p_old
__global__ void __launch_bounds__(kT)
    k_amr_dir(int64_t n, const double* __restrict__ z,
              const double* __restrict__ p_old, double* __restrict__ p,
              const double* __restrict__ sc, int first) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t >= n) return;
  p[t] = first ? z[t] : z[t] - (sc[0] / sc[1]) * p_old[t];
}

// x += a p, r -= a q with a = sc[2] / sc[3]; per-block sums of the
// volume-weighted r . r
__global__ void __launch_bounds__(kT)
    k_amr_update(AmrGeom G, const double* __restrict__ p,
                 const double* __restrict__ q, double* __restrict__ x,
                 double* __restrict__ r, const double* __restrict__ sc,
                 double* __restrict__ partials) {
  __shared__ double sh[kT / 64];
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  double rr = 0.0;
  if (t < G.Nb + G.Nf) {
    const double a = sc[2] / sc[3];
    x[t] += a * p[t];
    const double rv = r[t] - a * q[t];
    r[t] = rv;
    rr = amr_weight(G, t) * rv * rv;
  }
  const double tot = block_sum<kT>(rr, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

inline int nblk(int64_t n) { return (int)((n + kT - 1) / kT); }

inline int64_t level_cells(const AmrGeom& G, int l) {
  return G.off[l] - G.off[l - 1];
}

}  // namespace

hipError_t amr_views(const AmrGeom& G, const double* Eb, const double* rb,
                     const double* kb, const double* Ef, const double* rf,
                     const double* kf, double* Ev, double* rv, double* kv,
                     double* Evf, double* rvf, double* kvf, hipStream_t s) {
  for (int l = G.L; l >= 1; --l)  // finest first: children before parents
    if (level_cells(G, l) > 0)
      hipLaunchKernelGGL(k_amr_fine_views, dim3(nblk(level_cells(G, l))),
                         dim3(kT), 0, s, G, l, Ef, rf, kf, Evf, rvf, kvf);
  hipLaunchKernelGGL(k_amr_base_views, dim3(nblk(G.Nb)), dim3(kT), 0, s, G,
                     Eb, rb, kb, Evf, rvf, kvf, Ev, rv, kv);
  return hipGetLastError();
}

hipError_t amr_coefficients(const AmrGeom& G, const AmrPhys& P, double dt,
                            const double* Ev, const double* rv,
                            const double* kv, const double* Evf,
                            const double* rvf, const double* kvf, double* Db,
                            double* Df, double* cf, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_dbase, dim3(nblk(G.Nb)), dim3(kT), 0, s, G, P, Ev,
                     rv, kv, Db, bad);
  if (G.Nf > 0) {
    hipLaunchKernelGGL(k_amr_dfine, dim3(nblk(G.Nf)), dim3(kT), 0, s, G, P,
                       Ev, Evf, rvf, kvf, Df, bad);
    hipLaunchKernelGGL(k_amr_faces, dim3(nblk(G.Nf)), dim3(kT), 0, s, G, P,
                       dt, Db, Df, cf);
  }
  return hipGetLastError();
}

hipError_t amr_apply(const AmrGeom& G, const double* ax, const double* ay,
                     const double* cf, const double* x, double* y,
                     hipStream_t s, const double* r, double* partials) {
  hipLaunchKernelGGL(k_amr_apply, dim3(nblk(G.Nb + G.Nf)), dim3(kT), 0, s, G,
                     ax, ay, cf, x, y, r, partials);
  return hipGetLastError();
}

hipError_t amr_smooth_level(const AmrGeom& G, int level, const double* cf,
                            const double* g, double* e, int colour,
                            hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const int64_t n = level_cells(G, level);
  if (n == 0) return hipSuccess;
  if (ev0 && ev1)  // the launch records its own start and end
    hipExtLaunchKernelGGL(k_amr_smooth_level, dim3(nblk(n)), dim3(kT), 0, s,
                          ev0, ev1, 0, G, level, cf, g, e, colour);
  else
    hipLaunchKernelGGL(k_amr_smooth_level, dim3(nblk(n)), dim3(kT), 0, s, G,
                       level, cf, g, e, colour);
  return hipGetLastError();
}

hipError_t amr_resid_level(const AmrGeom& G, int level, const double* cf,
                           const double* g, const double* e, double* t,
                           hipStream_t s) {
  const int64_t n = level_cells(G, level);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_amr_resid_level, dim3(nblk(n)), dim3(kT), 0, s, G,
                     level, cf, g, e, t);
  return hipGetLastError();
}

hipError_t amr_coarse_rhs(const AmrGeom& G, int level, const double* cf,
                          const double* e, const double* t, double* g,
                          hipStream_t s) {
  const int64_t n = level == 0 ? G.Nb : level_cells(G, level);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_amr_coarse_rhs, dim3(nblk(n)), dim3(kT), 0, s, G,
                     level, cf, e, t, g);
  return hipGetLastError();
}

hipError_t amr_restrict_level(const AmrGeom& G, int level, double* v,
                              hipStream_t s) {
  const int64_t n = level_cells(G, level);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_amr_restrict_level, dim3(nblk(n)), dim3(kT), 0, s, G,
                     level, v);
  return hipGetLastError();
}

hipError_t amr_prolong_level(const AmrGeom& G, int level, double* e,
                             hipStream_t s) {
  const int64_t n = level_cells(G, level);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_amr_prolong_level, dim3(nblk(n)), dim3(kT), 0, s, G,
                     level, e);
  return hipGetLastError();
}

hipError_t amr_zero_covered(const AmrGeom& G, double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_zero_covered, dim3(nblk(G.Nb + G.Nf)), dim3(kT), 0,
                     s, G, v);
  return hipGetLastError();
}

hipError_t amr_pack(const AmrGeom& G, const double* vb, const double* vf,
                    double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_pack, dim3(nblk(G.Nb + G.Nf)), dim3(kT), 0, s, G,
                     vb, vf, v);
  return hipGetLastError();
}

hipError_t amr_unpack(const AmrGeom& G, double* v, double* vb, double* vf,
                      hipStream_t s) {
  for (int l = G.L - 1; l >= 1; --l) {  // covered fine cells, finest first
    const hipError_t e = amr_restrict_level(G, l, v, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_amr_unpack, dim3(nblk(G.Nb + G.Nf)), dim3(kT), 0, s, G,
                     v, vb, vf);
  return hipGetLastError();
}

hipError_t amr_axpy(int64_t n, double a, const double* p, const double* x,
                    double* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_amr_axpy, dim3(nblk(n)), dim3(kT), 0, s, n, a, p, x,
                     y);
  return hipGetLastError();
}

int amr_dot_blocks(const AmrGeom& G) { return nblk(G.Nb + G.Nf); }

hipError_t amr_dots(const AmrGeom& G, const AmrDots& D, double* partials,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_amr_dots, dim3(amr_dot_blocks(G)), dim3(kT), 0, s, G, D,
                     partials);
  return hipGetLastError();
}

hipError_t amr_reduce(const double* partials, int nb, int npair, double* sc,
                      int slot, int copy, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_reduce, dim3(1), dim3(kRT), 0, s, partials, nb,
                     npair, sc, slot, copy);
  return hipGetLastError();
}

hipError_t amr_dir(int64_t n, const double* z, const double* p_old, double* p,
                   const double* sc, int first, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_dir, dim3(nblk(n)), dim3(kT), 0, s, n, z, p_old, p,
                     sc, first);
  return hipGetLastError();
}

hipError_t amr_update(const AmrGeom& G, const double* p, const double* q,
                      double* x, double* r, const double* sc,
                      double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_update, dim3(nblk(G.Nb + G.Nf)), dim3(kT), 0, s, G,
                     p, q, x, r, sc, partials);
  return hipGetLastError();
}

}  // namespace fld
