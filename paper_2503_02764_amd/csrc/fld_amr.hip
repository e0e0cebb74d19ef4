// Kernels of the block-adaptive 2D step (fld_amr.cpp): a base grid and one
// level of refined blocks, the backward-Euler diffusion of eq. mhd_r_e on
// the leaf cells (Sect. 3 solves it by multigrid on MPI-AMRVAC's
// block-adaptive grids).
//
// Vectors of leaf values are one array: the base grid's nx*ny cells (the
// entries of cells covered by refined blocks held at 0), then the fine
// blocks, each S x S = 2b x 2b cells, row-major.  Fine-resolution
// coordinates (I, J) run over a 2nx x 2ny lattice; a fine-level value there
// is the refined block's cell where the base cell (I/2, J/2) is refined,
// else that base cell's value (the fine level's view of the base grid).
// One thread per cell everywhere; tables (block of a base block, corner of
// a refined block) come from the host.
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

// refined block of base cell (i, j), or -1
__device__ __forceinline__ int amr_block(const AmrGeom& G, int i, int j) {
  return G.bmap[(j / G.b) * G.nbx + i / G.b];
}

// fine-level value at fine coordinates (I, J), inside the lattice
__device__ __forceinline__ double amr_fine_at(const AmrGeom& G,
                                              const double* vb,
                                              const double* vf, int I, int J) {
  const int i = I >> 1, j = J >> 1;
  const int blk = amr_block(G, i, j);
  if (blk < 0) return vb[(int64_t)j * G.nx + i];
  const int lx = I - G.S * G.bxy[2 * blk], ly = J - G.S * G.bxy[2 * blk + 1];
  return vf[((int64_t)blk * G.S + ly) * G.S + lx];
}

// index of the fine cell at fine coordinates (I, J) in the fine part
__device__ __forceinline__ int64_t amr_fine_idx(const AmrGeom& G, int blk,
                                                int I, int J) {
  const int lx = I - G.S * G.bxy[2 * blk], ly = J - G.S * G.bxy[2 * blk + 1];
  return ((int64_t)blk * G.S + ly) * G.S + lx;
}

// z at the fine neighbour of fine cell f (block-local (lx, ly), lattice
// (I, J)) in direction k (0 -x, 1 +x, 2 -y, 3 +y), for a face that exists:
// in-block neighbours by offset, the others through the tables
__device__ __forceinline__ double amr_nb(const AmrGeom& G, const double* vb,
                                         const double* vf, int64_t f, int lx,
                                         int ly, int I, int J, int k) {
  const int d = k >> 1, s = (k & 1) ? 1 : -1;
  const int l = d == 0 ? lx + s : ly + s;
  if (l >= 0 && l < G.S) return vf[f + (d == 0 ? s : s * G.S)];
  const int II = amr_wrap(I + (d == 0 ? s : 0), 2 * G.nx, 1);
  const int JJ = amr_wrap(J + (d == 1 ? s : 0), 2 * G.ny, 1);
  return amr_fine_at(G, vb, vf, II, JJ);
}

__device__ __forceinline__ double amr_mean(double a, double b, int kind) {
  return kind == 0 ? 0.5 * (a + b) : 2.0 * a * b / (a + b);
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

// base views: a covered base cell takes the mean of its four fine children
__global__ void __launch_bounds__(kT)
    k_amr_views(AmrGeom G, const double* __restrict__ Eb,
                const double* __restrict__ rb, const double* __restrict__ kb,
                const double* __restrict__ Ef, const double* __restrict__ rf,
                const double* __restrict__ kf, double* __restrict__ Ev,
                double* __restrict__ rv, double* __restrict__ kv) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c >= G.Nb) return;
  const int i = (int)(c % G.nx), j = (int)(c / G.nx);
  const int blk = amr_block(G, i, j);
  if (blk < 0) {
    Ev[c] = Eb[c];
    rv[c] = rb[c];
    kv[c] = kb[c];
    return;
  }
  const int64_t f = amr_fine_idx(G, blk, 2 * i, 2 * j);
  const int64_t q[4] = {f, f + 1, f + G.S, f + G.S + 1};
  const double* src[3] = {Ef, rf, kf};
  double* dst[3] = {Ev, rv, kv};
  for (int k = 0; k < 3; ++k)
    dst[k][c] = 0.25 * (src[k][q[0]] + src[k][q[1]] + src[k][q[2]] +
                        src[k][q[3]]);
}

// D of every base cell from the base views
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
  if (!(E0 > 0.0) || !(rk > 0.0) || !isfinite(E0) || !isfinite(rk))
    atomicAdd(bad, 1);
  Db[c] = amr_D(P, E0, rk, ex, ey, G.dx, G.dy);
}

// D of every fine cell from the fine-level view
__global__ void __launch_bounds__(kT)
    k_amr_dfine(AmrGeom G, AmrPhys P, const double* __restrict__ Ev,
                const double* __restrict__ Ef, const double* __restrict__ rf,
                const double* __restrict__ kf, double* __restrict__ Df,
                int* __restrict__ bad) {
  const int64_t f = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (f >= G.Nf) return;
  const int blk = (int)(f / ((int64_t)G.S * G.S));
  const int loc = (int)(f % ((int64_t)G.S * G.S));
  const int I = G.S * G.bxy[2 * blk] + loc % G.S;
  const int J = G.S * G.bxy[2 * blk + 1] + loc / G.S;
  const int NX = 2 * G.nx, NY = 2 * G.ny;
  double ex[4], ey[4];
  const int o[4] = {-2, -1, 1, 2};
  for (int k = 0; k < 4; ++k) {
    ex[k] = amr_fine_at(G, Ev, Ef, amr_wrap(I + o[k], NX, G.per[0]), J);
    ey[k] = amr_fine_at(G, Ev, Ef, I, amr_wrap(J + o[k], NY, G.per[1]));
  }
  const double E0 = Ef[f], rk = rf[f] * kf[f];
  if (!(E0 > 0.0) || !(rk > 0.0) || !isfinite(E0) || !isfinite(rk))
    atomicAdd(bad, 1);
  Df[f] = amr_D(P, E0, rk, ex, ey, 0.5 * G.dx, 0.5 * G.dy);
}

// the four faces of every fine cell (0: -x, 1: +x, 2: -y, 3: +y): to a
// fine neighbour alpha = dt D_face / h_f^2, to a base leaf cell across a
// block edge beta = (2/3) dt D_face / h_f^2, 0 at a wall
__global__ void __launch_bounds__(kT)
    k_amr_faces(AmrGeom G, AmrPhys P, double dt,
                const double* __restrict__ Db, const double* __restrict__ Df,
                double* __restrict__ cf) {
  const int64_t f = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (f >= G.Nf) return;
  const int blk = (int)(f / ((int64_t)G.S * G.S));
  const int loc = (int)(f % ((int64_t)G.S * G.S));
  const int I = G.S * G.bxy[2 * blk] + loc % G.S;
  const int J = G.S * G.bxy[2 * blk + 1] + loc / G.S;
  const int NX = 2 * G.nx, NY = 2 * G.ny;
  const double hx = 0.5 * G.dx, hy = 0.5 * G.dy;
  for (int k = 0; k < 4; ++k) {
    const int d = k >> 1, s = (k & 1) ? 1 : -1;
    int II = I + (d == 0 ? s : 0), JJ = J + (d == 1 ? s : 0);
    const int n = d == 0 ? NX : NY, cc = d == 0 ? II : JJ;
    double a = 0.0;
    if ((cc >= 0 && cc < n) || G.per[d]) {
      II = amr_wrap(II, NX, 1);
      JJ = amr_wrap(JJ, NY, 1);
      const double h2 = d == 0 ? hx * hx : hy * hy;
      const int nb = amr_block(G, II >> 1, JJ >> 1);
      if (nb >= 0) {
        a = dt * amr_mean(Df[f], Df[amr_fine_idx(G, nb, II, JJ)], P.face_mean) /
            h2;
      } else {
        const double Dc = Db[(int64_t)(JJ >> 1) * G.nx + (II >> 1)];
        a = (2.0 / 3.0) * dt * amr_mean(Df[f], Dc, P.face_mean) / h2;
      }
    }
    cf[(int64_t)k * G.Nf + f] = a;
  }
}

// The base cell's coupling to the fine cells across its face in direction
// k (0 -x, 1 +x, 2 -y, 3 +y) when that neighbour is covered: sum over the
// two fine cells along the face of (beta / 4) (x_c - x_f); returns false
// when the neighbour is a base leaf cell (or a wall).
__device__ __forceinline__ bool amr_base_to_fine(const AmrGeom& G,
                                                 const double* __restrict__ cf,
                                                 const double* __restrict__ xf,
                                                 int i, int j, int k, double xc,
                                                 double& acc) {
  const int d = k >> 1, s = (k & 1) ? 1 : -1;
  int ii = i + (d == 0 ? s : 0), jj = j + (d == 1 ? s : 0);
  const int n = d == 0 ? G.nx : G.ny, cc = d == 0 ? ii : jj;
  if ((cc < 0 || cc >= n) && !G.per[d]) return false;
  ii = amr_wrap(ii, G.nx, 1);
  jj = amr_wrap(jj, G.ny, 1);
  const int blk = amr_block(G, ii, jj);
  if (blk < 0) return false;
  // the fine cells of the neighbour along the shared face, and their face
  // pointing back at this cell (the opposite direction)
  const int back = k ^ 1;
  const int NX = 2 * G.nx, NY = 2 * G.ny;
  for (int q = 0; q < 2; ++q) {
    int I, J;
    if (d == 0) {
      I = s > 0 ? 2 * ii : 2 * ii + 1;
      J = 2 * jj + q;
    } else {
      I = 2 * ii + q;
      J = s > 0 ? 2 * jj : 2 * jj + 1;
    }
    I = amr_wrap(I, NX, 1);
    J = amr_wrap(J, NY, 1);
    const int64_t fi = amr_fine_idx(G, blk, I, J);
    acc += 0.25 * cf[(int64_t)back * G.Nf + fi] * (xc - xf[fi]);
  }
  return true;
}

// y = A x over the leaf cells (covered base entries: 0)
__device__ __forceinline__ double amr_apply_cell(
    const AmrGeom& G, const double* __restrict__ ax,
    const double* __restrict__ ay, const double* __restrict__ cf,
    const double* __restrict__ x, int64_t t) {
  const double* xf = x + G.Nb;
  if (t < G.Nb) {
    const int i = (int)(t % G.nx), j = (int)(t / G.nx);
    if (amr_block(G, i, j) >= 0) return 0.0;
    const double xc = x[t];
    double acc = xc;
    for (int k = 0; k < 4; ++k) {
      double part = 0.0;
      if (amr_base_to_fine(G, cf, xf, i, j, k, xc, part)) {
        acc += part;
        continue;
      }
      const int d = k >> 1, s = (k & 1) ? 1 : -1;
      const int n = d == 0 ? G.nx : G.ny;
      const int cc = d == 0 ? i + s : j + s;
      if ((cc < 0 || cc >= n) && !G.per[d]) continue;  // wall
      const int ii = d == 0 ? amr_wrap(i + s, G.nx, 1) : i;
      const int jj = d == 1 ? amr_wrap(j + s, G.ny, 1) : j;
      // the face between this cell and its neighbour belongs to the lower one
      const int64_t owner = s > 0 ? t : (int64_t)jj * G.nx + ii;
      const double a = (d == 0 ? ax : ay)[owner];
      acc += a * (xc - x[(int64_t)jj * G.nx + ii]);
    }
    return acc;
  }
  const int64_t f = t - G.Nb;
  const int blk = (int)(f / ((int64_t)G.S * G.S));
  const int loc = (int)(f % ((int64_t)G.S * G.S));
  const int lx = loc % G.S, ly = loc / G.S;
  const int I = G.S * G.bxy[2 * blk] + lx, J = G.S * G.bxy[2 * blk + 1] + ly;
  const double xi = xf[f];
  double acc = xi;
  for (int k = 0; k < 4; ++k) {
    const double a = cf[(int64_t)k * G.Nf + f];
    if (a == 0.0) continue;
    acc += a * (xi - amr_nb(G, x, xf, f, lx, ly, I, J, k));
  }
  return acc;
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
    const double w = t < G.Nb ? G.vb : G.vf;
    if (partials) {
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
    rr = (t < G.Nb ? G.vb : G.vf) * rv * rv;
  }
  const double tot = block_sum<kT>(rr, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// one colour ((I + J) & 1) of a Gauss-Seidel sweep over the fine cells for
// the correction z, with the base entries of z as fixed neighbour values
__global__ void __launch_bounds__(kT)
    k_amr_smooth(AmrGeom G, const double* __restrict__ cf,
                 const double* __restrict__ r, double* __restrict__ z,
                 int colour) {
  const int64_t f = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (f >= G.Nf) return;
  const int blk = (int)(f / ((int64_t)G.S * G.S));
  const int loc = (int)(f % ((int64_t)G.S * G.S));
  const int lx = loc % G.S, ly = loc / G.S;
  // S is even, so the colour of (I, J) is that of (lx, ly)
  if (((lx + ly) & 1) != colour) return;
  const int I = G.S * G.bxy[2 * blk] + lx, J = G.S * G.bxy[2 * blk + 1] + ly;
  const double* zf = z + G.Nb;
  double num = r[G.Nb + f], den = 1.0;
  for (int k = 0; k < 4; ++k) {
    const double a = cf[(int64_t)k * G.Nf + f];
    if (a == 0.0) continue;
    num += a * amr_nb(G, z, zf, f, lx, ly, I, J, k);
    den += a;
  }
  z[G.Nb + f] = num / den;
}

// right-hand side of the base correction after the fine pre-smoothing:
// a base leaf cell's residual with the fine correction's flux into it; a
// covered cell's the mean of its children's residuals (base entries of z
// are 0 here).  The pre-smoothing ends with a half-sweep of colour 1, which
// leaves those cells' residuals at 0 (up to rounding): only the two
// colour-0 children are evaluated.
__global__ void __launch_bounds__(kT)
    k_amr_base_rhs(AmrGeom G, const double* __restrict__ cf,
                   const double* __restrict__ r, const double* __restrict__ z,
                   double* __restrict__ rhs) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c >= G.Nb) return;
  const int i = (int)(c % G.nx), j = (int)(c / G.nx);
  const double* zf = z + G.Nb;
  const int blk = amr_block(G, i, j);
  if (blk < 0) {
    double acc = 0.0;  // sum of (beta / 4) (0 - z_f): minus the flux term
    for (int k = 0; k < 4; ++k) amr_base_to_fine(G, cf, zf, i, j, k, 0.0, acc);
    rhs[c] = r[c] - acc;
    return;
  }
  double s = 0.0;
  for (int q = 0; q < 2; ++q) {  // (0, 0) and (1, 1) of the 2 x 2 children
    const int I = 2 * i + q, J = 2 * j + q;
    const int64_t f = amr_fine_idx(G, blk, I, J);
    const int lx = I - G.S * G.bxy[2 * blk], ly = J - G.S * G.bxy[2 * blk + 1];
    double az = zf[f];
    for (int k = 0; k < 4; ++k) {
      const double a = cf[(int64_t)k * G.Nf + f];
      if (a == 0.0) continue;
      az += a * (zf[f] - amr_nb(G, z, zf, f, lx, ly, I, J, k));
    }
    s += r[G.Nb + f] - az;
  }
  rhs[c] = 0.25 * s;
}

// z_f += the base correction, bilinear from the parent cell and its
// neighbours towards the fine cell (weights 9, 3, 3, 1 over 16)
__global__ void __launch_bounds__(kT)
    k_amr_prolong(AmrGeom G, double* __restrict__ z) {
  const int64_t f = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (f >= G.Nf) return;
  const int blk = (int)(f / ((int64_t)G.S * G.S));
  const int loc = (int)(f % ((int64_t)G.S * G.S));
  const int I = G.S * G.bxy[2 * blk] + loc % G.S;
  const int J = G.S * G.bxy[2 * blk + 1] + loc / G.S;
  const int i = I >> 1, j = J >> 1;
  const int i2 = amr_wrap(i + ((I & 1) ? 1 : -1), G.nx, G.per[0]);
  const int j2 = amr_wrap(j + ((J & 1) ? 1 : -1), G.ny, G.per[1]);
  const double* zb = z;
  const double v = (9.0 * zb[(int64_t)j * G.nx + i] +
                    3.0 * zb[(int64_t)j * G.nx + i2] +
                    3.0 * zb[(int64_t)j2 * G.nx + i] +
                    zb[(int64_t)j2 * G.nx + i2]) / 16.0;
  z[G.Nb + f] += v;
}

// covered base entries of a leaf vector back to 0
__global__ void __launch_bounds__(kT)
    k_amr_zero_covered(AmrGeom G, double* __restrict__ v) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c >= G.Nb) return;
  if (amr_block(G, (int)(c % G.nx), (int)(c / G.nx)) >= 0) v[c] = 0.0;
}

// leaf vector from (base, fine) arrays, covered base entries 0
__global__ void __launch_bounds__(kT)
    k_amr_pack(AmrGeom G, const double* __restrict__ vb,
               const double* __restrict__ vf, double* __restrict__ v) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t < G.Nb) {
    const int i = (int)(t % G.nx), j = (int)(t / G.nx);
    v[t] = amr_block(G, i, j) >= 0 ? 0.0 : vb[t];
  } else if (t < G.Nb + G.Nf) {
    v[t] = vf[t - G.Nb];
  }
}

// (base, fine) arrays from a leaf vector: a covered base cell gets the mean
// of its four fine children
__global__ void __launch_bounds__(kT)
    k_amr_unpack(AmrGeom G, const double* __restrict__ v,
                 double* __restrict__ vb, double* __restrict__ vf) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t < G.Nb) {
    const int i = (int)(t % G.nx), j = (int)(t / G.nx);
    const int blk = amr_block(G, i, j);
    if (blk < 0) {
      vb[t] = v[t];
    } else {
      const int64_t f = G.Nb + amr_fine_idx(G, blk, 2 * i, 2 * j);
      vb[t] = 0.25 * (v[f] + v[f + 1] + v[f + G.S] + v[f + G.S + 1]);
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
  const double w = t < G.Nb ? G.vb : G.vf;
  for (int k = 0; k < D.n; ++k) {
    const double s = t < G.Nb + G.Nf ? w * D.u[k][t] * D.v[k][t] : 0.0;
    const double tot = block_sum<kT>(s, sh);
    __syncthreads();  // sh is reused by the next sum
    if (threadIdx.x == 0) partials[(int64_t)k * gridDim.x + blockIdx.x] = tot;
  }
}

inline int nblk(int64_t n) { return (int)((n + kT - 1) / kT); }

}  // namespace

hipError_t amr_views(const AmrGeom& G, const double* Eb, const double* rb,
                     const double* kb, const double* Ef, const double* rf,
                     const double* kf, double* Ev, double* rv, double* kv,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_amr_views, dim3(nblk(G.Nb)), dim3(kT), 0, s, G, Eb, rb,
                     kb, Ef, rf, kf, Ev, rv, kv);
  return hipGetLastError();
}

hipError_t amr_coefficients(const AmrGeom& G, const AmrPhys& P, double dt,
                            const double* Ev, const double* rv,
                            const double* kv, const double* Ef,
                            const double* rf, const double* kf, double* Db,
                            double* Df, double* cf, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_dbase, dim3(nblk(G.Nb)), dim3(kT), 0, s, G, P, Ev,
                     rv, kv, Db, bad);
  if (G.Nf > 0) {
    hipLaunchKernelGGL(k_amr_dfine, dim3(nblk(G.Nf)), dim3(kT), 0, s, G, P,
                       Ev, Ef, rf, kf, Df, bad);
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

hipError_t amr_smooth(const AmrGeom& G, const double* cf, const double* r,
                      double* z, int colour, hipStream_t s, hipEvent_t ev0,
                      hipEvent_t ev1) {
  if (G.Nf == 0) return hipSuccess;
  if (ev0 && ev1)  // the launch records its own start and end
    hipExtLaunchKernelGGL(k_amr_smooth, dim3(nblk(G.Nf)), dim3(kT), 0, s, ev0,
                          ev1, 0, G, cf, r, z, colour);
  else
    hipLaunchKernelGGL(k_amr_smooth, dim3(nblk(G.Nf)), dim3(kT), 0, s, G, cf,
                       r, z, colour);
  return hipGetLastError();
}

hipError_t amr_base_rhs(const AmrGeom& G, const double* cf, const double* r,
                        const double* z, double* rhs, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_base_rhs, dim3(nblk(G.Nb)), dim3(kT), 0, s, G, cf,
                     r, z, rhs);
  return hipGetLastError();
}

hipError_t amr_prolong(const AmrGeom& G, double* z, hipStream_t s) {
  if (G.Nf == 0) return hipSuccess;
  hipLaunchKernelGGL(k_amr_prolong, dim3(nblk(G.Nf)), dim3(kT), 0, s, G, z);
  return hipGetLastError();
}

hipError_t amr_zero_covered(const AmrGeom& G, double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_zero_covered, dim3(nblk(G.Nb)), dim3(kT), 0, s, G,
                     v);
  return hipGetLastError();
}

hipError_t amr_pack(const AmrGeom& G, const double* vb, const double* vf,
                    double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_pack, dim3(nblk(G.Nb + G.Nf)), dim3(kT), 0, s, G,
                     vb, vf, v);
  return hipGetLastError();
}

hipError_t amr_unpack(const AmrGeom& G, const double* v, double* vb,
                      double* vf, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_unpack, dim3(nblk(G.Nb + G.Nf)), dim3(kT), 0, s, G,
                     v, vb, vf);
  return hipGetLastError();
}

hipError_t amr_axpy(int64_t n, double a, const double* p, const double* x,
                    double* y, hipStream_t s) {
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

}  // namespace fld
