// Coefficient stage of a 2D grid, LDS-tiled (gfx950).
//
// The arithmetic is that of k_coef (eqs. fld_F, fld_lambda, fld_R and the
// face mean of Sect. 3): five-point fourth-order gradient with mirror or
// periodic ghosts, R = |grad E| / (rho kappa E), the limiter, D = c lambda /
// (rho kappa) at the cell centre, face D by the arithmetic or harmonic mean,
// alpha = dt D_f / dx^2 on each face (0 on a Neumann wall face).  Here a block
// owns a tile of 64 x 16 cells: it stages E of the tile plus three ghost
// cells per side in LDS, computes D once per cell of the tile plus one ring,
// and forms both face coefficients of every tile cell from LDS (k_coef
// computes the neighbour's D again for each face).  The operations and their
// order per value are k_coef's, so the coefficients are the same bits.
//
// Optionally (the iterate starts at E^n, the right-hand side) the block also
// forms the initial residual b - A E^n = -sum_f alpha_f (E - E_f) of its
// cells, so that the first stop test needs no separate pass; block partial
// sums of |E|^2 and |r|^2 go to partials[blk] and partials[nblocks + blk].
#include "fld_internal.h"
#include "fld_device.h"

namespace fld {

namespace {

constexpr int CX = 64, CY = 16;           // output tile
constexpr int DX = CX + 2, DY = CY + 2;   // D: tile plus one ring
constexpr int EX = CX + 6, EY = CY + 6;   // E: tile plus three rings
constexpr int NTC = 256;                  // threads: 64 columns x 4 row groups
constexpr int RPT = CY / (NTC / CX);      // rows per thread (4)

struct Coef2DArgs {
  CoefArgs A;
  const double* E;
  const double* rho;
  const double* kappa;
  CoefOut O;
  int tiles_x;
  int resid;  // also form the initial residual (x0 = b = E^n)
};

__device__ __forceinline__ int wrap_clamp(int m, int n, int per) {
  if (per) {
    m %= n;
    return m < 0 ? m + n : m;
  }
  return m < 0 ? 0 : (m >= n ? n - 1 : m);
}

}  // namespace

__global__ void __launch_bounds__(NTC) k_coef2d(Coef2DArgs P) {
  const CoefArgs& A = P.A;
  __shared__ double Es[EY][EX];
  __shared__ double Ds[DY][DX];
  __shared__ double sh[NTC / 64];
  __shared__ int bad_count;
  const int nx = A.g.n[0], ny = A.g.n[1];
  const int perx = A.g.per[0], pery = A.g.per[1];
  const int ty_ = blockIdx.x / P.tiles_x, tx_ = blockIdx.x - ty_ * P.tiles_x;
  const int x0 = tx_ * CX, y0 = ty_ * CY;
  const int t = threadIdx.x;
  if (t == 0) bad_count = 0;

  // E of the tile and three ghost rings, through the stage's ghost mapping
  // (rings beyond the second only feed D of cells behind a Neumann wall,
  // which no coefficient uses; their indices are clamped into the array)
  for (int k = t; k < EX * EY; k += NTC) {
    const int ly = k / EX, lx = k - ly * EX;
    const int gx = ghost(x0 + lx - 3, nx, perx), gy = ghost(y0 + ly - 3, ny, pery);
    const int cx = gx < 0 ? 0 : (gx >= nx ? nx - 1 : gx);
    const int cy = gy < 0 ? 0 : (gy >= ny ? ny - 1 : gy);
    Es[ly][lx] = P.E[(int64_t)cy * nx + cx];
  }
  __syncthreads();

  // D of the tile and one ring (cell_D's arithmetic, E from LDS)
  for (int k = t; k < DX * DY; k += NTC) {
    const int ly = k / DX, lx = k - ly * DX;
    const int gx = wrap_clamp(x0 + lx - 1, nx, perx);
    const int gy = wrap_clamp(y0 + ly - 1, ny, pery);
    const int64_t idx = (int64_t)gy * nx + gx;
    const int ex = lx + 2, ey = ly + 2;  // this cell in Es
    const double E0 = Es[ey][ex];
    const double rk = P.rho[idx] * P.kappa[idx];
    double g2 = 0.0;
    {
      const double G = (Es[ey][ex - 2] - 8.0 * Es[ey][ex - 1] +
                        8.0 * Es[ey][ex + 1] - Es[ey][ex + 2]) *
                       A.gscale[0];
      g2 += G * G;
    }
    {
      const double G = (Es[ey - 2][ex] - 8.0 * Es[ey - 1][ex] +
                        8.0 * Es[ey + 1][ex] - Es[ey + 2][ex]) *
                       A.gscale[1];
      g2 += G * G;
    }
    const double R = sqrt(g2) / (rk * E0);
    const double lam = flux_limiter(A.limiter, R);
    Ds[ly][lx] = A.c * lam / rk;
    // non-physical state of a tile cell
    const bool inside = lx >= 1 && lx <= CX && ly >= 1 && ly <= CY &&
                        x0 + lx - 1 < nx && y0 + ly - 1 < ny;
    if (inside &&
        (!(E0 > 0.0) || !(rk > 0.0) || !isfinite(E0) || !isfinite(rk)))
      atomicAdd(&bad_count, 1);
  }
  __syncthreads();

  auto face = [&](double D0, double Dn, int d) {
    const double Df =
        A.face_mean == 0 ? 0.5 * (D0 + Dn) : 2.0 * D0 * Dn / (D0 + Dn);
    return A.dt * Df / (A.dx[d] * A.dx[d]);
  };
  const int cxl = t % CX, rg = t / CX;
  double e2 = 0.0, r2 = 0.0;
  const int i = x0 + cxl;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int ly = rg * RPT + k;
    const int j = y0 + ly;
    if (i >= nx || j >= ny) continue;
    const int64_t idx = (int64_t)j * nx + i;
    const double D0 = Ds[ly + 1][cxl + 1];
    const bool hr = i < nx - 1 || perx, hu = j < ny - 1 || pery;
    const double ar = hr ? face(D0, Ds[ly + 1][cxl + 2], 0) : 0.0;
    const double au = hu ? face(D0, Ds[ly + 2][cxl + 1], 1) : 0.0;
    P.O.a64[0][idx] = ar;
    P.O.a64[1][idx] = au;
    if (P.O.a32[0]) {
      P.O.a32[0][idx] = (float)ar;
      P.O.a32[1][idx] = (float)au;
    }
    const double Ei = Es[ly + 3][cxl + 3];
    if (P.O.copy_dst) P.O.copy_dst[idx] = Ei;
    e2 += Ei * Ei;
    if (P.resid) {
      // the faces on the left and below, as the neighbours compute them
      const bool hl = i > 0 || perx, hd = j > 0 || pery;
      const double al = hl ? face(Ds[ly + 1][cxl], D0, 0) : 0.0;
      const double ad = hd ? face(Ds[ly][cxl + 1], D0, 1) : 0.0;
      // neighbours of the iterate: periodic wrap (a Neumann wall has a zero
      // coefficient, so its ghost value does not enter)
      const double El = Es[ly + 3][cxl + 2], Er = Es[ly + 3][cxl + 4];
      const double Ed = Es[ly + 2][cxl + 3], Eu = Es[ly + 4][cxl + 3];
      const double r = -(al * (Ei - El) + ar * (Ei - Er) + ad * (Ei - Ed) +
                         au * (Ei - Eu));
      r2 += r * r;
    }
  }
  const double s1 = block_sum<NTC>(e2, sh);
  __syncthreads();
  const double s2 = P.resid ? block_sum<NTC>(r2, sh) : 0.0;
  if (t == 0) {
    const int nb = gridDim.x;
    P.O.partials[blockIdx.x] = s1;
    if (P.resid) P.O.partials[nb + blockIdx.x] = s2;
    if (bad_count > 0) atomicAdd(&P.O.ctrl->flagged, bad_count);
  }
}

int coef2d_blocks(const Geom& g) {
  return ((g.n[0] + CX - 1) / CX) * ((g.n[1] + CY - 1) / CY);
}

bool coef2d_ok(const Geom& g) {
  return g.ndim == 2 && g.n[0] >= 4 && g.n[1] >= 4;
}

hipError_t launch_coef2d(const CoefArgs& a, const double* E, const double* rho,
                         const double* kappa, double* const a64[3],
                         float* const a32[3], double* copy_dst,
                         double* partials, Control* ctrl, bool resid,
                         hipStream_t s) {
  Coef2DArgs P;
  P.A = a;
  P.E = E;
  P.rho = rho;
  P.kappa = kappa;
  for (int d = 0; d < 3; ++d) {
    P.O.a64[d] = a64[d];
    P.O.a32[d] = a32[d];
  }
  P.O.copy_dst = copy_dst;
  // Dirichlet walls and held cells take the one-pass kernel
  P.O.sd = P.O.rhs = nullptr;
  P.O.held = nullptr;
  P.O.hold = nullptr;
  P.O.partials = partials;
  P.O.ctrl = ctrl;
  P.tiles_x = (a.g.n[0] + CX - 1) / CX;
  P.resid = resid ? 1 : 0;
  hipLaunchKernelGGL(k_coef2d, dim3(coef2d_blocks(a.g)), dim3(NTC), 0, s, P);
  return hipGetLastError();
}

}  // namespace fld
