// Two-dimensional multigrid tail with every cell's Gauss-Seidel weights in
// registers (gfx950).
//
// One block of 256 threads runs one sub-V-cycle over the tail levels (at
// most 1024 cells on the first; each later level is a quarter of the one
// before).  Levels come in three kinds:
//   wide   (257..1024 cells): thread t owns the 2x2 cell block t, so two of
//          every cell's four neighbours, the 2x2 restriction and the
//          injection of the coarse correction's own term are in registers;
//   narrow (65..256 cells): thread t owns cell t;
//   tiny   (<= 64 cells): wave 0 alone, lane t owns cell t; its phases are
//          ordered by LDS fences instead of block barriers.
// The sequence is therefore [wide] [narrow] tiny+, and the coarsest level
// is tiny.  Weights and the LDS offsets of the neighbours are computed once
// per call from the face coefficients; a red-black update is then
//   x = b/d + sum_f (alpha_f/d) x_f,   d = 1 + sum_f alpha_f,
// with the rounding of the tiled kernels, and the residual is
// d (x_update - x).  Only the iterates (and a residual scratch for the
// restriction onto tiny levels) live in LDS.
//
// A second kernel, k_tail2d_big (1024 threads), starts one level higher,
// on a level of 1025..4096 cells held as 2x2 blocks, and runs the next two
// levels one cell per thread: on a 1024^2 grid that replaces the tiled
// down and up passes of the 64^2 level (two launches per V-cycle).
//
// The multigrid itself is that of the other tail kernels: pre-smoothing,
// residual restricted by the mean of the 2x2 children, coarse correction
// from zero, coarsest red-black sweeps until the residual drops by 1e-3
// (tested every 2 sweeps, at most 4000), cell-centred bilinear prolongation
// (weights 9/16, 3/16, 3/16, 1/16), post-smoothing.
#include "fld_internal.h"
#include "fld_wave.h"

namespace fld {

namespace {

constexpr int NT2 = 256;
constexpr int kTinyMax = 3;
constexpr int kWideMax = 1024, kNarrowMax = 256, kTinyCells = 64;
// LDS layout (elements of T)
constexpr int kSW = 0;                        // wide iterate
constexpr int kSN = kSW + kWideMax;           // narrow iterate
constexpr int kST = kSN + kNarrowMax;         // tiny iterates, 64 each
constexpr int kSR = kST + kTinyMax * kTinyCells;  // residual scratch
constexpr int kSTotal = kSR + kNarrowMax;

enum Kind { kWide = 0, kNarrow = 1, kTinyKind = 2 };

__host__ __device__ inline int kind_of(int64_t n) {
  return n > kNarrowMax ? kWide : (n > kTinyCells ? kNarrow : kTinyKind);
}

template <typename T>
__device__ __forceinline__ T gs_val(T bp, T wl, T xl, T wr, T xr, T wd, T xd,
                                    T wu, T xu) {
  return fma(wu, xu, fma(wd, xd, fma(wr, xr, fma(wl, xl, bp))));
}

template <typename T>
__device__ __forceinline__ T bilin(T e0, T e1, T e2, T e3) {
  return fma(T(0.0625), e3,
             fma(T(0.1875), e2, fma(T(0.1875), e1, T(0.5625) * e0)));
}

// Weights of one cell and the LDS offsets of its neighbours (the cell's own
// offset behind a Neumann wall, where the weight is zero).
template <typename T>
struct CellW {
  T wl, wr, wd, wu, inv, dn;
  int ol, orr, od, ou;
};

// Face coefficients around cell (i, j) of a level, as loaded: left, right,
// down, up (the left and lower loads are clamped into the array and masked
// later, behind a Neumann wall).
template <typename T>
struct CellA {
  T al, ar, ad, au;
  int i, j;
};

template <typename T>
__device__ __forceinline__ CellA<T> cell_alpha(const LevelView<T>& L, int i,
                                               int j) {
  const int nx = L.g.n[0], ny = L.g.n[1];
  const int idx = j * nx + i;
  const int il = i > 0 ? idx - 1 : idx + nx - 1;
  const int id = j > 0 ? idx - nx : idx + (ny - 1) * nx;
  CellA<T> a;
  a.al = L.a[0][il];
  a.ad = L.a[1][id];
  a.ar = L.a[0][idx];  // zero on a Neumann wall face
  a.au = L.a[1][idx];
  a.i = i;
  a.j = j;
  return a;
}

template <typename T>
__device__ __forceinline__ CellW<T> cell_weights(const Geom& g, const CellA<T>& a,
                                                 int base) {
  const int nx = g.n[0], ny = g.n[1];
  const int px = g.per[0], py = g.per[1];
  const int i = a.i, j = a.j;
  const int idx = j * nx + i;
  const bool hl = i > 0 || px, hd = j > 0 || py;
  const bool hr = i < nx - 1 || px, hu = j < ny - 1 || py;
  const int il = i > 0 ? idx - 1 : idx + nx - 1;
  const int id = j > 0 ? idx - nx : idx + (ny - 1) * nx;
  const int ir = i < nx - 1 ? idx + 1 : idx - (nx - 1);
  const int iu = j < ny - 1 ? idx + nx : idx - (ny - 1) * nx;
  const T al = hl ? a.al : T(0);
  const T ad = hd ? a.ad : T(0);
  const T d = T(1) + al + a.ar + ad + a.au;
  const T inv = T(1) / d;
  CellW<T> c;
  c.wl = al * inv;
  c.wr = a.ar * inv;
  c.wd = ad * inv;
  c.wu = a.au * inv;
  c.inv = inv;
  c.dn = d;
  c.ol = base + (hl ? il : idx);
  c.orr = base + (hr ? ir : idx);
  c.od = base + (hd ? id : idx);
  c.ou = base + (hu ? iu : idx);
  return c;
}

// LDS writes of this wave complete before its later reads (tiny levels).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Second coarse index of a fine cell along one dimension (bilinear
// prolongation): the nearer neighbour of its parent, wrapped or clamped.
__device__ __forceinline__ int second_parent(int f, int nc, int per) {
  const int p = f >> 1;
  int o = (f & 1) ? p + 1 : p - 1;
  if (o < 0) o = per ? nc - 1 : 0;
  if (o >= nc) o = per ? 0 : nc - 1;
  return o;
}

}  // namespace

// Host check: the tail levels of `a` fit this kernel.
template <typename T>
bool tail2d_ok(const TailArgs<T>& a) {
  if (a.whole) return false;
  const int nt = a.L - a.l0;
  if (nt < 2) return false;
  int ntiny = 0;
  for (int j = 0; j < nt; ++j) {
    const Geom& g = a.lv[a.l0 + j].g;
    if (g.ndim != 2) return false;
    // red-black colouring only (no odd periodic dimension)
    if (gs_colors(g) != 2) return false;
    const int k = kind_of(g.N);
    if (j == 0 && g.N > kWideMax) return false;
    if (j > 0) {
      const int kp = kind_of(a.lv[a.l0 + j - 1].g.N);
      // wide -> narrow -> tiny...: each level a quarter of the one before
      if (g.N * 4 != a.lv[a.l0 + j - 1].g.N) return false;
      if (kp == kWide && k != kNarrow) return false;
      if (kp != kWide && k != kTinyKind) return false;
    }
    if (k == kWide && (g.n[0] % 2 || g.n[1] % 2)) return false;
    if (k == kTinyKind) ++ntiny;
  }
  if (kind_of(a.lv[a.L - 1].g.N) != kTinyKind) return false;
  return ntiny <= kTinyMax;
}

template <typename T>
__device__ __forceinline__ void tail2d_body(const TailArgs<T>& A) {
  __shared__ T S[kSTotal];
  // The stop flag and every set-up operand are loaded before the first is
  // used (loads of absent levels read valid cells of the first level and
  // are discarded), so the set-up costs one memory round trip.
  const int done = A.ctrl->done;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const bool wave0 = t < 64;
  const int l0 = A.l0, nt = A.L - l0;
  const int k0 = kind_of(A.lv[l0].g.N);
  const bool has_wide = k0 == kWide;
  const bool has_narrow = k0 != kTinyKind;
  const int jn = has_wide ? 1 : 0;        // narrow level index
  const int jt0 = has_narrow ? jn + 1 : 0;  // first tiny level
  const int ntiny = nt - jt0;

  // ---- set-up loads ----
  const LevelView<T>& Lw = A.lv[l0];
  const int hx = Lw.g.n[0] / 2;
  const bool own_w = has_wide && t < (int)Lw.g.N / 4;
  const int bi = own_w ? t % hx : 0, bj = own_w ? t / hx : 0;
  const int wnx = Lw.g.n[0];
  CellA<T> aw[2][2];
  T xw[2][2], bw[2][2];
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = min(2 * bi + u, Lw.g.n[0] - 1);
      const int j = min(2 * bj + v, Lw.g.n[1] - 1);
      aw[v][u] = cell_alpha(Lw, i, j);
      xw[v][u] = Lw.x[j * wnx + i];
      bw[v][u] = Lw.b[j * wnx + i];
    }
  const LevelView<T>& Ln = A.lv[l0 + jn];
  const bool own_n = has_narrow && t < (int)Ln.g.N;
  const int ni = own_n ? t % Ln.g.n[0] : 0, nj = own_n ? t / Ln.g.n[0] : 0;
  const CellA<T> an = cell_alpha(Ln, ni, nj);
  T xn = Ln.x[nj * Ln.g.n[0] + ni];
  T bn = Ln.b[nj * Ln.g.n[0] + ni];
  CellA<T> at[kTinyMax];
  bool own_t[kTinyMax];
#pragma unroll
  for (int q = 0; q < kTinyMax; ++q) {
    const LevelView<T>& L = A.lv[l0 + min(jt0 + q, nt - 1)];
    own_t[q] = wave0 && q < ntiny && lane < (int)L.g.N;
    at[q] = cell_alpha(L, own_t[q] ? lane % L.g.n[0] : 0,
                       own_t[q] ? lane / L.g.n[0] : 0);
  }
  const LevelView<T>& Lt = A.lv[l0 + jt0];
  T xt0 = Lt.x[own_t[0] ? lane : 0];
  T bt0 = Lt.b[own_t[0] ? lane : 0];
  if (done != kRunning) return;

  // ---- weights, starting iterates ----
  CellW<T> cw[2][2];
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      cw[v][u] = cell_weights(Lw.g, aw[v][u], kSW);
      if (A.zero || !own_w) xw[v][u] = T(0);
      if (!own_w) bw[v][u] = T(0);
    }
  const CellW<T> cn = cell_weights(Ln.g, an, kSN);
  if (has_wide || !own_n) {
    xn = T(0);
    bn = T(0);
  } else if (A.zero) {
    xn = T(0);
  }
  CellW<T> ct[kTinyMax];
  T bt[kTinyMax];
  int ti[kTinyMax], tj[kTinyMax];
#pragma unroll
  for (int q = 0; q < kTinyMax; ++q) {
    const LevelView<T>& L = A.lv[l0 + min(jt0 + q, nt - 1)];
    ct[q] = cell_weights(L.g, at[q], kST + q * kTinyCells);
    ti[q] = at[q].i;
    tj[q] = at[q].j;
    bt[q] = T(0);
  }
  if (jt0 == 0 && own_t[0]) {
    bt[0] = bt0;
    if (A.zero) xt0 = T(0);
  } else {
    xt0 = T(0);
  }
  if (has_wide) {
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int u = 0; u < 2; ++u)
        if (own_w) S[kSW + (2 * bj + v) * wnx + 2 * bi + u] = xw[v][u];
  } else if (has_narrow) {
    if (own_n) S[kSN + t] = xn;
  } else if (own_t[0]) {
    S[kST + lane] = xt0;
  }
  __syncthreads();

  // ---- wide level: pre-smoothing, residual, restriction onto narrow ----
  T bpw[2][2];
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int u = 0; u < 2; ++u) bpw[v][u] = bw[v][u] * cw[v][u].inv;
  auto wide_pass = [&](int c) {
    if (own_w) {
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          if (((u + v) & 1) != c) continue;
          const CellW<T>& w = cw[v][u];
          const T xl = u ? xw[v][0] : S[w.ol];
          const T xr = u ? S[w.orr] : xw[v][1];
          const T xd = v ? xw[0][u] : S[w.od];
          const T xu = v ? S[w.ou] : xw[1][u];
          xw[v][u] = gs_val(bpw[v][u], w.wl, xl, w.wr, xr, w.wd, xd, w.wu, xu);
          S[kSW + (2 * bj + v) * wnx + 2 * bi + u] = xw[v][u];
        }
    }
    __syncthreads();
  };
  if (has_wide) {
    for (int s = 0; s < A.pre; ++s) {
      wide_pass(0);
      wide_pass(1);
    }
    // residual of the 2x2 block; its mean is the narrow cell t's rhs
    if (own_w) {
      T r[2][2];
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const CellW<T>& w = cw[v][u];
          const T xl = u ? xw[v][0] : S[w.ol];
          const T xr = u ? S[w.orr] : xw[v][1];
          const T xd = v ? xw[0][u] : S[w.od];
          const T xu = v ? S[w.ou] : xw[1][u];
          r[v][u] = w.dn * (gs_val(bpw[v][u], w.wl, xl, w.wr, xr, w.wd, xd,
                                   w.wu, xu) -
                            xw[v][u]);
        }
      bn = T(0.25) * ((r[0][0] + r[0][1]) + (r[1][0] + r[1][1]));
    }
    xn = T(0);
    if (own_n) S[kSN + t] = T(0);
    __syncthreads();
  }

  // ---- narrow level ----
  const T bpn = bn * cn.inv;
  const int ncolor = (ni + nj) & 1;
  auto narrow_pass = [&](int c) {
    if (own_n && ncolor == c) {
      xn = gs_val(bpn, cn.wl, S[cn.ol], cn.wr, S[cn.orr], cn.wd, S[cn.od],
                  cn.wu, S[cn.ou]);
      S[kSN + t] = xn;
    }
    __syncthreads();
  };
  if (has_narrow) {
    for (int s = 0; s < A.pre; ++s) {
      narrow_pass(0);
      narrow_pass(1);
    }
    if (own_n)
      S[kSR + t] = cn.dn * (gs_val(bpn, cn.wl, S[cn.ol], cn.wr, S[cn.orr],
                                   cn.wd, S[cn.od], cn.wu, S[cn.ou]) -
                            xn);
    __syncthreads();
  }

  // ---- tiny levels: wave 0 alone ----
  if (wave0) {
    T xt[kTinyMax], bpt[kTinyMax];
    xt[0] = xt0;
#pragma unroll
    for (int q = 0; q < kTinyMax; ++q) {
      if (q >= ntiny) break;
      const int base = kST + q * kTinyCells;
      if (q > 0 || jt0 > 0) {
        // rhs: mean of the four children's residuals (scratch), x = 0
        if (own_t[q]) {
          const int fnx = A.lv[l0 + jt0 + q - 1].g.n[0];
          const int f0 = 2 * tj[q] * fnx + 2 * ti[q];
          const T r00 = S[kSR + f0], r01 = S[kSR + f0 + 1];
          const T r10 = S[kSR + f0 + fnx], r11 = S[kSR + f0 + fnx + 1];
          bt[q] = T(0.25) * ((r00 + r01) + (r10 + r11));
          S[base + lane] = T(0);
        }
        xt[q] = T(0);
      }
      bpt[q] = bt[q] * ct[q].inv;
      wave_lds_sync();
      const int color = (ti[q] + tj[q]) & 1;
      const CellW<T>& w = ct[q];
      const bool last = q == ntiny - 1;
      auto tiny_sweeps = [&](int sweeps) {
        for (int s = 0; s < sweeps; ++s)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            if (own_t[q] && color == c) {
              xt[q] = gs_val(bpt[q], w.wl, S[w.ol], w.wr, S[w.orr], w.wd,
                             S[w.od], w.wu, S[w.ou]);
              S[base + lane] = xt[q];
            }
            wave_lds_sync();
          }
      };
      auto tiny_r2 = [&]() {
        double r2 = 0.0;
        if (own_t[q]) {
          const double r = (double)(w.dn * (gs_val(bpt[q], w.wl, S[w.ol], w.wr,
                                                   S[w.orr], w.wd, S[w.od],
                                                   w.wu, S[w.ou]) -
                                            xt[q]));
          r2 = r * r;
        }
        return wave_sum(r2);
      };
      if (!last) {
        tiny_sweeps(A.pre);
        if (own_t[q])
          S[kSR + lane] = w.dn * (gs_val(bpt[q], w.wl, S[w.ol], w.wr, S[w.orr],
                                         w.wd, S[w.od], w.wu, S[w.ou]) -
                                  xt[q]);
        wave_lds_sync();
      } else {
        // coarsest: sweeps from zero until the residual dropped by 1e-3
        const double b = own_t[q] ? (double)bt[q] : 0.0;
        const double r0 = wave_sum(b * b);
        tiny_sweeps(2);
        if (tiny_r2() > 1e-6 * r0) {  // squared norms
          for (int it = 0; it < 4000; it += 2) {
            tiny_sweeps(2);
            if (!(tiny_r2() > 1e-6 * r0)) break;
          }
        }
      }
    }
    // up through the tiny levels
#pragma unroll
    for (int q = kTinyMax - 2; q >= 0; --q) {
      if (q + 1 >= ntiny) continue;
      const LevelView<T>& C = A.lv[l0 + jt0 + q + 1];
      const int cbase = kST + (q + 1) * kTinyCells;
      const int base = kST + q * kTinyCells;
      if (own_t[q]) {
        const int cnx = C.g.n[0], cny = C.g.n[1];
        const int I = ti[q] >> 1, J = tj[q] >> 1;
        const int I2 = second_parent(ti[q], cnx, C.g.per[0]);
        const int J2 = second_parent(tj[q], cny, C.g.per[1]);
        xt[q] += bilin(S[cbase + J * cnx + I], S[cbase + J * cnx + I2],
                       S[cbase + J2 * cnx + I], S[cbase + J2 * cnx + I2]);
        S[base + lane] = xt[q];
      }
      wave_lds_sync();
      const int color = (ti[q] + tj[q]) & 1;
      const CellW<T>& w = ct[q];
      for (int s = 0; s < A.post; ++s)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          if (own_t[q] && color == c) {
            xt[q] = gs_val(bpt[q], w.wl, S[w.ol], w.wr, S[w.orr], w.wd,
                           S[w.od], w.wu, S[w.ou]);
            S[base + lane] = xt[q];
          }
          wave_lds_sync();
        }
    }
    if (jt0 == 0 && own_t[0]) A.lv[l0].x[lane] = xt[0];
  }
  __syncthreads();

  // ---- narrow level: correction from the first tiny level, post-smoothing
  if (has_narrow) {
    if (own_n) {
      const LevelView<T>& C = A.lv[l0 + jt0];
      const int cnx = C.g.n[0], cny = C.g.n[1];
      const int I = ni >> 1, J = nj >> 1;
      const int I2 = second_parent(ni, cnx, C.g.per[0]);
      const int J2 = second_parent(nj, cny, C.g.per[1]);
      xn += bilin(S[kST + J * cnx + I], S[kST + J * cnx + I2],
                  S[kST + J2 * cnx + I], S[kST + J2 * cnx + I2]);
      S[kSN + t] = xn;
    }
    __syncthreads();
    for (int s = 0; s < A.post; ++s) {
      narrow_pass(0);
      narrow_pass(1);
    }
    if (!has_wide && own_n) A.lv[l0].x[t] = xn;
  }

  // ---- wide level: correction from the narrow level, post-smoothing ----
  if (has_wide) {
    if (own_w) {
      const LevelView<T>& C = A.lv[l0 + 1];
      const int cnx = C.g.n[0], cny = C.g.n[1];
      const T e = xn;  // the parent (bi, bj) is this thread's narrow cell
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int I2 = second_parent(2 * bi + u, cnx, C.g.per[0]);
          const int J2 = second_parent(2 * bj + v, cny, C.g.per[1]);
          xw[v][u] += bilin(e, S[kSN + bj * cnx + I2], S[kSN + J2 * cnx + bi],
                            S[kSN + J2 * cnx + I2]);
          S[kSW + (2 * bj + v) * wnx + 2 * bi + u] = xw[v][u];
        }
    }
    __syncthreads();
    for (int s = 0; s < A.post; ++s) {
      wide_pass(0);
      wide_pass(1);
    }
    if (own_w) {
      const LevelView<T>& L = A.lv[l0];
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int u = 0; u < 2; ++u)
          L.x[(2 * bj + v) * wnx + 2 * bi + u] = xw[v][u];
    }
  }
}

namespace {

// ---- tails whose first level has 1025..4096 cells ----
//
// One block of 1024 threads.  The first level ("big") is owned as 2x2 cell
// blocks, thread t owning block t; the next two levels (257..1024 and
// 65..256 cells) one cell per thread; the tiny levels run in wave 0 as in
// tail2d_body.  Big thread t's block restricts onto cell t of the next
// level, which thread t owns, and that cell is the block's own parent in
// the prolongation, so neither transfer goes through LDS.  At this block
// size a thread has at most 128 registers: the tiny levels' weights wait in
// LDS, and the LDS copy of the big iterate serves as the residual scratch
// while the coarser levels run (the big level's prolongation rewrites it).
// Every operation and its rounding are those of the tiled down and up
// passes on the big level followed by tail2d_body on the rest.

constexpr int NTB = 1024;
constexpr int kBigMax = 4 * NTB;
constexpr int kSingles = 2;
constexpr int kGX = 0;                            // big iterate
constexpr int kGR = kGX;                          // residual scratch
constexpr int kG1 = kGX + kBigMax;                // first single level
constexpr int kG2 = kG1 + kWideMax;               // second single level
constexpr int kGT = kG2 + kNarrowMax;             // tiny iterates
constexpr int kGW = kGT + kTinyMax * kTinyCells;  // tiny weights, 6 a cell
constexpr int kGTotal = kGW + 6 * kTinyMax * kTinyCells;

}  // namespace

// Levels g[0..nt) fit k_tail2d_big: 2D with a red-black colouring, the
// first of 1025..4096 cells, every next one with both sides halved, and
// one to kTinyMax levels after the two single ones.
bool tail2d_big_fits(const Geom* g, int nt) {
  if (nt < 2 + kSingles || nt > 1 + kSingles + kTinyMax) return false;
  if (g[0].N <= kWideMax || g[0].N > kBigMax) return false;
  for (int j = 0; j < nt; ++j) {
    if (g[j].ndim != 2 || gs_colors(g[j]) != 2) return false;
    if (j > 0 && (g[j - 1].n[0] != 2 * g[j].n[0] ||
                  g[j - 1].n[1] != 2 * g[j].n[1]))
      return false;
  }
  return true;
}

template <typename T>
bool tail2d_big_ok(const TailArgs<T>& a) {
  if (a.whole || a.l0 < 0 || a.L > kMaxLevels || a.L - a.l0 < 1) return false;
  Geom g[kMaxLevels];
  for (int l = a.l0; l < a.L; ++l) g[l - a.l0] = a.lv[l].g;
  return tail2d_big_fits(g, a.L - a.l0);
}

namespace {

// Weights of a one-cell-per-thread level with the four LDS offsets packed
// in pairs (left | right << 16, below | above << 16; every offset of the
// layout is below 2^16).
template <typename T>
struct CellS {
  T wl, wr, wd, wu, inv, dn;
  int lr, du;
};
static_assert(kGTotal < (1 << 16), "LDS offsets fit 16 bits");

template <typename T>
__device__ __forceinline__ CellS<T> pack_cell(const CellW<T>& w) {
  CellS<T> c;
  c.wl = w.wl;
  c.wr = w.wr;
  c.wd = w.wd;
  c.wu = w.wu;
  c.inv = w.inv;
  c.dn = w.dn;
  c.lr = w.ol | (w.orr << 16);
  c.du = w.od | (w.ou << 16);
  return c;
}

template <typename T>
__global__ void __launch_bounds__(NTB) k_tail2d_big(TailArgs<T> A) {
  __shared__ T S[kGTotal];
  __shared__ int SO[4 * kTinyMax * kTinyCells];
  const int done = A.ctrl->done;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const bool wave0 = t < 64;
  const int l0 = A.l0;
  const int ntiny = A.L - l0 - 1 - kSingles;

  // ---- set-up loads, all issued before the stop flag is tested ----
  const LevelView<T>& Lb = A.lv[l0];
  const int bnx = Lb.g.n[0], hx = bnx / 2;
  const bool own_b = t < (int)Lb.g.N / 4;
  const int bi = own_b ? t % hx : 0, bj = own_b ? t / hx : 0;
  // the block's 12 distinct face coefficients (the faces between its own
  // cells are loaded once), as cell_alpha loads them
  CellA<T> ab[2][2];
  T xb[2][2], bb[2][2];
  {
    const int x0 = 2 * bi, y0 = 2 * bj;
    const int xl = x0 > 0 ? x0 - 1 : bnx - 1;
    const int yd = y0 > 0 ? y0 - 1 : Lb.g.n[1] - 1;
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int row = (y0 + v) * bnx;
      const T left = Lb.a[0][row + xl];
      const T r0 = Lb.a[0][row + x0], r1 = Lb.a[0][row + x0 + 1];
      ab[v][0].al = left;
      ab[v][0].ar = r0;
      ab[v][1].al = r0;
      ab[v][1].ar = r1;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const T down = Lb.a[1][yd * bnx + x0 + u];
      const T u0 = Lb.a[1][y0 * bnx + x0 + u];
      const T u1 = Lb.a[1][(y0 + 1) * bnx + x0 + u];
      ab[0][u].ad = down;
      ab[0][u].au = u0;
      ab[1][u].ad = u0;
      ab[1][u].au = u1;
    }
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int i = x0 + u, j = y0 + v;
        ab[v][u].i = i;
        ab[v][u].j = j;
        xb[v][u] = A.zero ? T(0) : Lb.x[j * bnx + i];
        bb[v][u] = Lb.b[j * bnx + i];
      }
  }
  const LevelView<T>& L1 = A.lv[l0 + 1];
  const bool own_1 = t < (int)L1.g.N;
  const int i1 = own_1 ? t % L1.g.n[0] : 0, j1 = own_1 ? t / L1.g.n[0] : 0;
  const CellA<T> a1 = cell_alpha(L1, i1, j1);
  const LevelView<T>& L2 = A.lv[l0 + 2];
  const bool own_2 = t < (int)L2.g.N;
  const int i2 = own_2 ? t % L2.g.n[0] : 0, j2 = own_2 ? t / L2.g.n[0] : 0;
  const CellA<T> a2 = cell_alpha(L2, i2, j2);
  // tiny cell (qw, lane) is set up by thread 64 qw + lane (waves 0..2);
  // wave 0 runs every tiny level
  bool own_t[kTinyMax];
#pragma unroll
  for (int q = 0; q < kTinyMax; ++q)
    own_t[q] = wave0 && q < ntiny &&
               lane < (int)A.lv[l0 + 1 + kSingles + min(q, ntiny - 1)].g.N;
  const int qw = min(t >> 6, ntiny - 1);
  const LevelView<T>& Lq = A.lv[l0 + 1 + kSingles + qw];
  const bool set_t = (t >> 6) < ntiny && lane < (int)Lq.g.N;
  const CellA<T> aq = cell_alpha(Lq, set_t ? lane % Lq.g.n[0] : 0,
                                 set_t ? lane / Lq.g.n[0] : 0);
  if (done != kRunning) return;

  // ---- weights; the tiny levels' go to LDS ----
  // big level: weights in registers; the neighbours outside the 2x2 block
  // by column (left of u = 0, right of u = 1) and row (below v = 0, above
  // v = 1), the block's own cell behind a Neumann wall as in cell_weights
  T bpb[2][2], wlb[2][2], wrb[2][2], wdb[2][2], wub[2][2], dnb[2][2];
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const CellW<T> w = cell_weights(Lb.g, ab[v][u], kGX);
      bpb[v][u] = bb[v][u] * w.inv;
      wlb[v][u] = w.wl;
      wrb[v][u] = w.wr;
      wdb[v][u] = w.wd;
      wub[v][u] = w.wu;
      dnb[v][u] = w.dn;
      if (!own_b) xb[v][u] = T(0);
    }
  int colb[2], rowb[2];
  {
    const int nx = bnx, ny = Lb.g.n[1], x0 = 2 * bi, y0 = 2 * bj;
    const int px = Lb.g.per[0], py = Lb.g.per[1];
    colb[0] = x0 > 0 ? x0 - 1 : (px ? nx - 1 : x0);
    colb[1] = x0 + 2 < nx ? x0 + 2 : (px ? 0 : x0 + 1);
    rowb[0] = y0 > 0 ? y0 - 1 : (py ? ny - 1 : y0);
    rowb[1] = y0 + 2 < ny ? y0 + 2 : (py ? 0 : y0 + 1);
  }
  // the iterate of the big level's neighbour of cell (u, v) on side
  // 0 left, 1 right, 2 below, 3 above
  auto big_nb = [&](int v, int u, int side) -> T {
    if (side == 0) return u ? xb[v][0] : S[kGX + (2 * bj + v) * bnx + colb[0]];
    if (side == 1) return u ? S[kGX + (2 * bj + v) * bnx + colb[1]] : xb[v][1];
    if (side == 2) return v ? xb[0][u] : S[kGX + rowb[0] * bnx + 2 * bi + u];
    return v ? S[kGX + rowb[1] * bnx + 2 * bi + u] : xb[1][u];
  };
  const CellS<T> c1 = pack_cell(cell_weights(L1.g, a1, kG1));
  const CellS<T> c2 = pack_cell(cell_weights(L2.g, a2, kG2));
  if ((t >> 6) < ntiny) {
    const CellW<T> w = cell_weights(Lq.g, aq, kGT + qw * kTinyCells);
    {
      T* W = S + kGW + qw * 6 * kTinyCells + lane;
      W[0] = w.wl;
      W[kTinyCells] = w.wr;
      W[2 * kTinyCells] = w.wd;
      W[3 * kTinyCells] = w.wu;
      W[4 * kTinyCells] = w.inv;
      W[5 * kTinyCells] = w.dn;
      int* O = SO + qw * 4 * kTinyCells + lane;
      O[0] = w.ol;
      O[kTinyCells] = w.orr;
      O[2 * kTinyCells] = w.od;
      O[3 * kTinyCells] = w.ou;
    }
  }
  if (own_b) {
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int u = 0; u < 2; ++u)
        S[kGX + (2 * bj + v) * bnx + 2 * bi + u] = xb[v][u];
  }
  __syncthreads();

  // ---- big level: pre-smoothing, residual restricted onto cell t ----
  auto big_pass = [&](int c) {
    if (own_b) {
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          if (((u + v) & 1) != c) continue;
          xb[v][u] = gs_val(bpb[v][u], wlb[v][u], big_nb(v, u, 0), wrb[v][u],
                            big_nb(v, u, 1), wdb[v][u], big_nb(v, u, 2),
                            wub[v][u], big_nb(v, u, 3));
          S[kGX + (2 * bj + v) * bnx + 2 * bi + u] = xb[v][u];
        }
    }
    __syncthreads();
  };
  for (int s = 0; s < A.pre; ++s) {
    big_pass(0);
    big_pass(1);
  }
  T b1 = T(0);
  if (own_b) {
    T r[2][2];
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int u = 0; u < 2; ++u)
        r[v][u] = dnb[v][u] * (gs_val(bpb[v][u], wlb[v][u], big_nb(v, u, 0),
                                      wrb[v][u], big_nb(v, u, 1), wdb[v][u],
                                      big_nb(v, u, 2), wub[v][u],
                                      big_nb(v, u, 3)) -
                               xb[v][u]);
    b1 = T(0.25) * ((r[0][0] + r[0][1]) + (r[1][0] + r[1][1]));
  }

  // ---- single levels: cell t, x from zero ----
  auto single_pass = [&](bool own, const CellS<T>& w, T bp, T& x, int base,
                         int color, int c) {
    if (own && color == c) {
      x = gs_val(bp, w.wl, S[w.lr & 0xffff], w.wr, S[w.lr >> 16], w.wd,
                 S[w.du & 0xffff], w.wu, S[w.du >> 16]);
      S[base + t] = x;
    }
    __syncthreads();
  };
  auto single_resid = [&](const CellS<T>& w, T bp, T x) {
    return w.dn * (gs_val(bp, w.wl, S[w.lr & 0xffff], w.wr, S[w.lr >> 16],
                          w.wd, S[w.du & 0xffff], w.wu, S[w.du >> 16]) -
                   x);
  };
  T x1 = T(0);
  const T bp1 = b1 * c1.inv;
  const int col1 = (i1 + j1) & 1;
  if (own_1) S[kG1 + t] = T(0);
  __syncthreads();  // also: the big residual's reads precede the scratch
  for (int s = 0; s < A.pre; ++s) {
    single_pass(own_1, c1, bp1, x1, kG1, col1, 0);
    single_pass(own_1, c1, bp1, x1, kG1, col1, 1);
  }
  if (own_1) S[kGR + t] = single_resid(c1, bp1, x1);
  __syncthreads();

  T x2 = T(0), b2 = T(0);
  if (own_2) {
    const int fnx = L1.g.n[0];
    const int f0 = 2 * j2 * fnx + 2 * i2;
    b2 = T(0.25) * ((S[kGR + f0] + S[kGR + f0 + 1]) +
                    (S[kGR + f0 + fnx] + S[kGR + f0 + fnx + 1]));
    S[kG2 + t] = T(0);
  }
  const T bp2 = b2 * c2.inv;
  const int col2 = (i2 + j2) & 1;
  __syncthreads();
  for (int s = 0; s < A.pre; ++s) {
    single_pass(own_2, c2, bp2, x2, kG2, col2, 0);
    single_pass(own_2, c2, bp2, x2, kG2, col2, 1);
  }
  if (own_2) S[kGR + t] = single_resid(c2, bp2, x2);
  __syncthreads();

  // ---- tiny levels: wave 0 alone ----
  // Weights, offsets and b/d are read from LDS at every update (kept in
  // registers they would push the block past 128 registers a thread).
  if (wave0) {
    // Gauss-Seidel value of lane's cell on tiny level q (b/d in slot 4)
    auto tiny_gs = [&](int q) {
      const T* W = S + kGW + q * 6 * kTinyCells + lane;
      const int* O = SO + q * 4 * kTinyCells + lane;
      return gs_val(W[4 * kTinyCells], W[0], S[O[0]], W[kTinyCells],
                    S[O[kTinyCells]], W[2 * kTinyCells], S[O[2 * kTinyCells]],
                    W[3 * kTinyCells], S[O[3 * kTinyCells]]);
    };
    auto tiny_pass = [&](int q, int color, int c) {
      if (own_t[q] && color == c)
        S[kGT + q * kTinyCells + lane] = tiny_gs(q);
      wave_lds_sync();
    };
    auto tiny_resid = [&](int q) {
      return S[kGW + (q * 6 + 5) * kTinyCells + lane] *
             (tiny_gs(q) - S[kGT + q * kTinyCells + lane]);
    };
#pragma unroll
    for (int q = 0; q < kTinyMax; ++q) {
      if (q >= ntiny) break;
      const LevelView<T>& L = A.lv[l0 + 1 + kSingles + q];
      const int ti = lane % L.g.n[0], tj = lane / L.g.n[0];
      // rhs: mean of the four children's residuals (scratch), x = 0; b/d
      // replaces 1/d in slot 4
      T bt = T(0);
      if (own_t[q]) {
        const int fnx = A.lv[l0 + kSingles + q].g.n[0];
        const int f0 = 2 * tj * fnx + 2 * ti;
        bt = T(0.25) * ((S[kGR + f0] + S[kGR + f0 + 1]) +
                        (S[kGR + f0 + fnx] + S[kGR + f0 + fnx + 1]));
      }
      T* slot = S + kGW + (q * 6 + 4) * kTinyCells + lane;
      *slot = bt * *slot;
      S[kGT + q * kTinyCells + lane] = T(0);
      wave_lds_sync();
      const int color = (ti + tj) & 1;
      if (q < ntiny - 1) {
        for (int s = 0; s < A.pre; ++s) {
          tiny_pass(q, color, 0);
          tiny_pass(q, color, 1);
        }
        if (own_t[q]) S[kGR + lane] = tiny_resid(q);
        wave_lds_sync();
      } else {
        // coarsest: sweeps from zero until the residual dropped by 1e-3
        const double b = own_t[q] ? (double)bt : 0.0;
        const double r0 = wave_sum(b * b);
        auto r2 = [&]() {
          double v = 0.0;
          if (own_t[q]) {
            const double r = (double)tiny_resid(q);
            v = r * r;
          }
          return wave_sum(v);
        };
        auto sweeps2 = [&]() {
          for (int s = 0; s < 2; ++s) {
            tiny_pass(q, color, 0);
            tiny_pass(q, color, 1);
          }
        };
        sweeps2();
        if (r2() > 1e-6 * r0) {  // squared norms
          for (int it = 0; it < 4000; it += 2) {
            sweeps2();
            if (!(r2() > 1e-6 * r0)) break;
          }
        }
      }
    }
    // up through the tiny levels
#pragma unroll
    for (int q = kTinyMax - 2; q >= 0; --q) {
      if (q + 1 >= ntiny) continue;
      const LevelView<T>& L = A.lv[l0 + 1 + kSingles + q];
      const LevelView<T>& C = A.lv[l0 + 2 + kSingles + q];
      const int ti = lane % L.g.n[0], tj = lane / L.g.n[0];
      const int cbase = kGT + (q + 1) * kTinyCells;
      if (own_t[q]) {
        const int cnx = C.g.n[0], cny = C.g.n[1];
        const int I = ti >> 1, J = tj >> 1;
        const int I2 = second_parent(ti, cnx, C.g.per[0]);
        const int J2 = second_parent(tj, cny, C.g.per[1]);
        S[kGT + q * kTinyCells + lane] +=
            bilin(S[cbase + J * cnx + I], S[cbase + J * cnx + I2],
                  S[cbase + J2 * cnx + I], S[cbase + J2 * cnx + I2]);
      }
      wave_lds_sync();
      const int color = (ti + tj) & 1;
      for (int s = 0; s < A.post; ++s) {
        tiny_pass(q, color, 0);
        tiny_pass(q, color, 1);
      }
    }
  }
  __syncthreads();

  // ---- single levels: correction from the next coarser, post-smoothing
  auto correct = [&](bool own, int i, int j, const Geom& gc, int cbase, T& x,
                     int base) {
    if (own) {
      const int cnx = gc.n[0], cny = gc.n[1];
      const int I = i >> 1, J = j >> 1;
      const int I2 = second_parent(i, cnx, gc.per[0]);
      const int J2 = second_parent(j, cny, gc.per[1]);
      x += bilin(S[cbase + J * cnx + I], S[cbase + J * cnx + I2],
                 S[cbase + J2 * cnx + I], S[cbase + J2 * cnx + I2]);
      S[base + t] = x;
    }
    __syncthreads();
  };
  correct(own_2, i2, j2, A.lv[l0 + 1 + kSingles].g, kGT, x2, kG2);
  for (int s = 0; s < A.post; ++s) {
    single_pass(own_2, c2, bp2, x2, kG2, col2, 0);
    single_pass(own_2, c2, bp2, x2, kG2, col2, 1);
  }
  correct(own_1, i1, j1, L2.g, kG2, x1, kG1);
  for (int s = 0; s < A.post; ++s) {
    single_pass(own_1, c1, bp1, x1, kG1, col1, 0);
    single_pass(own_1, c1, bp1, x1, kG1, col1, 1);
  }

  // ---- big level: correction (its own parent is x1), post-smoothing ----
  if (own_b) {
    const int cnx = L1.g.n[0], cny = L1.g.n[1];
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int I2 = second_parent(2 * bi + u, cnx, L1.g.per[0]);
        const int J2 = second_parent(2 * bj + v, cny, L1.g.per[1]);
        xb[v][u] += bilin(x1, S[kG1 + bj * cnx + I2], S[kG1 + J2 * cnx + bi],
                          S[kG1 + J2 * cnx + I2]);
        S[kGX + (2 * bj + v) * bnx + 2 * bi + u] = xb[v][u];
      }
  }
  __syncthreads();
  for (int s = 0; s < A.post; ++s) {
    big_pass(0);
    big_pass(1);
  }
  if (own_b) {
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int u = 0; u < 2; ++u)
        Lb.x[(2 * bj + v) * bnx + 2 * bi + u] = xb[v][u];
  }
}

}  // namespace

template <typename T>
hipError_t launch_tail2d_big(const TailArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((k_tail2d_big<T>), dim3(1), dim3(NTB), 0, s, a);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(NT2) k_tail2d(TailArgs<T> A) {
  tail2d_body<T>(A);
}

template <typename T>
__global__ void __launch_bounds__(NT2)
    k_tail2d_batch(const TailArgs<T>* __restrict__ tab) {
  tail2d_body<T>(tab[blockIdx.x]);
}

template <typename T>
hipError_t launch_tail2d(const TailArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((k_tail2d<T>), dim3(1), dim3(NT2), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tail2d_batch(const TailArgs<T>* tab, int ng, hipStream_t s) {
  if (ng == 0) return hipSuccess;
  hipLaunchKernelGGL((k_tail2d_batch<T>), dim3(ng), dim3(NT2), 0, s, tab);
  return hipGetLastError();
}

template bool tail2d_ok<double>(const TailArgs<double>&);
template bool tail2d_big_ok<double>(const TailArgs<double>&);
template bool tail2d_big_ok<float>(const TailArgs<float>&);
template hipError_t launch_tail2d_big<double>(const TailArgs<double>&,
                                              hipStream_t);
template hipError_t launch_tail2d_big<float>(const TailArgs<float>&,
                                             hipStream_t);
template bool tail2d_ok<float>(const TailArgs<float>&);
template hipError_t launch_tail2d<double>(const TailArgs<double>&, hipStream_t);
template hipError_t launch_tail2d<float>(const TailArgs<float>&, hipStream_t);
template hipError_t launch_tail2d_batch<double>(const TailArgs<double>*, int,
                                                hipStream_t);
template hipError_t launch_tail2d_batch<float>(const TailArgs<float>*, int,
                                               hipStream_t);

}  // namespace fld
