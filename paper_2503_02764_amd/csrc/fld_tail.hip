// Single-workgroup multigrid tail in LDS (gfx950).
//
// Levels of at most kTailLdsCells (= kReduceBlock) cells are solved by one
// block of kReduceBlock threads: the face coefficients of every tail level,
// the packed cell coordinates, the right-hand side of the first level and
// all iterates live in LDS;
// thread t owns cell t of each level, and the phases of the sub-V-cycle
// (red-black smoothing, residual and 2^d restriction fused, coarsest
// red-black iteration, prolongation) are separated by block barriers only.
// The level loops are ordinary runtime loops over a level table in LDS, so
// the kernel stays small and spill-free; a phase costs a few LDS round
// trips and a barrier.  All global loads of the set-up are issued before the
// first is used.  Indices are 32-bit offsets into one LDS array.
//
// Non-whole mode: one sub-V-cycle from level l0 (x(l0) zero or read), the
// result x(l0) written back.  Whole mode (the whole problem fits): the cycle
// loop with the stop test runs here too, exactly as in the multi-launch
// path: pre-smoothing, residual norm of the finest level, stop or continue.
#include "fld_internal.h"
#include "fld_wave.h"

namespace fld {

namespace {

constexpr int kMaxTail = 10;  // tail levels handled in LDS
constexpr int NTH = kReduceBlock;
static_assert(kTailLdsCells <= NTH, "one cell per thread");

struct TL {
  int n[3];
  int per[3];
  int N;
  int ox, ob, oi, oa[3];  // offsets (elements of T) of x, b, -, faces
  int oc;                 // offset (ints) of the packed coordinates
};

// coordinates packed 10 bits each (sides <= 1024)
__device__ __forceinline__ void unpack(int p, int c[3]) {
  c[0] = p & 1023;
  c[1] = (p >> 10) & 1023;
  c[2] = p >> 20;
}

// sum over the faces of cell i of alpha * x_neighbour, and of alpha
template <typename T, int ND>
__device__ __forceinline__ void gather(const T* S, const TL& t, int i,
                                       const int c[3], T& sax, T& sa) {
  int st = 1;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const int n = t.n[d];
    T al = T(0);
    int nl = i;
    if (c[d] > 0) {
      nl = i - st;
      al = S[t.oa[d] + nl];
    } else if (t.per[d]) {
      nl = i + (n - 1) * st;
      al = S[t.oa[d] + nl];
    }
    const T au = S[t.oa[d] + i];
    int nu = i;
    if (c[d] < n - 1)
      nu = i + st;
    else if (t.per[d])
      nu = i - (n - 1) * st;
    sax += al * S[t.ox + nl] + au * S[t.ox + nu];
    sa += al + au;
    st *= n;
  }
}

template <typename T, int ND>
__device__ __forceinline__ T resid_at(const T* S, const TL& t, int i,
                                      const int c[3]) {
  T sax = T(0), sa = T(0);
  gather<T, ND>(S, t, i, c, sax, sa);
  const T xi = S[t.ox + i];
  return S[t.ob + i] - (xi + sa * xi - sax);
}

// sum of v over the block, returned to every thread
__device__ __forceinline__ double tail_block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int q = 0; q < NTH / 64; ++q) r += sh[q];
  return r;
}

// (the level descriptor is copied into registers once per call: LDS
// contents may change at every barrier, so the compiler would reload it)
template <typename T, int ND>
__device__ __forceinline__ void smooth(T* S, const int* C, const TL& tls,
                                    int sweeps) {
  const TL t = tls;
  const int i = threadIdx.x;
  int c[3] = {0, 0, 0};
  if (i < t.N) unpack(C[t.oc + i], c);
  const int color = gs_color(t, c);
  const int ncol = gs_colors(t);
  for (int s = 0; s < sweeps; ++s)
    for (int col = 0; col < ncol; ++col) {
      if (i < t.N && color == col) {
        T sax = T(0), sa = T(0);
        gather<T, ND>(S, t, i, c, sax, sa);
        S[t.ox + i] = (S[t.ob + i] + sax) / (T(1) + sa);
      }
      __syncthreads();
    }
}

// coarse b = mean of the 2^d children's residuals (computed here), coarse
// x = 0; returns this thread's share of the fine |r|^2
template <typename T, int ND>
__device__ __forceinline__ double resid_restrict(T* S, const int* C,
                                              const TL& fs, const TL& ccs) {
  const TL f = fs, cc = ccs;
  constexpr int nd = ND;
  const int o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
  const int I = threadIdx.x;
  double r2 = 0.0;
  if (I < cc.N) {
    int k[3];
    unpack(C[cc.oc + I], k);
    T s = T(0);
    for (int q2 = 0; q2 < o2; ++q2)
      for (int q1 = 0; q1 < o1; ++q1)
        for (int q0 = 0; q0 < 2; ++q0) {
          const int fc[3] = {2 * k[0] + q0, nd > 1 ? 2 * k[1] + q1 : 0,
                             nd > 2 ? 2 * k[2] + q2 : 0};
          const int fi = fc[0] + f.n[0] * (fc[1] + f.n[1] * fc[2]);
          const T r = resid_at<T, ND>(S, f, fi, fc);
          s += r;
          r2 += (double)r * (double)r;
        }
    S[cc.ob + I] = s / T(2 * o1 * o2);
    S[cc.ox + I] = T(0);
  }
  __syncthreads();
  return r2;
}

template <typename T, int ND>
__device__ __forceinline__ void prolong(T* S, const int* C, const TL& ccs,
                                     const TL& fs) {
  const TL cc = ccs, f = fs;
  constexpr int nd = ND;
  const int i = threadIdx.x;
  if (i < f.N) {
    int fc[3];
    unpack(C[f.oc + i], fc);
    int p[3] = {0, 0, 0}, q[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < nd; ++d) {
      p[d] = fc[d] >> 1;
      int o = (fc[d] & 1) ? p[d] + 1 : p[d] - 1;
      if (o < 0) o = cc.per[d] ? cc.n[d] - 1 : 0;
      if (o >= cc.n[d]) o = cc.per[d] ? 0 : cc.n[d] - 1;
      q[d] = o;
    }
    const int o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
    T e = T(0);
    for (int s2 = 0; s2 < o2; ++s2)
      for (int s1 = 0; s1 < o1; ++s1)
        for (int s0 = 0; s0 < 2; ++s0) {
          const int ii = s0 ? q[0] : p[0];
          const int jj = s1 ? q[1] : p[1];
          const int kk = s2 ? q[2] : p[2];
          const T w = T((s0 ? 0.25 : 0.75) * (nd > 1 ? (s1 ? 0.25 : 0.75) : 1.0) *
                        (nd > 2 ? (s2 ? 0.25 : 0.75) : 1.0));
          e += w * S[cc.ox + ii + cc.n[0] * (jj + cc.n[1] * kk)];
        }
    S[f.ox + i] += e;
  }
  __syncthreads();
}

// this thread's |r|^2 on level t
template <typename T, int ND>
__device__ __forceinline__ double resid2(const T* S, const int* C,
                                         const TL& t) {
  const int i = threadIdx.x;
  if (i >= t.N) return 0.0;
  int c[3];
  unpack(C[t.oc + i], c);
  const double r = (double)resid_at<T, ND>(S, t, i, c);
  return r * r;
}

// sums of a and b over the block, returned to every thread
__device__ __forceinline__ void tail_block_sum2(double& a, double& b,
                                                double* sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sh[w] = a;
    sh[NTH / 64 + w] = b;
  }
  __syncthreads();
  a = b = 0.0;
#pragma unroll
  for (int q = 0; q < NTH / 64; ++q) {
    a += sh[q];
    b += sh[NTH / 64 + q];
  }
}

// Coarsest level: red-black Gauss-Seidel sweeps until the residual norm has
// dropped by 1e-3 from its value at entry (tested every 2 sweeps; at most
// 4000 sweeps).  With a zero start (x0_zero) that value is |b|, summed
// together with the first test.
template <typename T, int ND>
__device__ __forceinline__ void coarsest(T* S, const int* C, const TL& ts,
                                         double* sh, bool x0_zero) {
  const TL t = ts;
  double r0 = 0.0;
  if (x0_zero) {
    double b2 = 0.0;
    if ((int)threadIdx.x < t.N) {
      const double b = (double)S[t.ob + threadIdx.x];
      b2 = b * b;
    }
    smooth<T, ND>(S, C, t, 2);
    double r2 = resid2<T, ND>(S, C, t);
    tail_block_sum2(b2, r2, sh);
    r0 = b2;
    if (!(r2 > 1e-6 * r0)) return;  // squared norms
  } else {
    r0 = tail_block_sum(resid2<T, ND>(S, C, t), sh);
    if (!(r0 > 0.0)) return;
  }
  for (int it = 0; it < 4000; it += 2) {
    smooth<T, ND>(S, C, t, 2);
    const double rn = tail_block_sum(resid2<T, ND>(S, C, t), sh);
    if (!(rn > 1e-6 * r0)) break;
  }
}

// sub-V-cycle over tail levels j0 .. nt-1 (tl[j] = level l0 + j)
template <typename T, int ND>
__device__ __forceinline__ void subcycle(T* S, const int* C, const TL* tl,
                                         int nt, int j0, int pre, int post,
                                         double* sh) {
  for (int j = j0; j + 1 < nt; ++j) {
    smooth<T, ND>(S, C, tl[j], pre);
    (void)resid_restrict<T, ND>(S, C, tl[j], tl[j + 1]);
  }
  coarsest<T, ND>(S, C, tl[nt - 1], sh, nt > 1 || j0 > 0);
  for (int j = nt - 2; j >= j0; --j) {
    prolong<T, ND>(S, C, tl[j + 1], tl[j]);
    smooth<T, ND>(S, C, tl[j], post);
  }
}

// LDS bytes of the level arrays (T region, then the packed coordinates)
__host__ __device__ inline size_t tail_bytes_of(const Geom* g, int nt,
                                                size_t tsize) {
  size_t cells = 0, ints = 0;
  for (int j = 0; j < nt; ++j) {
    cells += (size_t)g[j].N * (2 + g[j].ndim);
    ints += (size_t)g[j].N;
  }
  return cells * tsize + ints * sizeof(int);
}

}  // namespace

template <typename T, int ND>
__device__ __forceinline__ void tail_lds_body(const TailArgs<T>& A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double sh[2 * (NTH / 64)];
  __shared__ TL tl[kMaxTail];
  __shared__ int stop;
  if (A.ctrl->done != kRunning) return;
  T* S = (T*)smem_raw;
  const int l0 = A.l0;
  const int nt = A.L - l0;  // number of tail levels (<= kMaxTail)
  const int i = threadIdx.x;
  if (i == 0) {
    int o = 0;
    for (int j = 0; j < nt; ++j) {
      const Geom& g = A.lv[l0 + j].g;
      TL& t = tl[j];
      for (int d = 0; d < 3; ++d) {
        t.n[d] = g.n[d];
        t.per[d] = g.per[d];
      }
      t.N = (int)g.N;
      t.ox = o;
      o += t.N;
      t.ob = o;
      o += t.N;
      t.oi = -1;
      for (int d = 0; d < 3; ++d) {
        t.oa[d] = o;
        if (d < ND) o += t.N;
      }
    }
    int oc = 0;
    for (int j = 0; j < nt; ++j) {
      tl[j].oc = oc;
      oc += tl[j].N;
    }
    stop = o;  // start of the int region, in elements of T
  }
  // this thread's elements of the level-l0 rhs and iterate
  const int N0 = (int)A.lv[l0].g.N;
  T vb = T(0), vx = T(0);
  if (i < N0) {
    vb = A.lv[l0].b[i];
    vx = A.zero ? T(0) : A.lv[l0].x[i];
  }
  // face coefficients of the first levels, loaded before any is stored
  constexpr int kPre = 4;
  T pa[kPre][ND];
#pragma unroll
  for (int j = 0; j < kPre; ++j)
#pragma unroll
    for (int d = 0; d < ND; ++d)
      pa[j][d] = (j < nt && i < (int)A.lv[l0 + j].g.N) ? A.lv[l0 + j].a[d][i]
                                                       : T(0);
  __syncthreads();
  int* C = (int*)(S + stop);
#pragma unroll
  for (int j = 0; j < kPre; ++j)
    if (j < nt && i < tl[j].N)
#pragma unroll
      for (int d = 0; d < ND; ++d) S[tl[j].oa[d] + i] = pa[j][d];
  for (int j = 0; j < nt; ++j) {
    const TL& t = tl[j];
    if (i < t.N) {
      if (j >= kPre)
        for (int d = 0; d < ND; ++d) S[t.oa[d] + i] = A.lv[l0 + j].a[d][i];
      const int c0 = i % t.n[0], r = i / t.n[0];
      C[t.oc + i] = c0 | ((r % t.n[1]) << 10) | ((r / t.n[1]) << 20);
    }
  }
  if (i < N0) {
    S[tl[0].ob + i] = vb;
    S[tl[0].ox + i] = vx;
  }
  __syncthreads();
  if (!A.whole) {
    subcycle<T, ND>(S, C, tl, nt, 0, A.pre, A.post, sh);
  } else {
    for (;;) {
      double r2;
      if (nt > 1) {
        smooth<T, ND>(S, C, tl[0], A.pre);
        r2 = resid_restrict<T, ND>(S, C, tl[0], tl[1]);
      } else {
        coarsest<T, ND>(S, C, tl[0], sh, false);
        r2 = resid2<T, ND>(S, C, tl[0]);
      }
      const double s = tail_block_sum(r2, sh);
      if (threadIdx.x == 0) {
        Control* Cb = A.ctrl;
        const double r = sqrt(s / Cb->bnorm2);
        Cb->res = r;
        Cb->cycles += 1;
        if (r <= Cb->rtol)
          Cb->done = kConverged;
        else if (Cb->cycles >= Cb->max_cycles)
          Cb->done = kCapped;
        sh[0] = Cb->done != kRunning ? 1.0 : 0.0;
        if (Cb->done != kRunning && Cb->mirror) *Cb->mirror = *Cb;
      }
      __syncthreads();
      const bool halt = sh[0] != 0.0;
      __syncthreads();
      if (halt) break;
      if (nt > 1) {
        subcycle<T, ND>(S, C, tl, nt, 1, A.pre, A.post, sh);
        prolong<T, ND>(S, C, tl[1], tl[0]);
        smooth<T, ND>(S, C, tl[0], A.post);
      }
    }
  }
  // write back x(l0)
  if (i < N0) A.lv[l0].x[i] = S[tl[0].ox + i];
}

template <typename T, int ND>
__global__ void __launch_bounds__(NTH) k_tail_lds(TailArgs<T> A) {
  tail_lds_body<T, ND>(A);
}

// Batched form: block g runs the tail of grid g (arguments in device memory).
template <typename T, int ND>
__global__ void __launch_bounds__(NTH)
    k_tail_lds_batch(const TailArgs<T>* __restrict__ tab) {
  tail_lds_body<T, ND>(tab[blockIdx.x]);
}

template <typename T>
size_t tail_lds_bytes(const TailArgs<T>& a) {
  const int nt = a.L - a.l0;
  if (a.lv[a.l0].g.N > kTailLdsCells || nt > kMaxTail) return 0;
  Geom g[kMaxTail];
  for (int j = 0; j < nt; ++j) g[j] = a.lv[a.l0 + j].g;
  return tail_bytes_of(g, nt, sizeof(T));
}

template <typename T>
hipError_t launch_tail_lds(const TailArgs<T>& a, hipStream_t s, bool* used) {
  if (tail2d_ok(a)) {
    *used = true;
    return launch_tail2d(a, s);
  }
  if (tail2d_big_ok(a)) {
    *used = true;
    return launch_tail2d_big(a, s);
  }
  const size_t lds = tail_lds_bytes(a);
  *used = lds > 0 && lds <= 62 * 1024;
  if (!*used) return hipSuccess;
  const int nd = a.lv[a.l0].g.ndim;
  if (nd == 1)
    hipLaunchKernelGGL((k_tail_lds<T, 1>), dim3(1), dim3(NTH), lds, s, a);
  else if (nd == 2)
    hipLaunchKernelGGL((k_tail_lds<T, 2>), dim3(1), dim3(NTH), lds, s, a);
  else
    hipLaunchKernelGGL((k_tail_lds<T, 3>), dim3(1), dim3(NTH), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tail_lds_batch(const TailArgs<T>* tab, int ng, int nd,
                                 size_t lds, hipStream_t s) {
  if (ng == 0) return hipSuccess;
  if (nd == 1)
    hipLaunchKernelGGL((k_tail_lds_batch<T, 1>), dim3(ng), dim3(NTH), lds, s, tab);
  else if (nd == 2)
    hipLaunchKernelGGL((k_tail_lds_batch<T, 2>), dim3(ng), dim3(NTH), lds, s, tab);
  else
    hipLaunchKernelGGL((k_tail_lds_batch<T, 3>), dim3(ng), dim3(NTH), lds, s, tab);
  return hipGetLastError();
}

template size_t tail_lds_bytes<double>(const TailArgs<double>&);
template size_t tail_lds_bytes<float>(const TailArgs<float>&);
template hipError_t launch_tail_lds_batch<double>(const TailArgs<double>*, int,
                                                  int, size_t, hipStream_t);
template hipError_t launch_tail_lds_batch<float>(const TailArgs<float>*, int,
                                                 int, size_t, hipStream_t);
template hipError_t launch_tail_lds<double>(const TailArgs<double>&,
                                            hipStream_t, bool*);
template hipError_t launch_tail_lds<float>(const TailArgs<float>&, hipStream_t,
                                           bool*);

}  // namespace fld
