// Single-workgroup multigrid tail in LDS (gfx950).
//
// Levels of at most kTailLdsCells cells are solved by one block of
// kReduceBlock threads: the face coefficients of every tail level, the
// right-hand side of the first one and all iterates are copied into LDS,
// thread t owns cell t of each level, and the phases of the sub-V-cycle
// (red-black smoothing, residual, 2^d restriction, coarsest Jacobi,
// prolongation) are separated by block barriers only.  Indices are 32-bit
// offsets into one LDS array, so every access is a plain LDS access.
//
// Non-whole mode: one sub-V-cycle from level l0 (x(l0) zero or read), the
// result x(l0) written back.  Whole mode (the whole problem fits): the cycle
// loop with the stop test runs here too, exactly as in the multi-launch
// path: pre-smoothing, residual norm of the finest level, stop or continue.
#include "fld_internal.h"

namespace fld {

namespace {

constexpr int kMaxTail = 10;  // tail levels handled in LDS

struct TL {
  int n[3];
  int per[3];
  int N;
  int ox, ob, oa[3];  // offsets (elements) of x, b and the face arrays
};

__device__ __forceinline__ void cell_coords(const TL& t, int i, int c[3]) {
  c[0] = i % t.n[0];
  const int r = i / t.n[0];
  c[1] = r % t.n[1];
  c[2] = r / t.n[1];
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

__device__ __forceinline__ double tail_block_sum(double v, double* sh,
                                                 double* out) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int q = 0; q < kReduceBlock / 64; ++q) r += sh[q];
    *out = r;
  }
  __syncthreads();
  return *out;
}

// Per-thread, per-level constants: cell coordinates and 1 / (1 + sum alpha).
template <typename T>
struct Own {
  int c[3];
  T inv;
};

template <typename T, int ND>
__device__ __forceinline__ void smooth(T* S, const TL& t, int sweeps,
                       const Own<T>& o) {
  const int i = threadIdx.x;
  const int color = (o.c[0] + o.c[1] + o.c[2]) & 1;
  for (int s = 0; s < sweeps; ++s)
    for (int col = 0; col < 2; ++col) {
      if (i < t.N && color == col) {
        T sax = T(0), sa = T(0);
        gather<T, ND>(S, t, i, o.c, sax, sa);
        S[t.ox + i] = (S[t.ob + i] + sax) * o.inv;
      }
      __syncthreads();
    }
}

// r of level t into R; returns this thread's r^2
template <typename T, int ND>
__device__ __forceinline__ double residual(T* S, const TL& t, T* R,
                                           const Own<T>& o) {
  const int i = threadIdx.x;
  double r2 = 0.0;
  if (i < t.N) {
    const int* c = o.c;
    T sax = T(0), sa = T(0);
    gather<T, ND>(S, t, i, c, sax, sa);
    const T xi = S[t.ox + i];
    const T r = S[t.ob + i] - (xi + sa * xi - sax);
    R[i] = r;
    r2 = (double)r * (double)r;
  }
  __syncthreads();
  return r2;
}

// coarse b = mean of the 2^d children in R, coarse x = 0
template <typename T, int ND>
__device__ __forceinline__ void restrict_to(T* S, const TL& f, const TL& cc,
                                            const T* R) {
  constexpr int nd = ND;
  const int I = threadIdx.x;
  if (I < cc.N) {
    int c[3];
    cell_coords(cc, I, c);
    const int o1 = nd > 1 ? 2 : 1, o2 = nd > 2 ? 2 : 1;
    T s = T(0);
    for (int q2 = 0; q2 < o2; ++q2)
      for (int q1 = 0; q1 < o1; ++q1)
        for (int q0 = 0; q0 < 2; ++q0) {
          const int fi = (2 * c[0] + q0) +
                         f.n[0] * ((nd > 1 ? 2 * c[1] + q1 : 0) +
                                   f.n[1] * (nd > 2 ? 2 * c[2] + q2 : 0));
          s += R[fi];
        }
    S[cc.ob + I] = s / T(2 * o1 * o2);
    S[cc.ox + I] = T(0);
  }
  __syncthreads();
}

template <typename T, int ND>
__device__ __forceinline__ void prolong(T* S, const TL& cc, const TL& f) {
  constexpr int nd = ND;
  const int i = threadIdx.x;
  if (i < f.N) {
    int fc[3];
    cell_coords(f, i, fc);
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

// Jacobi until the residual norm dropped by 1e-6 (at most 4000 sweeps)
template <typename T, int ND>
__device__ __forceinline__ void coarsest(T* S, const TL& t, T* R, double* sh,
                                         double* red, const Own<T>& o) {
  const int i = threadIdx.x;
  const int* c = o.c;
  double r0 = 0.0;
  for (int it = 0; it < 4000; ++it) {
    T sax = T(0), sa = T(0);
    if (i < t.N) gather<T, ND>(S, t, i, c, sax, sa);
    if ((it & 7) == 0) {
      double v = 0.0;
      if (i < t.N) {
        const T xi = S[t.ox + i];
        const double r = (double)(S[t.ob + i] - (xi + sa * xi - sax));
        v = r * r;
      }
      const double rn = tail_block_sum(v, sh, red);
      if (it == 0) r0 = rn;
      if (!(rn > 1e-12 * r0)) break;
    }
    if (i < t.N) R[i] = (S[t.ob + i] + sax) * o.inv;
    __syncthreads();
    if (i < t.N) S[t.ox + i] = R[i];
    __syncthreads();
  }
}

// sub-V-cycle over tail levels j0 .. nt-1 (level l0 + j)
template <typename T, int ND>
__device__ __forceinline__ void subcycle(T* S, const TL* tl, int l0, int nt,
                                         int j0, int pre, int post,
                                         T* R, double* sh, double* red,
                                         const Own<T> (&own)[kMaxTail]) {
#pragma unroll
  for (int j = 0; j < kMaxTail - 1; ++j)
    if (j >= j0 && j + 1 < nt) {
      smooth<T, ND>(S, tl[l0 + j], pre, own[j]);
      (void)residual<T, ND>(S, tl[l0 + j], R, own[j]);
      restrict_to<T, ND>(S, tl[l0 + j], tl[l0 + j + 1], R);
    }
#pragma unroll
  for (int j = 0; j < kMaxTail; ++j)
    if (j == nt - 1) coarsest<T, ND>(S, tl[l0 + j], R, sh, red, own[j]);
#pragma unroll
  for (int j = kMaxTail - 2; j >= 0; --j)
    if (j >= j0 && j + 1 < nt) {
      prolong<T, ND>(S, tl[l0 + j + 1], tl[l0 + j]);
      smooth<T, ND>(S, tl[l0 + j], post, own[j]);
    }
}

}  // namespace

template <typename T, int ND>
__device__ __forceinline__ void tail_lds_body(const TailArgs<T>& A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double sh[kReduceBlock / 64];
  __shared__ double red;
  __shared__ TL tl[kMaxLevels];
  __shared__ int stop;
  __shared__ int roff;
  if (A.ctrl->done != kRunning) return;
  T* S = (T*)smem_raw;
  const int l0 = A.l0, L = A.L;
  constexpr int nd = ND;
  if (threadIdx.x == 0) {
    int o = 0;
    for (int l = l0; l < L; ++l) {
      TL& t = tl[l];
      for (int d = 0; d < 3; ++d) {
        t.n[d] = A.lv[l].g.n[d];
        t.per[d] = A.lv[l].g.per[d];
      }
      t.N = (int)A.lv[l].g.N;
      t.ox = o;
      o += t.N;
      t.ob = o;
      o += t.N;
      for (int d = 0; d < 3; ++d) {
        t.oa[d] = o;
        if (d < nd) o += t.N;
      }
    }
    roff = o;  // residual scratch after the level arrays
  }
  __syncthreads();
  T* R = S + roff;
  // load the face coefficients of every tail level, b and x of level l0
  for (int l = l0; l < L; ++l) {
    const TL& t = tl[l];
    for (int d = 0; d < nd; ++d)
      for (int i = threadIdx.x; i < t.N; i += kReduceBlock)
        S[t.oa[d] + i] = A.lv[l].a[d][i];
  }
  {
    const TL& t = tl[l0];
    for (int i = threadIdx.x; i < t.N; i += kReduceBlock) {
      S[t.ob + i] = A.lv[l0].b[i];
      S[t.ox + i] = A.zero ? T(0) : A.lv[l0].x[i];
    }
  }
  __syncthreads();

  // per-thread constants of every tail level (static indices: unrolled)
  Own<T> own[kMaxTail];
#pragma unroll
  for (int j = 0; j < kMaxTail; ++j) {
    own[j].c[0] = own[j].c[1] = own[j].c[2] = 0;
    own[j].inv = T(1);
    const int l = l0 + j;
    if (l < L && (int)threadIdx.x < tl[l].N) {
      cell_coords(tl[l], threadIdx.x, own[j].c);
      T sax = T(0), sa = T(0);
      gather<T, ND>(S, tl[l], threadIdx.x, own[j].c, sax, sa);
      own[j].inv = T(1) / (T(1) + sa);
    }
  }
  const int nt = L - l0;  // number of tail levels (<= kMaxTail)
  if (!A.whole) {
    subcycle<T, ND>(S, tl, l0, nt, 0, A.pre, A.post, R, sh, &red, own);
  } else {
    for (;;) {
      double r2;
      if (nt > 1) {
        smooth<T, ND>(S, tl[0], A.pre, own[0]);
        r2 = residual<T, ND>(S, tl[0], R, own[0]);
      } else {
        coarsest<T, ND>(S, tl[0], R, sh, &red, own[0]);
        r2 = residual<T, ND>(S, tl[0], R, own[0]);
      }
      const double s = tail_block_sum(r2, sh, &red);
      if (threadIdx.x == 0) {
        Control* C = A.ctrl;
        const double r = sqrt(s / C->bnorm2);
        C->res = r;
        C->cycles += 1;
        if (r <= C->rtol)
          C->done = kConverged;
        else if (C->cycles >= C->max_cycles)
          C->done = kCapped;
        stop = C->done != kRunning;
        if (stop && C->mirror) *C->mirror = *C;
      }
      __syncthreads();
      if (stop) break;
      if (nt > 1) {
        restrict_to<T, ND>(S, tl[0], tl[1], R);
        subcycle<T, ND>(S, tl, l0, nt, 1, A.pre, A.post, R, sh, &red, own);
        prolong<T, ND>(S, tl[1], tl[0]);
        smooth<T, ND>(S, tl[0], A.post, own[0]);
      }
    }
  }
  // write back x(l0)
  {
    const TL& t = tl[l0];
    for (int i = threadIdx.x; i < t.N; i += kReduceBlock)
      A.lv[l0].x[i] = S[t.ox + i];
  }
}

template <typename T, int ND>
__global__ void __launch_bounds__(kReduceBlock) k_tail_lds(TailArgs<T> A) {
  tail_lds_body<T, ND>(A);
}

// Batched form: block g runs the tail of grid g (arguments in device memory).
template <typename T, int ND>
__global__ void __launch_bounds__(kReduceBlock)
    k_tail_lds_batch(const TailArgs<T>* __restrict__ tab) {
  tail_lds_body<T, ND>(tab[blockIdx.x]);
}

template <typename T>
size_t tail_lds_bytes(const TailArgs<T>& a) {
  if (a.lv[a.l0].g.N > kTailLdsCells || a.L - a.l0 > kMaxTail) return 0;
  size_t cells = 0;
  for (int l = a.l0; l < a.L; ++l)
    cells += (size_t)a.lv[l].g.N * (2 + a.lv[l].g.ndim);
  cells += (size_t)a.lv[a.l0].g.N;  // residual scratch
  return cells * sizeof(T);
}

template <typename T>
hipError_t launch_tail_lds(const TailArgs<T>& a, hipStream_t s, bool* used) {
  const size_t lds = tail_lds_bytes(a);
  *used = lds > 0 && lds <= 62 * 1024;
  if (!*used) return hipSuccess;
  const int nd = a.lv[a.l0].g.ndim;
  if (nd == 1)
    hipLaunchKernelGGL((k_tail_lds<T, 1>), dim3(1), dim3(kReduceBlock), lds, s, a);
  else if (nd == 2)
    hipLaunchKernelGGL((k_tail_lds<T, 2>), dim3(1), dim3(kReduceBlock), lds, s, a);
  else
    hipLaunchKernelGGL((k_tail_lds<T, 3>), dim3(1), dim3(kReduceBlock), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tail_lds_batch(const TailArgs<T>* tab, int ng, int nd,
                                 size_t lds, hipStream_t s) {
  if (ng == 0) return hipSuccess;
  if (nd == 1)
    hipLaunchKernelGGL((k_tail_lds_batch<T, 1>), dim3(ng), dim3(kReduceBlock), lds, s, tab);
  else if (nd == 2)
    hipLaunchKernelGGL((k_tail_lds_batch<T, 2>), dim3(ng), dim3(kReduceBlock), lds, s, tab);
  else
    hipLaunchKernelGGL((k_tail_lds_batch<T, 3>), dim3(ng), dim3(kReduceBlock), lds, s, tab);
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
