// The simple (non-Ozaki) multi-component matrix multiplication that Section
// 4.4 compares with the Ozaki scheme on the GPU: C = A B by the triple loop in
// the format's own arithmetic, every term a_ip b_pj multiplied and added in
// DD, TD, QD or TS arithmetic, in the order p = 0, 1, ..., k - 1.  D+S (a
// binary64 leading part and a binary32 trailing part) reads each input as the
// DD number (hi, lo) (exact), runs in DD arithmetic and rounds each entry of C
// to D+S once at the end (hi kept, lo rounded to binary32).
//
// One workgroup of 256 threads computes a 16 R x 16 R tile of C, each thread
// an R x R grid of entries (rows tx + 16 r, columns ty + 16 s); R = 4 for DD,
// D+S and TS, 2 for TD and QD, whose accumulators and sorting take more
// registers.  Two ways of
// reading the operands, as the paper's comparison with and without shared
// memory:
//   direct: every thread reads its 4 entries of A's column p and of B's row p
//           from global memory for each p (through the caches);
//   staged: the workgroup copies 16 R x 16 panels of A and 16 x 16 R panels of B
//           (all components) into LDS with coalesced loads, then every thread
//           reads them from LDS.
// Both take the same operations in the same order, so they give the same C
// bit for bit.  The work is VALU-bound: about 25 binary64 operations per
// term for DD, several times more for the sort-and-renormalize arithmetic of
// TD, QD and TS (mc.h).
#include "dd.h"
#include "internal.h"
#include "mc.h"

namespace mp {
namespace {

constexpr int kKP = 16, kThreads = 256;

// Format traits: value type V, components and their loads / stores.
//   comp(X, r): plane r of X.
template <int F> struct Simple;

// DD: classical double-double arithmetic (dd.h).
template <> struct Simple<0> {
  static constexpr int C = 2, R = 4;
  using V = dd;
  using E = double;  // component type in memory
  static __device__ __forceinline__ V zero() { return dd{0.0, 0.0}; }
  static __device__ __forceinline__ V mac(V acc, V a, V b) { return dd_add(acc, dd_mul(a, b)); }
  static __device__ __forceinline__ V make(const double (&x)[2]) { return dd{x[0], x[1]}; }
  static __device__ __forceinline__ void parts(const V &v, double (&x)[2]) {
    x[0] = v.hi;
    x[1] = v.lo;
  }
};
// TD and QD: sort-and-renormalize arithmetic (mc.h), one renormalization per term.
template <int CC> struct SimpleMc {
  static constexpr int C = CC, R = 2;
  using V = mc<CC, double>;
  using E = double;
  static __device__ __forceinline__ V zero() {
    V v;
#pragma unroll
    for (int r = 0; r < CC; ++r) v.x[r] = 0.0;
    return v;
  }
  static __device__ __forceinline__ V mac(const V &acc, const V &a, const V &b) { return mc_fma<CC>(acc, a, b); }
  static __device__ __forceinline__ V make(const double (&x)[CC]) {
    V v;
#pragma unroll
    for (int r = 0; r < CC; ++r) v.x[r] = x[r];
    return v;
  }
  static __device__ __forceinline__ void parts(const V &v, double (&x)[CC]) {
#pragma unroll
    for (int r = 0; r < CC; ++r) x[r] = v.x[r];
  }
};
template <> struct Simple<1> : SimpleMc<3> {};
template <> struct Simple<2> : SimpleMc<4> {};
// TS: the same arithmetic on three binary32 components.
template <> struct Simple<3> {
  static constexpr int C = 3, R = 4;
  using V = mc<3, float>;
  using E = float;
  static __device__ __forceinline__ V zero() { return V{{0.0f, 0.0f, 0.0f}}; }
  static __device__ __forceinline__ V mac(const V &acc, const V &a, const V &b) { return mc_fma<3>(acc, a, b); }
  static __device__ __forceinline__ V make(const float (&x)[3]) { return V{{x[0], x[1], x[2]}}; }
  static __device__ __forceinline__ void parts(const V &v, float (&x)[3]) {
    for (int r = 0; r < 3; ++r) x[r] = v.x[r];
  }
};

// Operand views.  Plane r of a planar operand starts at X + r * stride
// elements; D+S has a binary64 plane (hi) and a binary32 plane (lo).
template <int F> struct Planes {
  using E = typename Simple<F>::E;
  const E *X;
  int64_t stride;
  int ld;
  __device__ __forceinline__ void load(int64_t off, E (&x)[Simple<F>::C]) const {
#pragma unroll
    for (int r = 0; r < Simple<F>::C; ++r) x[r] = X[r * stride + off];
  }
};

struct DsView {
  const double *hi;
  const float *lo;
  int ld;
  __device__ __forceinline__ void load(int64_t off, double (&x)[2]) const {
    x[0] = hi[off];
    x[1] = (double)lo[off];
  }
};

// Arithmetic of format F, operand view View, output writer.
template <int F, class View, bool DS_OUT, bool STAGED>
__device__ __forceinline__ void simple_tile(int m, int n, int k, const View &A, const View &B, void *Cv0, void *Cv1,
                                            int ldc, int64_t c_stride) {
  using S = Simple<F>;
  using V = typename S::V;
  using E = typename S::E;
  constexpr int C = S::C, R = S::R, kTile = 16 * R;
  // tile (tm, tn): neighbouring workgroups share a column panel of B
  const int tiles_m = (m + kTile - 1) / kTile;
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int i0 = tm * kTile, j0 = tn * kTile;

  V acc[R][R];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int s = 0; s < R; ++s) acc[r][s] = S::zero();

  if constexpr (!STAGED) {
    for (int p = 0; p < k; ++p) {
      V a[R], b[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = i0 + tx + 16 * r;
        E x[C];
        if (i < m) {
          A.load(i + (int64_t)p * A.ld, x);
        } else {
#pragma unroll
          for (int q = 0; q < C; ++q) x[q] = E(0);
        }
        a[r] = S::make(x);
      }
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const int j = j0 + ty + 16 * s;
        E x[C];
        if (j < n) {
          B.load(p + (int64_t)j * B.ld, x);
        } else {
#pragma unroll
          for (int q = 0; q < C; ++q) x[q] = E(0);
        }
        b[s] = S::make(x);
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int s = 0; s < R; ++s) acc[r][s] = S::mac(acc[r][s], a[r], b[s]);
    }
  } else {
    // panels: sA[q][pp][ii] = component q of A(i0 + ii, p0 + pp); sB[q][pp][jj] likewise
    __shared__ E sA[C][kKP][kTile];
    __shared__ E sB[C][kKP][kTile];
    for (int p0 = 0; p0 < k; p0 += kKP) {
      // A panel: 64 rows x 16 k; consecutive threads take consecutive rows
#pragma unroll
      for (int w = 0; w < kTile * kKP / kThreads; ++w) {
        const int e = tid + kThreads * w, ii = e % kTile, pp = e / kTile;
        const int i = i0 + ii, p = p0 + pp;
        E x[C];
        if (i < m && p < k) {
          A.load(i + (int64_t)p * A.ld, x);
        } else {
#pragma unroll
          for (int q = 0; q < C; ++q) x[q] = E(0);
        }
#pragma unroll
        for (int q = 0; q < C; ++q) sA[q][pp][ii] = x[q];
      }
      // B panel: 16 k x 64 columns; consecutive threads take consecutive k
#pragma unroll
      for (int w = 0; w < kTile * kKP / kThreads; ++w) {
        const int e = tid + kThreads * w, pp = e % kKP, jj = e / kKP;
        const int j = j0 + jj, p = p0 + pp;
        E x[C];
        if (j < n && p < k) {
          B.load(p + (int64_t)j * B.ld, x);
        } else {
#pragma unroll
          for (int q = 0; q < C; ++q) x[q] = E(0);
        }
#pragma unroll
        for (int q = 0; q < C; ++q) sB[q][pp][jj] = x[q];
      }
      __syncthreads();
      const int np = k - p0 < kKP ? k - p0 : kKP;
      for (int pp = 0; pp < np; ++pp) {
        V a[R], b[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          E x[C];
#pragma unroll
          for (int q = 0; q < C; ++q) x[q] = sA[q][pp][tx + 16 * r];
          a[r] = S::make(x);
        }
#pragma unroll
        for (int s = 0; s < R; ++s) {
          E x[C];
#pragma unroll
          for (int q = 0; q < C; ++q) x[q] = sB[q][pp][ty + 16 * s];
          b[s] = S::make(x);
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int s = 0; s < R; ++s) acc[r][s] = S::mac(acc[r][s], a[r], b[s]);
      }
      __syncthreads();
    }
  }

  // store (rows along the lanes: contiguous in column-major C)
#pragma unroll
  for (int s = 0; s < R; ++s)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = i0 + tx + 16 * r, j = j0 + ty + 16 * s;
      if (i >= m || j >= n) continue;
      E x[C];
      S::parts(acc[r][s], x);
      const int64_t off = i + (int64_t)j * ldc;
      if constexpr (DS_OUT) {
        // D+S: hi is the DD's leading part (already RN of the sum), lo rounded to binary32
        static_cast<double *>(Cv0)[off] = x[0];
        static_cast<float *>(Cv1)[off] = (float)x[1];
      } else {
#pragma unroll
        for (int q = 0; q < C; ++q) static_cast<E *>(Cv0)[q * c_stride + off] = x[q];
      }
    }
}

template <int F, bool STAGED>
__global__ __launch_bounds__(kThreads) void k_simple(int m, int n, int k, Planes<F> A, Planes<F> B,
                                                      typename Simple<F>::E *Cm, int ldc, int64_t c_stride) {
  simple_tile<F, Planes<F>, false, STAGED>(m, n, k, A, B, Cm, nullptr, ldc, c_stride);
}

template <bool STAGED>
__global__ __launch_bounds__(kThreads) void k_simple_ds(int m, int n, int k, DsView A, DsView B, double *Chi,
                                                         float *Clo, int ldc) {
  simple_tile<0, DsView, true, STAGED>(m, n, k, A, B, Chi, Clo, ldc, 0);
}

template <int F>
unsigned tiles_of(int m, int n) {
  constexpr int kTile = 16 * Simple<F>::R;
  return (unsigned)(((m + kTile - 1) / kTile) * ((n + kTile - 1) / kTile));
}

}  // namespace

template <int F>
hipError_t launch_simple(int m, int n, int k, const void *A, int lda, const void *B, int ldb, void *Cm, int ldc,
                         bool staged, hipStream_t st) {
  using E = typename Simple<F>::E;
  Planes<F> a{static_cast<const E *>(A), (int64_t)lda * k, lda};
  Planes<F> b{static_cast<const E *>(B), (int64_t)ldb * n, ldb};
  if (staged)
    hipLaunchKernelGGL((k_simple<F, true>), dim3(tiles_of<F>(m, n)), dim3(kThreads), 0, st, m, n, k, a, b,
                       static_cast<E *>(Cm), ldc, (int64_t)ldc * n);
  else
    hipLaunchKernelGGL((k_simple<F, false>), dim3(tiles_of<F>(m, n)), dim3(kThreads), 0, st, m, n, k, a, b,
                       static_cast<E *>(Cm), ldc, (int64_t)ldc * n);
  return hipGetLastError();
}

hipError_t launch_simple_ds(int m, int n, int k, const double *Ahi, const float *Alo, int lda, const double *Bhi,
                            const float *Blo, int ldb, double *Chi, float *Clo, int ldc, bool staged,
                            hipStream_t st) {
  DsView a{Ahi, Alo, lda}, b{Bhi, Blo, ldb};
  if (staged)
    hipLaunchKernelGGL((k_simple_ds<true>), dim3(tiles_of<0>(m, n)), dim3(kThreads), 0, st, m, n, k, a, b, Chi, Clo,
                       ldc);
  else
    hipLaunchKernelGGL((k_simple_ds<false>), dim3(tiles_of<0>(m, n)), dim3(kThreads), 0, st, m, n, k, a, b, Chi, Clo,
                       ldc);
  return hipGetLastError();
}

// D+S <-> DD planes.  to_dd: (hi, lo) of a rows x cols matrix with leading
// dimension ld into two compact binary64 planes (rows x cols each, exact).
// from_dd: a normalized DD matrix (two compact planes) into D+S with leading
// dimension ld: hi kept (it is the rounding of the sum), lo rounded to binary32.
__global__ __launch_bounds__(kThreads) void k_ds_to_dd(int rows, int cols, const double *hi, const float *lo, int ld,
                                                        double *out) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
    const int64_t i = t % rows, j = t / rows, off = i + j * ld;
    out[t] = hi[off];
    out[total + t] = (double)lo[off];
  }
}

__global__ __launch_bounds__(kThreads) void k_dd_to_ds(int rows, int cols, const double *in, double *hi, float *lo,
                                                        int ld) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
    const int64_t i = t % rows, j = t / rows, off = i + j * ld;
    hi[off] = in[t];
    lo[off] = (float)in[total + t];
  }
}

unsigned grid_of(int64_t total) {
  const int64_t b = (total + kThreads - 1) / kThreads;
  return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

hipError_t launch_ds_to_dd(int rows, int cols, const double *hi, const float *lo, int ld, double *out,
                           hipStream_t st) {
  if ((int64_t)rows * cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ds_to_dd, dim3(grid_of((int64_t)rows * cols)), dim3(kThreads), 0, st, rows, cols, hi, lo, ld,
                     out);
  return hipGetLastError();
}

hipError_t launch_dd_to_ds(int rows, int cols, const double *in, double *hi, float *lo, int ld, hipStream_t st) {
  if ((int64_t)rows * cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dd_to_ds, dim3(grid_of((int64_t)rows * cols)), dim3(kThreads), 0, st, rows, cols, in, hi, lo,
                     ld);
  return hipGetLastError();
}

template hipError_t launch_simple<0>(int, int, int, const void *, int, const void *, int, void *, int, bool,
                                     hipStream_t);
template hipError_t launch_simple<1>(int, int, int, const void *, int, const void *, int, void *, int, bool,
                                     hipStream_t);
template hipError_t launch_simple<2>(int, int, int, const void *, int, const void *, int, void *, int, bool,
                                     hipStream_t);
template hipError_t launch_simple<3>(int, int, int, const void *, int, const void *, int, void *, int, bool,
                                     hipStream_t);

}  // namespace mp
