// Blocked LU factorization of a DD matrix with the Schur updates done by the
// slice-product GEMM (Section 4.6), and the triangular solves that use it.
//
// For a block width K the algorithm of Section 4.6 repeats, on the trailing
// matrix: factor the K x K diagonal block A11 = L11 U11; turn A12 into
// U12 = L11^-1 A12 and A21 into L21 = A21 U11^-1; update A22 := A22 - L21 U12,
// the product formed by the GEMM of this library.  No pivoting, as in the
// paper.  L (unit lower, without its diagonal) and U overwrite A.
//
// A DD matrix is two planes (hi, lo), each column-major with leading dimension
// ld, the lo plane `plane` elements after the hi plane.  Everything here is DD
// arithmetic (dd.h) in a fixed order, so a factorization is reproducible.
#include <algorithm>

#include "dd.h"
#include "internal.h"
#include "layout.h"

namespace mp {
namespace {

struct DDMat {
  double *p;
  int64_t ld, plane;
  __device__ __forceinline__ dd get(int64_t i, int64_t j) const {
    return dd{p[i + j * ld], p[plane + i + j * ld]};
  }
  __device__ __forceinline__ void put(int64_t i, int64_t j, dd v) const {
    p[i + j * ld] = v.hi;
    p[plane + i + j * ld] = v.lo;
  }
};

constexpr int kLuThreads = 1024;

// Unblocked LU of the K x K block at (j0, j0), in one workgroup: for each
// column, divide below the pivot, then the rank-1 update of the rest.
__global__ __launch_bounds__(kLuThreads) void k_lu_diag(DDMat A, int j0, int K) {
  for (int j = 0; j < K; ++j) {
    const dd piv = A.get(j0 + j, j0 + j);
    for (int i = j + 1 + (int)threadIdx.x; i < K; i += kLuThreads)
      A.put(j0 + i, j0 + j, dd_div(A.get(j0 + i, j0 + j), piv));
    __syncthreads();
    const int r = K - j - 1;
    for (int idx = threadIdx.x; idx < r * r; idx += kLuThreads) {
      const int i = j + 1 + idx % r, l = j + 1 + idx / r;
      A.put(j0 + i, j0 + l, dd_sub(A.get(j0 + i, j0 + l), dd_mul(A.get(j0 + i, j0 + j), A.get(j0 + j, j0 + l))));
    }
    __syncthreads();
  }
}

// U12 = L11^-1 A12 in place: thread per column l of A12, forward substitution
// down the column with the unit lower L11.
__global__ __launch_bounds__(256) void k_trsm_lower(DDMat A, int j0, int K, int n) {
  const int l = j0 + K + blockIdx.x * 256 + threadIdx.x;
  if (l >= n) return;
  for (int i = 1; i < K; ++i) {
    dd s = A.get(j0 + i, l);
    for (int q = 0; q < i; ++q) s = dd_sub(s, dd_mul(A.get(j0 + i, j0 + q), A.get(j0 + q, l)));
    A.put(j0 + i, l, s);
  }
}

// L21 = A21 U11^-1 in place: thread per row i of A21, solving x U11 = a left to
// right.
__global__ __launch_bounds__(256) void k_trsm_upper(DDMat A, int j0, int K, int n) {
  const int i = j0 + K + blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  for (int q = 0; q < K; ++q) {
    dd s = A.get(i, j0 + q);
    for (int r = 0; r < q; ++r) s = dd_sub(s, dd_mul(A.get(i, j0 + r), A.get(j0 + r, j0 + q)));
    A.put(i, j0 + q, dd_div(s, A.get(j0 + q, j0 + q)));
  }
}

// out = A[r0 .. r0 + rows, c0 .. c0 + cols) as a contiguous DD matrix
// (leading dimension rows, lo plane rows * cols later).
__global__ __launch_bounds__(256) void k_copy_block(DDMat A, int r0, int c0, int rows, int cols, double *out) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int i = (int)(idx % rows), j = (int)(idx / rows);
    const dd v = A.get(r0 + i, c0 + j);
    out[idx] = v.hi;
    out[total + idx] = v.lo;
  }
}

// A[r0 + i, c0 + j] -= P[i, j] (P contiguous as written by the GEMM).
__global__ __launch_bounds__(256) void k_sub_block(DDMat A, int r0, int c0, int rows, int cols, const double *P) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int i = (int)(idx % rows), j = (int)(idx / rows);
    A.put(r0 + i, c0 + j, dd_sub(A.get(r0 + i, c0 + j), dd{P[idx], P[total + idx]}));
  }
}

// Sum of one DD value per thread over the workgroup, in a fixed tree order.
__device__ dd block_sum(dd v, dd *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kLuThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = dd_add(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const dd out = red[0];
  __syncthreads();
  return out;
}

// Solve L U x = b in place (x holds b on entry; hi plane, then lo plane of n),
// one workgroup: forward substitution with the unit lower L, then backward
// with U, each inner product split over the threads and summed in a tree.
__global__ __launch_bounds__(kLuThreads) void k_lu_solve(DDMat A, int n, double *x) {
  __shared__ dd red[kLuThreads];
  for (int i = 0; i < n; ++i) {
    dd part{0.0, 0.0};
    for (int q = threadIdx.x; q < i; q += kLuThreads) part = dd_add(part, dd_mul(A.get(i, q), dd{x[q], x[n + q]}));
    const dd s = block_sum(part, red);
    if (threadIdx.x == 0) {
      const dd y = dd_sub(dd{x[i], x[n + i]}, s);
      x[i] = y.hi;
      x[n + i] = y.lo;
    }
    __syncthreads();
  }
  for (int i = n - 1; i >= 0; --i) {
    dd part{0.0, 0.0};
    for (int q = i + 1 + (int)threadIdx.x; q < n; q += kLuThreads)
      part = dd_add(part, dd_mul(A.get(i, q), dd{x[q], x[n + q]}));
    const dd s = block_sum(part, red);
    if (threadIdx.x == 0) {
      const dd v = dd_div(dd_sub(dd{x[i], x[n + i]}, s), A.get(i, i));
      x[i] = v.hi;
      x[n + i] = v.lo;
    }
    __syncthreads();
  }
}

unsigned grid_for(int64_t work) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(work, 256), 8192)); }

}  // namespace

hipError_t launch_lu_panel(double *A, int64_t ld, int64_t plane, int j0, int K, int n, hipStream_t st) {
  const DDMat M{A, ld, plane};
  hipLaunchKernelGGL(k_lu_diag, dim3(1), dim3(kLuThreads), 0, st, M, j0, K);
  if (j0 + K < n) {
    hipLaunchKernelGGL(k_trsm_lower, dim3((unsigned)ceil_div(n - j0 - K, 256)), dim3(256), 0, st, M, j0, K, n);
    hipLaunchKernelGGL(k_trsm_upper, dim3((unsigned)ceil_div(n - j0 - K, 256)), dim3(256), 0, st, M, j0, K, n);
  }
  return hipGetLastError();
}

hipError_t launch_lu_copy(double *A, int64_t ld, int64_t plane, int r0, int c0, int rows, int cols, double *out,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_copy_block, dim3(grid_for((int64_t)rows * cols)), dim3(256), 0, st, DDMat{A, ld, plane}, r0,
                     c0, rows, cols, out);
  return hipGetLastError();
}

hipError_t launch_lu_sub(double *A, int64_t ld, int64_t plane, int r0, int c0, int rows, int cols, const double *P,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_sub_block, dim3(grid_for((int64_t)rows * cols)), dim3(256), 0, st, DDMat{A, ld, plane}, r0, c0,
                     rows, cols, P);
  return hipGetLastError();
}

hipError_t launch_lu_solve(const double *A, int64_t ld, int64_t plane, int n, double *x, hipStream_t st) {
  hipLaunchKernelGGL(k_lu_solve, dim3(1), dim3(kLuThreads), 0, st, DDMat{const_cast<double *>(A), ld, plane}, n, x);
  return hipGetLastError();
}

}  // namespace mp
