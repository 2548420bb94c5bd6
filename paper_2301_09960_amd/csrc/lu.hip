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

// The same two solves with one wavefront per column (row), for K <= kSweepMax:
// the vector sits in LDS and is swept left to right; at step q the lanes
// update the entries after q with x_q.  Every entry receives the same DD
// operations in the same order as in the kernels above (the subtractions for
// q = 0, 1, ... and then, for U, the division), so the results are identical;
// the chain per wavefront is K steps instead of K^2 / 2.
constexpr int kSweepMax = 512;
constexpr int kSweepWaves = 4;

__global__ __launch_bounds__(64 * kSweepWaves) void k_trsm_lower_sweep(DDMat A, int j0, int K, int n) {
  __shared__ dd col[kSweepWaves][kSweepMax];
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int l = j0 + K + blockIdx.x * kSweepWaves + w;
  const bool live = l < n;
  if (live)
    for (int i = lane; i < K; i += 64) col[w][i] = A.get(j0 + i, l);
  __syncthreads();
  for (int q = 0; q < K - 1; ++q) {
    if (live) {
      const dd xq = col[w][q];
      for (int i = q + 1 + lane; i < K; i += 64) col[w][i] = dd_sub(col[w][i], dd_mul(A.get(j0 + i, j0 + q), xq));
    }
    __syncthreads();
  }
  if (live)
    for (int i = lane; i < K; i += 64) A.put(j0 + i, l, col[w][i]);
}

__global__ __launch_bounds__(64 * kSweepWaves) void k_trsm_upper_sweep(DDMat A, int j0, int K, int n) {
  __shared__ dd row[kSweepWaves][kSweepMax];
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int i = j0 + K + blockIdx.x * kSweepWaves + w;
  const bool live = i < n;
  if (live)
    for (int t = lane; t < K; t += 64) row[w][t] = A.get(i, j0 + t);
  __syncthreads();
  for (int q = 0; q < K; ++q) {
    if (live && lane == 0) row[w][q] = dd_div(row[w][q], A.get(j0 + q, j0 + q));
    __syncthreads();
    if (live) {
      const dd xq = row[w][q];
      for (int t = q + 1 + lane; t < K; t += 64) row[w][t] = dd_sub(row[w][t], dd_mul(xq, A.get(j0 + q, j0 + t)));
    }
    __syncthreads();
  }
  if (live)
    for (int t = lane; t < K; t += 64) A.put(i, j0 + t, row[w][t]);
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

// Blocked solve of L U x = b (x holds b on entry): blocks of kSolveB rows.
// Forward: one wavefront solves the block's rows against the unit lower
// diagonal block (lane per row, x_q passed by shuffle), then every later row
// subtracts the block's contribution (thread per row, q ascending).  Backward:
// the same from the last block up, with the division by U's diagonal.  Each
// entry's subtractions come in a fixed order, so the solve is reproducible.
constexpr int kSolveB = 64;

__device__ __forceinline__ dd shfl_dd(dd v, int src) {
  return dd{__shfl(v.hi, src, 64), __shfl(v.lo, src, 64)};
}

__global__ __launch_bounds__(64) void k_solve_fwd_diag(DDMat A, int n, double *x, int b0, int B) {
  const int lane = threadIdx.x, i = b0 + lane;
  dd xi = lane < B ? dd{x[i], x[n + i]} : dd{0.0, 0.0};
  for (int q = 0; q < B - 1; ++q) {
    const dd xq = shfl_dd(xi, q);
    if (lane > q && lane < B) xi = dd_sub(xi, dd_mul(A.get(i, b0 + q), xq));
  }
  if (lane < B) {
    x[i] = xi.hi;
    x[n + i] = xi.lo;
  }
}

__global__ __launch_bounds__(256) void k_solve_fwd_update(DDMat A, int n, double *x, int b0, int B) {
  const int i = b0 + B + blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  dd s{x[i], x[n + i]};
  for (int q = b0; q < b0 + B; ++q) s = dd_sub(s, dd_mul(A.get(i, q), dd{x[q], x[n + q]}));
  x[i] = s.hi;
  x[n + i] = s.lo;
}

__global__ __launch_bounds__(64) void k_solve_bwd_diag(DDMat A, int n, double *x, int b0, int B) {
  const int lane = threadIdx.x, i = b0 + lane;
  dd xi = lane < B ? dd{x[i], x[n + i]} : dd{0.0, 0.0};
  for (int q = B - 1; q >= 0; --q) {
    if (lane == q) xi = dd_div(xi, A.get(i, i));
    const dd xq = shfl_dd(xi, q);
    if (lane < q) xi = dd_sub(xi, dd_mul(A.get(i, b0 + q), xq));
  }
  if (lane < B) {
    x[i] = xi.hi;
    x[n + i] = xi.lo;
  }
}

__global__ __launch_bounds__(256) void k_solve_bwd_update(DDMat A, int n, double *x, int b0, int B) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= b0) return;
  dd s{x[i], x[n + i]};
  for (int q = b0; q < b0 + B; ++q) s = dd_sub(s, dd_mul(A.get(i, q), dd{x[q], x[n + q]}));
  x[i] = s.hi;
  x[n + i] = s.lo;
}

unsigned grid_for(int64_t work) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(work, 256), 8192)); }

}  // namespace

hipError_t launch_lu_panel(double *A, int64_t ld, int64_t plane, int j0, int K, int n, hipStream_t st) {
  const DDMat M{A, ld, plane};
  hipLaunchKernelGGL(k_lu_diag, dim3(1), dim3(kLuThreads), 0, st, M, j0, K);
  if (j0 + K < n && K <= kSweepMax) {
    const dim3 grid((unsigned)ceil_div(n - j0 - K, kSweepWaves));
    hipLaunchKernelGGL(k_trsm_lower_sweep, grid, dim3(64 * kSweepWaves), 0, st, M, j0, K, n);
    hipLaunchKernelGGL(k_trsm_upper_sweep, grid, dim3(64 * kSweepWaves), 0, st, M, j0, K, n);
  } else if (j0 + K < n) {
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
  const DDMat M{const_cast<double *>(A), ld, plane};
  for (int b0 = 0; b0 < n; b0 += kSolveB) {
    const int B = std::min(kSolveB, n - b0);
    hipLaunchKernelGGL(k_solve_fwd_diag, dim3(1), dim3(64), 0, st, M, n, x, b0, B);
    if (b0 + B < n)
      hipLaunchKernelGGL(k_solve_fwd_update, dim3((unsigned)ceil_div(n - b0 - B, 256)), dim3(256), 0, st, M, n, x,
                         b0, B);
  }
  for (int b0 = (n - 1) / kSolveB * kSolveB; b0 >= 0; b0 -= kSolveB) {
    const int B = std::min(kSolveB, n - b0);
    hipLaunchKernelGGL(k_solve_bwd_diag, dim3(1), dim3(64), 0, st, M, n, x, b0, B);
    if (b0 > 0)
      hipLaunchKernelGGL(k_solve_bwd_update, dim3((unsigned)ceil_div(b0, 256)), dim3(256), 0, st, M, n, x, b0, B);
  }
  return hipGetLastError();
}

}  // namespace mp
