// Blocked LU factorization of a DD or TD matrix with the Schur updates done by
// the slice-product GEMM (Section 4.6), and the triangular solves that use it.
//
// For a block width K the algorithm of Section 4.6 repeats, on the trailing
// matrix: factor the K x K diagonal block A11 = L11 U11; turn A12 into
// U12 = L11^-1 A12 and A21 into L21 = A21 U11^-1; update A22 := A22 - L21 U12,
// the product formed by the GEMM of this library.  No pivoting, as in the
// paper.  L (unit lower, without its diagonal) and U overwrite A.
//
// A matrix is c planes of components, each column-major with leading dimension
// ld, plane r `r * plane` elements after the first.  Everything here is DD
// (dd.h) or TD (mc.h) arithmetic in a fixed order, so a factorization is
// reproducible.
#include <algorithm>

#include "dd.h"
#include "internal.h"
#include "layout.h"
#include "mc.h"

namespace mp {
namespace {

// The scalar operations, for DD (dd.h) and TD (mc.h) values.
__device__ __forceinline__ dd nadd(dd a, dd b) { return dd_add(a, b); }
__device__ __forceinline__ dd nsub(dd a, dd b) { return dd_sub(a, b); }
__device__ __forceinline__ dd nmul(dd a, dd b) { return dd_mul(a, b); }
__device__ __forceinline__ dd ndiv(dd a, dd b) { return dd_div(a, b); }
__device__ __forceinline__ dd nfms(dd s, dd a, dd b) { return dd_sub(s, dd_mul(a, b)); }
using td = mc<3>;
__device__ __forceinline__ td nadd(const td &a, const td &b) { return mc_add<3>(a, b); }
__device__ __forceinline__ td nsub(const td &a, const td &b) { return mc_sub<3>(a, b); }
__device__ __forceinline__ td nmul(const td &a, const td &b) { return mc_mul<3>(a, b); }
__device__ __forceinline__ td ndiv(const td &a, const td &b) { return mc_div<3>(a, b); }
// s - a b (TD: one renormalization of 8 terms)
__device__ __forceinline__ td nfms(const td &s, const td &a, const td &b) { return mc_fms<3>(s, a, b); }
// 1 / b, by the division above: a solve multiplies by it so that the division
// leaves the chain of dependent steps.
__device__ __forceinline__ dd ninv(dd b) { return dd_div(dd{1.0, 0.0}, b); }
__device__ __forceinline__ td ninv(const td &b) { return mc_div<3>(td{{1.0, 0.0, 0.0}}, b); }

template <typename Num>
struct Comps;
template <>
struct Comps<dd> {
  static constexpr int C = 2;
  __device__ static double get(const dd &v, int r) { return r == 0 ? v.hi : v.lo; }
  __device__ static void set(dd &v, int r, double x) { (r == 0 ? v.hi : v.lo) = x; }
};
template <>
struct Comps<td> {
  static constexpr int C = 3;
  __device__ static double get(const td &v, int r) { return v.x[r]; }
  __device__ static void set(td &v, int r, double x) { v.x[r] = x; }
};

template <typename Num>
__device__ __forceinline__ Num nzero() {
  Num v;
#pragma unroll
  for (int r = 0; r < Comps<Num>::C; ++r) Comps<Num>::set(v, r, 0.0);
  return v;
}

// A c-component vector stored as planes of n (x[r * n + i]).
template <typename Num>
__device__ __forceinline__ Num vget(const double *x, int n, int i) {
  Num v;
#pragma unroll
  for (int r = 0; r < Comps<Num>::C; ++r) Comps<Num>::set(v, r, x[(int64_t)r * n + i]);
  return v;
}
template <typename Num>
__device__ __forceinline__ void vput(double *x, int n, int i, const Num &v) {
#pragma unroll
  for (int r = 0; r < Comps<Num>::C; ++r) x[(int64_t)r * n + i] = Comps<Num>::get(v, r);
}

template <typename Num>
struct Mat {
  double *p;
  int64_t ld, plane;
  __device__ __forceinline__ Num get(int64_t i, int64_t j) const {
    Num v;
#pragma unroll
    for (int r = 0; r < Comps<Num>::C; ++r) Comps<Num>::set(v, r, p[r * plane + i + j * ld]);
    return v;
  }
  __device__ __forceinline__ void put(int64_t i, int64_t j, const Num &v) const {
#pragma unroll
    for (int r = 0; r < Comps<Num>::C; ++r) p[r * plane + i + j * ld] = Comps<Num>::get(v, r);
  }
};

constexpr int kLuThreads = 1024;

// Unblocked LU of the K x K block at (j0, j0), in one workgroup: for each
// column, divide below the pivot, then the rank-1 update of the rest.
template <typename Num>
__global__ __launch_bounds__(kLuThreads) void k_lu_diag(Mat<Num> A, int j0, int K) {
  for (int j = 0; j < K; ++j) {
    const Num piv = A.get(j0 + j, j0 + j);
    for (int i = j + 1 + (int)threadIdx.x; i < K; i += kLuThreads)
      A.put(j0 + i, j0 + j, ndiv(A.get(j0 + i, j0 + j), piv));
    __syncthreads();
    const int r = K - j - 1;
    for (int idx = threadIdx.x; idx < r * r; idx += kLuThreads) {
      const int i = j + 1 + idx % r, l = j + 1 + idx / r;
      A.put(j0 + i, j0 + l, nfms(A.get(j0 + i, j0 + l), A.get(j0 + i, j0 + j), A.get(j0 + j, j0 + l)));
    }
    __syncthreads();
  }
}

// The same factorization with the block held in LDS (K <= kDiagLds): the
// operations and their order are those of k_lu_diag, so the factors are
// identical; each column's chain waits on LDS instead of the L2.
constexpr int kDiagLds = 32;

template <typename Num>
__global__ __launch_bounds__(kLuThreads) void k_lu_diag_lds(Mat<Num> A, int j0, int K) {
  __shared__ Num blk[kDiagLds * kDiagLds];  // column-major, leading dimension K
  for (int idx = threadIdx.x; idx < K * K; idx += kLuThreads) blk[idx] = A.get(j0 + idx % K, j0 + idx / K);
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    const Num piv = blk[j + j * K];
    for (int i = j + 1 + (int)threadIdx.x; i < K; i += kLuThreads) blk[i + j * K] = ndiv(blk[i + j * K], piv);
    __syncthreads();
    const int r = K - j - 1;
    for (int idx = threadIdx.x; idx < r * r; idx += kLuThreads) {
      const int i = j + 1 + idx % r, l = j + 1 + idx / r;
      blk[i + l * K] = nfms(blk[i + l * K], blk[i + j * K], blk[j + l * K]);
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < K * K; idx += kLuThreads) A.put(j0 + idx % K, j0 + idx / K, blk[idx]);
}

template <typename Num>
void launch_lu_diag(const Mat<Num> &M, int j0, int K, hipStream_t st) {
  if (K <= kDiagLds)
    hipLaunchKernelGGL((k_lu_diag_lds<Num>), dim3(1), dim3(kLuThreads), 0, st, M, j0, K);
  else
    hipLaunchKernelGGL((k_lu_diag<Num>), dim3(1), dim3(kLuThreads), 0, st, M, j0, K);
}

// U12 = L11^-1 A12 in place: thread per column l of A12, forward substitution
// down the column with the unit lower L11.
template <typename Num>
__global__ __launch_bounds__(256) void k_trsm_lower(Mat<Num> A, int j0, int K, int n) {
  const int l = j0 + K + blockIdx.x * 256 + threadIdx.x;
  if (l >= n) return;
  for (int i = 1; i < K; ++i) {
    Num s = A.get(j0 + i, l);
    for (int q = 0; q < i; ++q) s = nfms(s, A.get(j0 + i, j0 + q), A.get(j0 + q, l));
    A.put(j0 + i, l, s);
  }
}

// L21 = A21 U11^-1 in place: thread per row i of A21, solving x U11 = a left to
// right; x_q is the remaining sum times the reciprocal of u_qq.
template <typename Num>
__global__ __launch_bounds__(256) void k_trsm_upper(Mat<Num> A, int j0, int K, int n) {
  const int i = j0 + K + blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  for (int q = 0; q < K; ++q) {
    Num s = A.get(i, j0 + q);
    for (int r = 0; r < q; ++r) s = nfms(s, A.get(i, j0 + r), A.get(j0 + r, j0 + q));
    A.put(i, j0 + q, nmul(s, ninv(A.get(j0 + q, j0 + q))));
  }
}

// The same two solves with one wavefront per column (row), for K <= kSweepMax:
// the vector sits in LDS and is swept left to right; at step q the lanes
// update the entries after q with x_q.  Every entry receives the same
// operations in the same order as in the kernels above (the subtractions for
// q = 0, 1, ... and then, for U, the product with 1 / u_qq), so the results
// are identical; the chain per wavefront is K steps instead of K^2 / 2, and
// the reciprocals of U's diagonal are formed before it, all at once.
constexpr int kSweepMax = 512;
constexpr int kSweepWaves = 4;

// KMAX: the largest K of the instance.  With KMAX <= kDiagLds the K x K
// diagonal block is also staged in LDS, so each step of the chain reads it
// there; the operations are the same either way.
template <typename Num, int KMAX>
__global__ __launch_bounds__(64 * kSweepWaves) void k_trsm_lower_sweep(Mat<Num> A, int j0, int K, int n) {
  constexpr bool kStage = KMAX <= kDiagLds;
  __shared__ Num col[kSweepWaves][KMAX];
  __shared__ Num blk[kStage ? KMAX * KMAX : 1];
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int l = j0 + K + blockIdx.x * kSweepWaves + w;
  const bool live = l < n;
  if constexpr (kStage)
    for (int idx = threadIdx.x; idx < K * K; idx += 64 * kSweepWaves) blk[idx] = A.get(j0 + idx % K, j0 + idx / K);
  if (live)
    for (int i = lane; i < K; i += 64) col[w][i] = A.get(j0 + i, l);
  __syncthreads();
  for (int q = 0; q < K - 1; ++q) {
    if (live) {
      const Num xq = col[w][q];
      for (int i = q + 1 + lane; i < K; i += 64) {
        Num lq;
        if constexpr (kStage)
          lq = blk[i + q * K];
        else
          lq = A.get(j0 + i, j0 + q);
        col[w][i] = nfms(col[w][i], lq, xq);
      }
    }
    __syncthreads();
  }
  if (live)
    for (int i = lane; i < K; i += 64) A.put(j0 + i, l, col[w][i]);
}

template <typename Num, int KMAX>
__global__ __launch_bounds__(64 * kSweepWaves) void k_trsm_upper_sweep(Mat<Num> A, int j0, int K, int n) {
  constexpr bool kStage = KMAX <= kDiagLds;
  __shared__ Num row[kSweepWaves][KMAX];
  __shared__ Num inv[KMAX];
  __shared__ Num blk[kStage ? KMAX * KMAX : 1];
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int i = j0 + K + blockIdx.x * kSweepWaves + w;
  const bool live = i < n;
  if constexpr (kStage)
    for (int idx = threadIdx.x; idx < K * K; idx += 64 * kSweepWaves) blk[idx] = A.get(j0 + idx % K, j0 + idx / K);
  for (int t = threadIdx.x; t < K; t += 64 * kSweepWaves) inv[t] = ninv(A.get(j0 + t, j0 + t));
  if (live)
    for (int t = lane; t < K; t += 64) row[w][t] = A.get(i, j0 + t);
  __syncthreads();
  for (int q = 0; q < K; ++q) {
    if (live) {
      // every lane forms x_q; lane 0 stores it
      const Num xq = nmul(row[w][q], inv[q]);
      if (lane == 0) row[w][q] = xq;
      for (int t = q + 1 + lane; t < K; t += 64) {
        Num uq;
        if constexpr (kStage)
          uq = blk[q + t * K];
        else
          uq = A.get(j0 + q, j0 + t);
        row[w][t] = nfms(row[w][t], xq, uq);
      }
    }
    __syncthreads();
  }
  if (live)
    for (int t = lane; t < K; t += 64) A.put(i, j0 + t, row[w][t]);
}

// Both panel sweeps for a K x K diagonal block at (j0, j0), rows and columns up
// to `end`.
template <typename Num>
void launch_sweeps(const Mat<Num> &M, int j0, int K, int end, hipStream_t st) {
  const dim3 grid((unsigned)ceil_div(end - j0 - K, kSweepWaves));
  if (K <= kDiagLds) {
    hipLaunchKernelGGL((k_trsm_lower_sweep<Num, kDiagLds>), grid, dim3(64 * kSweepWaves), 0, st, M, j0, K, end);
    hipLaunchKernelGGL((k_trsm_upper_sweep<Num, kDiagLds>), grid, dim3(64 * kSweepWaves), 0, st, M, j0, K, end);
  } else {
    hipLaunchKernelGGL((k_trsm_lower_sweep<Num, kSweepMax>), grid, dim3(64 * kSweepWaves), 0, st, M, j0, K, end);
    hipLaunchKernelGGL((k_trsm_upper_sweep<Num, kSweepMax>), grid, dim3(64 * kSweepWaves), 0, st, M, j0, K, end);
  }
}

// A[r0 + i, c0 + l] -= sum over q in [q0, q0 + kb) of A[r0 + i, q] A[q, c0 + l]
// (q ascending), thread per entry: the trailing update inside a diagonal block
// factored in inner blocks.
template <typename Num>
__global__ __launch_bounds__(256) void k_rank_update(Mat<Num> A, int r0, int c0, int rows, int cols, int q0,
                                                     int kb) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int i = r0 + (int)(idx % rows), l = c0 + (int)(idx / rows);
    Num s = A.get(i, l);
    for (int q = q0; q < q0 + kb; ++q) s = nfms(s, A.get(i, q), A.get(q, l));
    A.put(i, l, s);
  }
}

// out = A[r0 .. r0 + rows, c0 .. c0 + cols) as a contiguous DD matrix
// (leading dimension rows, lo plane rows * cols later).
template <typename Num>
__global__ __launch_bounds__(256) void k_copy_block(Mat<Num> A, int r0, int c0, int rows, int cols, double *out) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int i = (int)(idx % rows), j = (int)(idx / rows);
    const Num v = A.get(r0 + i, c0 + j);
#pragma unroll
    for (int r = 0; r < Comps<Num>::C; ++r) out[r * total + idx] = Comps<Num>::get(v, r);
  }
}

// A[r0 + i, c0 + j] -= P[i, j] (P contiguous as written by the GEMM).
template <typename Num>
__global__ __launch_bounds__(256) void k_sub_block(Mat<Num> A, int r0, int c0, int rows, int cols, const double *P) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int i = (int)(idx % rows), j = (int)(idx / rows);
    Num p;
#pragma unroll
    for (int r = 0; r < Comps<Num>::C; ++r) Comps<Num>::set(p, r, P[r * total + idx]);
    A.put(r0 + i, c0 + j, nsub(A.get(r0 + i, c0 + j), p));
  }
}

// Blocked solve of L U x = b (x holds b on entry): blocks of kSolveB rows.
// Forward: one wavefront solves the block's rows against the unit lower
// diagonal block (lane per row, x_q passed by shuffle), then every later row
// subtracts the block's contribution (k_solve_update).  Backward: the same
// from the last block up, with the product by the reciprocal of U's diagonal
// entry (each lane forms its own before the chain).  Every entry's operations
// come in a fixed order, so the solve is reproducible.
constexpr int kSolveB = 64;

template <typename Num>
__device__ __forceinline__ Num shfl_num(const Num &v, int src) {
  Num o;
#pragma unroll
  for (int r = 0; r < Comps<Num>::C; ++r) Comps<Num>::set(o, r, __shfl(Comps<Num>::get(v, r), src, 64));
  return o;
}

template <typename Num>
__global__ __launch_bounds__(64) void k_solve_fwd_diag(Mat<Num> A, int n, double *x, int b0, int B) {
  const int lane = threadIdx.x, i = b0 + lane;
  Num xi = lane < B ? vget<Num>(x, n, i) : nzero<Num>();
  for (int q = 0; q < B - 1; ++q) {
    const Num xq = shfl_num(xi, q);
    if (lane > q && lane < B) xi = nfms(xi, A.get(i, b0 + q), xq);
  }
  if (lane < B) vput<Num>(x, n, i, xi);
}

template <typename Num>
__global__ __launch_bounds__(64) void k_solve_bwd_diag(Mat<Num> A, int n, double *x, int b0, int B) {
  const int lane = threadIdx.x, i = b0 + lane;
  Num xi = lane < B ? vget<Num>(x, n, i) : nzero<Num>();
  Num inv = nzero<Num>();
  if (lane < B) inv = ninv(A.get(i, i));
  for (int q = B - 1; q >= 0; --q) {
    if (lane == q) xi = nmul(xi, inv);
    const Num xq = shfl_num(xi, q);
    if (lane < q) xi = nfms(xi, A.get(i, b0 + q), xq);
  }
  if (lane < B) vput<Num>(x, n, i, xi);
}

// x_i -= sum over q in [b0, b0 + B) of A(i, q) x_q for the rows i in
// [r0, r0 + rows): the sum in kSolveChunks runs of consecutive q, one thread
// each (32 rows per workgroup), then added to x_i in run order.
constexpr int kSolveChunks = 8;
constexpr int kSolveRows = 256 / kSolveChunks;

template <typename Num>
__global__ __launch_bounds__(256) void k_solve_update(Mat<Num> A, int n, double *x, int b0, int B, int r0,
                                                      int rows) {
  __shared__ Num part[kSolveChunks][kSolveRows];
  const int rl = threadIdx.x % kSolveRows, c = threadIdx.x / kSolveRows;
  const int i = r0 + blockIdx.x * kSolveRows + rl;
  const bool live = i < r0 + rows;
  const int per = (B + kSolveChunks - 1) / kSolveChunks;
  const int q0 = b0 + c * per, q1 = std::min(b0 + B, q0 + per);
  Num p = nzero<Num>();  // minus the run's sum
  if (live)
    for (int q = q0; q < q1; ++q) p = nfms(p, A.get(i, q), vget<Num>(x, n, q));
  part[c][rl] = p;
  __syncthreads();
  if (live && c == 0) {
    Num s = vget<Num>(x, n, i);
#pragma unroll
    for (int r = 0; r < kSolveChunks; ++r) s = nadd(s, part[r][rl]);
    vput<Num>(x, n, i, s);
  }
}

unsigned grid_for(int64_t work) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(work, 256), 8192)); }

// Diagonal blocks wider than kInner are factored in inner blocks of kInner:
// the unblocked kernel on the inner diagonal block (in LDS), the two panel
// solves restricted to the diagonal block, and a rank-kInner update of its
// rest (DD at n = 2048: K = 512 170 -> 13.6 ms, and K = 64 12.0 -> 10.7 ms
// once blocks of up to kInner were held in LDS).
constexpr int kInner = 32;

template <typename Num>
hipError_t lu_panel(double *A, int64_t ld, int64_t plane, int j0, int K, int n, hipStream_t st) {
  const Mat<Num> M{A, ld, plane};
  if (K <= kInner) {
    launch_lu_diag<Num>(M, j0, K, st);
  } else {
    const int end = j0 + K;
    for (int jj = j0; jj < end; jj += kInner) {
      const int kb = std::min(kInner, end - jj), r = end - jj - kb;
      launch_lu_diag<Num>(M, jj, kb, st);
      if (r == 0) break;
      launch_sweeps<Num>(M, jj, kb, end, st);
      hipLaunchKernelGGL((k_rank_update<Num>), dim3(grid_for((int64_t)r * r)), dim3(256), 0, st, M, jj + kb, jj + kb,
                         r, r, jj, kb);
    }
  }
  if (j0 + K < n && K <= kSweepMax) {
    launch_sweeps<Num>(M, j0, K, n, st);
  } else if (j0 + K < n) {
    hipLaunchKernelGGL((k_trsm_lower<Num>), dim3((unsigned)ceil_div(n - j0 - K, 256)), dim3(256), 0, st, M, j0, K,
                       n);
    hipLaunchKernelGGL((k_trsm_upper<Num>), dim3((unsigned)ceil_div(n - j0 - K, 256)), dim3(256), 0, st, M, j0, K,
                       n);
  }
  return hipGetLastError();
}

template <typename Num>
hipError_t lu_solve(const double *A, int64_t ld, int64_t plane, int n, double *x, hipStream_t st) {
  const Mat<Num> M{const_cast<double *>(A), ld, plane};
  for (int b0 = 0; b0 < n; b0 += kSolveB) {
    const int B = std::min(kSolveB, n - b0);
    hipLaunchKernelGGL((k_solve_fwd_diag<Num>), dim3(1), dim3(64), 0, st, M, n, x, b0, B);
    if (b0 + B < n)
      hipLaunchKernelGGL((k_solve_update<Num>), dim3((unsigned)ceil_div(n - b0 - B, kSolveRows)), dim3(256), 0, st, M,
                         n, x, b0, B, b0 + B, n - b0 - B);
  }
  for (int b0 = (n - 1) / kSolveB * kSolveB; b0 >= 0; b0 -= kSolveB) {
    const int B = std::min(kSolveB, n - b0);
    hipLaunchKernelGGL((k_solve_bwd_diag<Num>), dim3(1), dim3(64), 0, st, M, n, x, b0, B);
    if (b0 > 0)
      hipLaunchKernelGGL((k_solve_update<Num>), dim3((unsigned)ceil_div(b0, kSolveRows)), dim3(256), 0, st, M, n, x,
                         b0, B, 0, b0);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lu_panel(int comps, double *A, int64_t ld, int64_t plane, int j0, int K, int n, hipStream_t st) {
  return comps == 2 ? lu_panel<dd>(A, ld, plane, j0, K, n, st) : lu_panel<td>(A, ld, plane, j0, K, n, st);
}

hipError_t launch_lu_copy(int comps, double *A, int64_t ld, int64_t plane, int r0, int c0, int rows, int cols,
                          double *out, hipStream_t st) {
  if (comps == 2)
    hipLaunchKernelGGL((k_copy_block<dd>), dim3(grid_for((int64_t)rows * cols)), dim3(256), 0, st,
                       Mat<dd>{A, ld, plane}, r0, c0, rows, cols, out);
  else
    hipLaunchKernelGGL((k_copy_block<td>), dim3(grid_for((int64_t)rows * cols)), dim3(256), 0, st,
                       Mat<td>{A, ld, plane}, r0, c0, rows, cols, out);
  return hipGetLastError();
}

hipError_t launch_lu_sub(int comps, double *A, int64_t ld, int64_t plane, int r0, int c0, int rows, int cols,
                         const double *P, hipStream_t st) {
  if (comps == 2)
    hipLaunchKernelGGL((k_sub_block<dd>), dim3(grid_for((int64_t)rows * cols)), dim3(256), 0, st,
                       Mat<dd>{A, ld, plane}, r0, c0, rows, cols, P);
  else
    hipLaunchKernelGGL((k_sub_block<td>), dim3(grid_for((int64_t)rows * cols)), dim3(256), 0, st,
                       Mat<td>{A, ld, plane}, r0, c0, rows, cols, P);
  return hipGetLastError();
}

hipError_t launch_lu_solve(int comps, const double *A, int64_t ld, int64_t plane, int n, double *x, hipStream_t st) {
  return comps == 2 ? lu_solve<dd>(A, ld, plane, n, x, st) : lu_solve<td>(A, ld, plane, n, x, st);
}

}  // namespace mp
