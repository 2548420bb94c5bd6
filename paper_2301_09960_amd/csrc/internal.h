// Internal host-side interfaces between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"

namespace mp {

constexpr int kZeroExp = INT32_MIN;

// Work lists of a persistent launch, one per XCD (each XCD has its own L2).
// List q holds items [bounds[q], bounds[q + 1]); counters[q] counts the items
// taken from it (cleared before the launch).  Workgroups are dispatched to the
// XCDs in turn, so workgroup b runs on XCD b % kXcds: it takes items from its
// own list first, so that the workgroups sharing an L2 work on the tiles of the
// same products at the same time, then from the other lists, so that no list
// waits for one XCD.  Returns -1 once every list is drained.
constexpr int kXcds = 8;
__device__ __forceinline__ int take_item(int *counters, const int *bounds, int b) {
  for (int j = 0; j < kXcds; ++j) {
    const int q = (b + j) % kXcds;
    const int size = bounds[q + 1] - bounds[q];
    if (size <= 0) continue;
    const int i = atomicAdd(&counters[q], 1);
    if (i < size) return bounds[q] + i;
  }
  return -1;
}

// One operand of a split: `nvec` vectors (rows of A, or columns of B) of `len`
// multi-component elements; component r of element (v, p) is at
// X[r * comp_stride + v * sv + p * sp].  `orient` 0: v is the contiguous
// index (rows of a column-major A); 1: p is (columns of a column-major B).
template <typename T>
struct SplitOperand {
  const T *X;
  int64_t comp_stride, sv, sp;
  int nvec, len;
  int orient;
  // workspace
  T *resid;              // C planes of nvec * len, same orientation, compact
  void *packed;          // packed slices (layout.h)
  int64_t nbp, kbp;      // padded block counts of the packed slices
  void *mu;              // per pass: nvec maxima as IEEE bit patterns (uint64 / uint32)
  int *exps;             // D x nvec exponents (FLOAT) or nvec (INT8)
  int D, rho;            // slice count and shift (used by the batched kernels)
  int last_literal;      // 1: the last slice is the residual's leading component (FLOAT only)
};

// One product of an INT8-form batch, as read by the persistent INT8 GEMM and
// the batched combine.  The diagonals of a (tile, k chunk) are cut into
// `groups` work items of nearly equal pair counts.
struct Int8GemmDesc {
  const int8_t *Apk, *Bpk;
  const int *EA, *EB;
  int32_t *S;
  int64_t mbp, nbp, kbp, plane;
  int kbc, nchunks, groups, D, m, n, ldc;
  double *C;
  int64_t c_stride;
};

// One product of a batch, as read by the persistent GEMM kernel.
struct PlainGemmDesc {
  const void *Apk, *Bpk;
  int64_t mbp, nbp, kbp;
  int m, n, D, ldc;
  void *C;
  int64_t c_stride;
};

// Fused plain split: a workgroup of 512 or 1024 threads holds the residual of
// nv whole vectors in registers, fused_per_thread<T, C>() elements per thread.
template <typename T, int C>
__host__ __device__ constexpr int fused_per_thread() {
  return sizeof(T) == 8 ? (C == 2 ? 16 : C == 3 ? 10 : 8) : 16;
}
// Vectors per workgroup of `threads` threads (16, 8, 4, 2 or 1; a divisor of
// the 16 of a packed block) for vectors of padded length len_cover; 0 when not
// even one fits.
__host__ __device__ inline int fused_vectors(int64_t len_cover, int per_thread, int threads) {
  for (int nv = kBlk; nv >= 1; nv /= 2)
    if (nv * len_cover <= (int64_t)threads * per_thread) return nv;
  return 0;
}
// Threads of a fused-split workgroup for vectors of padded length len_cover:
// 512 while 4 or more vectors fit (two workgroups share a CU, one computing
// while the other waits for its loads); else 1024 while 2 fit (fewer vectors
// per workgroup cut the reads of A's rows and the slice stores into short
// runs); 0 when the vectors are too long to fuse.
template <typename T, int C>
inline int fused_threads(int64_t len_cover) {
  if (fused_vectors(len_cover, fused_per_thread<T, C>(), 512) >= 4) return 512;
  if (fused_vectors(len_cover, fused_per_thread<T, C>(), 1024) >= 2) return 1024;
  return 0;
}
// Workgroups of `threads` threads of the fused split for one operand; -1 if
// its vectors do not fit them as fused_threads allows.
template <typename T, int C, typename Op>
inline int fused_strips(const Op &op, int threads) {
  const int ft = fused_threads<T, C>(op.kbp * kKBlk);
  if (ft == 0 || ft > threads) return -1;
  const int nv = fused_vectors(op.kbp * kKBlk, fused_per_thread<T, C>(), threads);
  return op.nvec > 0 ? (int)(op.nbp * kBlk / nv) : 0;
}

// Plain split (Algorithm 1): D passes, slices written packed.  `rho` is the
// shift ceil((S + log2 k)/2).  Both operands in one sequence of launches: one
// fused launch when `fused` is set and their vectors fit, else D + 1 sweeps.
template <typename T, int C>
hipError_t launch_split_plain(const SplitOperand<T> &a, const SplitOperand<T> &b, int D, int rho, bool fused,
                              hipStream_t st);

// Plain split of many operands at once: ops[0..nops) in device memory.
// prefix_fused (nops + 1 entries, device) holds running sums of the fused
// workgroups (of fused_nt threads) of each operand (0 for operands left to the
// pass kernels);
// prefix_max0 / prefix_pass the running sums of the 64 x 64 tiles each
// remaining operand needs in the max and pass kernels (0 for fused operands).
// Operand i runs ops[i].D passes; pass launches cover dmax passes.  mu_all /
// mu_words: one region holding every operand's maxima, cleared first.
template <typename T, int C>
hipError_t launch_split_plain_batched(const SplitOperand<T> *ops, const int *prefix_max0, const int *prefix_pass,
                                      const int *prefix_fused, int nops, int tiles_max0, int tiles_pass,
                                      int strips_fused, int fused_nt, int dmax, void *mu_all, int64_t mu_words,
                                      hipStream_t st);

// Persistent GEMM over a batch: items (product index, tile index) in device
// memory, in kXcds per-XCD lists (bounds: kXcds + 1 running offsets; counters:
// kXcds words, cleared by the caller; take_item).
template <typename T, int C>
hipError_t launch_gemm_plain_batched(const PlainGemmDesc *descs, const int2 *items, const int *bounds, int *counters,
                                     int grid, int layout, hipStream_t st);

// INT8 digit split of both operands.
template <int C>
hipError_t launch_split_int8(const SplitOperand<double> &a, const SplitOperand<double> &b, int D, hipStream_t st);

// INT8 digit split of many operands at once (operand i: ops[i].D digits, at
// most dmax).  prefix_max0: running sums of each operand's 64 x 64 max-kernel
// tiles; prefix_blk: running sums of its 32 x 32 packed blocks (nbp * kbp).
template <int C>
hipError_t launch_split_int8_batched(const SplitOperand<double> *ops, const int *prefix_max0, const int *prefix_blk,
                                     int nops, int tiles_max0, int64_t blocks, int dmax, void *mu_all,
                                     int64_t mu_words, hipStream_t st);

// INT8-form batch: persistent GEMMs over items (product, tile, k chunk,
// diagonal group): items[0, nitems1) in the 128 x 128 configuration (their
// products' slices padded to 128 rows), then nitems3 in the 256 x 256 one,
// each in kXcds per-XCD lists (bounds[0, kXcds] over the first items,
// bounds[kXcds + 1, 2 kXcds + 1] over the second, relative to their first
// item; counters: 2 kXcds words, cleared by the caller; take_item); then the
// combine of every product, prefix_blocks giving the running sums of the
// 32 x 32 blocks of each product's C.
template <int C>
hipError_t launch_int8_batched(const Int8GemmDesc *descs, const int4 *items, int nitems1, int nitems3,
                               const int *bounds, int *counters, const int *prefix_blocks, int nprod, int64_t blocks,
                               hipStream_t st);

// Fused slice-product GEMM with error-free accumulation into C (C components).
// single_pair >= 0 selects debug mode: only pair (a, b) = (single_pair / D,
// single_pair % D) (0-based) is formed and written raw as binary64 into Cdbg.
// `layout` selects the wavefront layout of the 64 x 64 tile (1: 4 waves of
// 32 x 32, 2: 8 waves of 32 x 16, 3: 16 waves of 16 x 16).
template <typename T, int C>
hipError_t launch_gemm_plain(const void *Apk, const void *Bpk, int64_t mbp, int64_t nbp, int64_t kbp, int m, int n,
                             int D, T *Cout, int ldc, int64_t c_stride, int single_pair, double *Cdbg, int lddbg,
                             int layout, hipStream_t st);

// The fused GEMM with a pair set per 64 x 64 tile: tile (tm, tn) forms the
// pairs (a, b) (0-based) with b < lims[(tn * tiles_m + tm) * D + a], a
// staircase within D x D (D <= kMaxPairLim), written by launch_tile_pairs.
template <typename T, int C>
hipError_t launch_gemm_plain_pruned(const void *Apk, const void *Bpk, int64_t mbp, int64_t nbp, int64_t kbp, int m,
                                    int n, int D, T *Cout, int ldc, int64_t c_stride, const int8_t *lims, int layout,
                                    hipStream_t st);

// Pair sets from the data (binary64/binary32 slices, D passes done): for each
// 64 x 64 tile of C, the fewest pairs whose left-out bounds, added to the
// remainder and rounding terms of the certificate, keep every entry of the
// tile within 2^-t of its lower bound of (|A||B|)_ij.  raw: the binary64
// product |A_0| |B_0| (m x n, leading dimension m); rs_a / cs_b: row sums of
// |A_0| and column sums of |B_0|.  Writes lims (tiles x D bytes, tile index
// tn * tiles_m + tm).
hipError_t launch_tile_pairs(int m, int n, int k, int D, int rho, int S, int comps, int t, const int *eA,
                             const int *eB, const double *rs_a, const double *cs_b, const double *raw,
                             int64_t tiles_m, int64_t tiles_n, int8_t *lims, hipStream_t st);

// The certificate's pieces (certify.hip) without its final pass: |A_0| and
// |B_0| packed into pack_a / pack_b, the row and column sums into rs_a / cs_b,
// and the single-pair product |A_0| |B_0| into raw (two planes of m x n).
template <typename T>
hipError_t launch_abs_lead_product(const SplitOperand<T> &a, const SplitOperand<T> &b, int m, int n, double *raw,
                                   double *pack_a, double *pack_b, double *rs_a, double *cs_b, int layout,
                                   hipStream_t st);

// INT8 form GEMM: diagonal sums S_g into Sws (D x nchunks planes of m x n
// int32), then their exact combination into C.  debug_g > 0 writes S_g for
// that g as int64 into Sdbg instead of forming C.
// cfg: INT8 tile configuration (0 automatic; 1: 128 x 128 with 4 wavefronts,
// 2: 256 x 256 with 4, 3: 256 x 256 with 8).
template <int C>
hipError_t launch_gemm_int8(const void *Apk, const void *Bpk, const int *EA, const int *EB, int32_t *Sws, int64_t mbp,
                            int64_t nbp, int64_t kbp, int m, int n, int D, double *Cout, int ldc, int64_t c_stride,
                            int debug_g, int64_t *Sdbg, int lddbg, int cfg, hipStream_t st);
// k blocks (32 wide) per chunk of the INT8 GEMM for D digit slices.
int int8_kblocks_per_chunk(int D);
// INT8 GEMM tile configuration for an m x n product (cfg in 1..3 forces one,
// 0 chooses by size), and its tile edge in 32-row blocks.
int int8_tile_config(int64_t m, int64_t n, int cfg);
inline int int8_tile_blocks(int cfg) { return cfg == 1 ? 4 : 8; }

// A-posteriori certificate of a binary64/binary32-slice product whose split
// (a, b: exponents filled) and GEMM have been enqueued: per entry, an upper
// bound of |C - AB| into plane 0 of `cert` and a lower bound of (|A||B|)_ij
// into plane 1 (m x n each, column-major, leading dimension m), and the largest
// ratio of the two into *worst.  pack_a / pack_b (the packed slice planes,
// reused) and rs_a / cs_b (m and n doubles) are scratch.
// int8: the split was the INT8 digit split (exps: E per vector); a and b then
// carry the binary64 packed geometry (nbp, kbp) for |A_0| and |B_0|.
// lims (may be NULL): the per-tile pair sets of launch_tile_pairs the product
// was formed with (pairs outside them count as left out), else the triangle.
// raw_ready: the |A_0| |B_0| product and the sums are already in cert plane 0
// and rs_a / cs_b (the pair sets were chosen from them).
template <typename T>
hipError_t launch_certify(const SplitOperand<T> &a, const SplitOperand<T> &b, int m, int n, int k, int D, int rho,
                          int comps, int int8, double *cert, double *worst, double *pack_a, double *pack_b,
                          double *rs_a, double *cs_b, int layout, hipStream_t st, const int8_t *lims = nullptr,
                          bool raw_ready = false);

// LU of a DD (comps = 2) or TD (comps = 3) matrix (comps planes of ld x n,
// `plane` doubles apart): panel step at column j0 with width K (diagonal block,
// then U12 and L21), block copy into a contiguous matrix, A22 -= P, and the
// solve of L U x = b.
hipError_t launch_lu_panel(int comps, double *A, int64_t ld, int64_t plane, int j0, int K, int n, hipStream_t st);
hipError_t launch_lu_copy(int comps, double *A, int64_t ld, int64_t plane, int r0, int c0, int rows, int cols,
                          double *out, hipStream_t st);
hipError_t launch_lu_sub(int comps, double *A, int64_t ld, int64_t plane, int r0, int c0, int rows, int cols,
                         const double *P, hipStream_t st);
hipError_t launch_lu_solve(int comps, const double *A, int64_t ld, int64_t plane, int n, double *x,
                           hipStream_t st);

// Debug: unpack D packed slices into planes of rows x cols (column-major, ld rows).
hipError_t launch_unpack(int elem_bytes, const void *packed, int64_t nbp, int64_t kbp, int D, int orient, int rows,
                         int cols, void *out, hipStream_t st);

// Fill n 32-bit words with a value (used instead of memset so that the
// sequence stays capturable in a graph).
hipError_t launch_fill32(void *p, int64_t nwords, uint32_t value, hipStream_t st);

// Simple (non-Ozaki) in-format products: C = A B by the triple loop in the
// format's arithmetic (F = 0 DD, 1 TD, 2 QD, 3 TS), operands planar as the
// C-ABI's; staged: operand panels through LDS, else read from global memory.
template <int F>
hipError_t launch_simple(int m, int n, int k, const void *A, int lda, const void *B, int ldb, void *Cm, int ldc,
                         bool staged, hipStream_t st);
// The same for D+S (binary64 hi plane, binary32 lo plane): DD arithmetic, C
// rounded to D+S.
hipError_t launch_simple_ds(int m, int n, int k, const double *Ahi, const float *Alo, int lda, const double *Bhi,
                            const float *Blo, int ldb, double *Chi, float *Clo, int ldc, bool staged,
                            hipStream_t st);
// D+S (leading dimension ld) <-> two compact binary64 planes (rows x cols).
hipError_t launch_ds_to_dd(int rows, int cols, const double *hi, const float *lo, int ld, double *out,
                           hipStream_t st);
hipError_t launch_dd_to_ds(int rows, int cols, const double *in, double *hi, float *lo, int ld, hipStream_t st);

// C := 0 for an m x n multi-component matrix.
hipError_t launch_zero_matrix(void *C, int elem_bytes, int comps, int m, int n, int ldc, int64_t c_stride,
                              hipStream_t st);

}  // namespace mp
