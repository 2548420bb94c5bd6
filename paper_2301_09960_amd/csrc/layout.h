// Packed slice layout shared by the split kernels (writers) and the
// matrix-core GEMM kernels (readers).  Host and device.
//
// A slice matrix is stored as 16 x 16 blocks ("row/col block" x "k block"),
// each block laid out in the order in which one 64-lane wavefront feeds it to
// the 16x16x4 matrix-core instructions:
//   lane l holds the 16-element row/column index l % 16 and, over four
//   instructions s = 0..3, the k indices 4 s + l / 16 of the block.
// Within a block of 256 elements the value for (lane l, step s) sits at
//   binary64:  (s / 2) * 128 + 2 l + (s % 2)   (two 16-byte loads per lane,
//              each contiguous across the wavefront)
//   binary32:  4 l + s                         (one 16-byte load per lane)
// Blocks of one row/column block are consecutive along k; a slice is
// [nb][kb][256] with nb row/column blocks and kb k-blocks; slices follow one
// another.  Padding (rows beyond m, k beyond k) holds zeros.
//
// INT8 digit slices use 32 x 32 blocks for the 32x32x32 integer instruction:
// lane l holds row/column index l % 32 and the 16 consecutive k values
// 16 (l / 32) + t, t = 0..15, stored as 16 bytes at 16 l + t.  Rows/columns
// are padded to the INT8 GEMM tile in use (128 or 256), k to 128 (a multiple of
// every INT8 k step).
#pragma once

#include <stdint.h>

namespace mp {

constexpr int kBlk = 16;      // rows/cols per block
constexpr int kKBlk = 16;     // k per block (floating-point slices)
constexpr int kBlk8 = 32;     // rows/cols per block (INT8 slices)
constexpr int kKBlk8 = 32;    // k per block (INT8 slices)
constexpr int kTileBlocks8 = 8;   // largest INT8 tile: 8 blocks (256 rows); the 128-row tile uses 4
constexpr int kKStepBlocks8 = 2;  // INT8 k padding unit: 2 k-blocks (64); k steps are 2 or 4 blocks
constexpr int kTileBlocks = 4;  // GEMM tile = 4 x 4 blocks (64 x 64)
constexpr int kKStepBlocks = 2; // GEMM k step = 2 k-blocks (32)
constexpr int kMaxPairLim = 16; // most slices of the data-chosen pair sets (per-tile staircases)

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Padded block counts: rows/cols padded to the GEMM tile, k to the k step.
__host__ __device__ inline int64_t nblocks_padded(int64_t rows) {
  return ceil_div(rows, kBlk * kTileBlocks) * kTileBlocks;
}
__host__ __device__ inline int64_t kblocks_padded(int64_t k) {
  return ceil_div(k, kKBlk * kKStepBlocks) * kKStepBlocks;
}
// INT8 rows/columns are padded to the tile of the GEMM configuration that will
// consume them (tile_blocks = 4 or 8 blocks of 32).
__host__ __device__ inline int64_t nblocks8_padded(int64_t rows, int tile_blocks) {
  return ceil_div(rows, (int64_t)kBlk8 * tile_blocks) * tile_blocks;
}
__host__ __device__ inline int64_t kblocks8_padded(int64_t k) {
  return ceil_div(k, kKBlk8 * kKStepBlocks8) * kKStepBlocks8;
}

// Offset (in elements) of element (v, p) of slice a: v = row of A / column of B,
// p = k index.  nbp / kbp: padded block counts.
template <bool F64>
__host__ __device__ inline int64_t packed_index(int64_t a, int64_t v, int64_t p, int64_t nbp, int64_t kbp) {
  const int64_t vb = v / kBlk, vl = v % kBlk;
  const int64_t kb = p / kKBlk, kl = p % kKBlk;
  const int64_t lane = (kl % 4) * 16 + vl;
  const int64_t s = kl / 4;
  const int64_t within = F64 ? (s / 2) * 128 + 2 * lane + (s % 2) : 4 * lane + s;
  return ((a * nbp + vb) * kbp + kb) * 256 + within;
}

__host__ __device__ inline int64_t packed_index8(int64_t a, int64_t v, int64_t p, int64_t nbp, int64_t kbp) {
  const int64_t vb = v / kBlk8, vl = v % kBlk8;
  const int64_t kb = p / kKBlk8, kl = p % kKBlk8;
  const int64_t lane = (kl / 16) * 32 + vl;
  return ((a * nbp + vb) * kbp + kb) * 1024 + 16 * lane + (kl % 16);
}

}  // namespace mp
