// Fused slice-product GEMM with error-free accumulation (Section 3,
// Algorithm 1: C_ab = A_a B_b for a + b <= D + 1, then C := C + sum C_ab in
// the long format).
//
// One workgroup (4 wavefronts) owns a 64 x 64 tile of C.  For every slice pair
// of the triangle it runs the whole k loop on the matrix cores
// (v_mfma_f64_16x16x4f64 for binary64 slices, v_mfma_f32_16x16x4f32 for
// binary32); the split chose slice widths so that every partial sum of a slice
// product is representable, so the matrix-core result is the exact C_ab.  The
// exact tile is then added with TwoSum into a (c+1)-term accumulator held in
// registers; after the last pair the accumulator is renormalized and its top c
// terms are stored.  Slice products never reach memory.
//
// Operand staging: slices arrive packed in wavefront order (layout.h); each
// k step (32) of a pair moves a 64 x 32 panel of A_a and of B_b (16 KiB each
// for binary64) from global memory into one of two LDS buffers with 16-byte
// loads that are contiguous across each wavefront, while the matrix cores
// work on the other buffer.  The pair loop and the k loop form one pipelined
// sequence of steps.  Pairs are visited with b innermost, so a workgroup reads
// A_a for several consecutive pairs; workgroups on one XCD (its own L2) are
// given neighbouring tiles.
#include "internal.h"
#include "layout.h"
#include "mp_device.h"

namespace mp {
namespace {

constexpr int kThreads = 256;
constexpr int kGroupM = 8;  // tile rows per group in the XCD-local ordering

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<double> {
  using acc_t = d4;
  // out = src0 (16 x 4) * src1 (4 x 16) + acc; lane l holds src0[l%16][l/16], src1[l/16][l%16]
  static __device__ __forceinline__ acc_t run(double s0, double s1, acc_t acc) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(s0, s1, acc, 0, 0, 0);
  }
  // row (src0 index) of output element r of lane l; the column is l % 16
  static __device__ __forceinline__ int out_row(int l, int r) { return l / 16 + 4 * r; }
};
template <> struct Mma<float> {
  using acc_t = f4;
  static __device__ __forceinline__ acc_t run(float s0, float s1, acc_t acc) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(s0, s1, acc, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int l, int r) { return 4 * (l / 16) + r; }
};

// Remaps the hardware block index so that each XCD (blocks are dealt round
// robin over the 8 XCDs) works on a contiguous range of tiles, then orders
// tiles in groups of kGroupM tile rows so concurrent workgroups share panels.
__device__ __forceinline__ void tile_coords(int bid, int nblocks, int tiles_m, int tiles_n, int &tm, int &tn) {
  const int q = nblocks / 8, r = nblocks % 8;
  const int xcd = bid % 8, local = bid / 8;
  const int L = xcd * q + (xcd < r ? xcd : r) + local;
  const int per_group = kGroupM * tiles_n;
  const int group = L / per_group;
  const int first_m = group * kGroupM;
  const int gsize = (tiles_m - first_m) < kGroupM ? (tiles_m - first_m) : kGroupM;
  const int in_group = L % per_group;
  tm = first_m + in_group % gsize;
  tn = in_group / gsize;
}

template <typename T>
constexpr int panel_elems() {
  return kTileBlocks * kKStepBlocks * 256;  // 64 rows x 32 k
}

// All slice products of one 64 x 64 tile (tm, tn) of one product, folded into
// C.  `lds` is the workgroup's staging buffer [stage][A,B][panel].
template <typename T, int C>
__device__ void gemm_plain_tile(const T *__restrict__ Apk, const T *__restrict__ Bpk, int64_t mbp, int64_t nbp,
                                int64_t kbp, int m, int n, int D, T *__restrict__ Cout, int ldc, int64_t c_stride,
                                int single_pair, double *__restrict__ Cdbg, int lddbg, int tm, int tn,
                                T (*lds)[2][panel_elems<T>()]) {
  using M = Mma<T>;
  using acc_t = typename M::acc_t;
  constexpr int kSegElems = kKStepBlocks * 256;       // one row block x one k step
  constexpr int kPanelElems = panel_elems<T>();
  constexpr int kVec = sizeof(T) / 2;                   // 16-byte loads per thread per operand
  static_assert(kVec * 16 * kThreads == kPanelElems * (int)sizeof(T), "panel staging");

  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int wm = wave % 2, wn = wave / 2;  // 32 x 32 sub-tile of this wavefront

  const int nks = (int)(kbp / kKStepBlocks);
  const int npairs = single_pair >= 0 ? 1 : D * (D + 1) / 2;
  const int64_t total = (int64_t)npairs * nks;

  // load cursor
  int la = single_pair >= 0 ? single_pair / D : 0, lb = single_pair >= 0 ? single_pair % D : 0, lks = 0;
  const int seg = tid / 64;  // row block of the panel this thread moves
  u4 ra[kVec], rb[kVec];

  auto load_step = [&](int a, int b, int ks) {
    const u4 *pa = reinterpret_cast<const u4 *>(Apk + (((int64_t)a * mbp + tm * kTileBlocks + seg) * kbp +
                                                       (int64_t)ks * kKStepBlocks) * 256);
    const u4 *pb = reinterpret_cast<const u4 *>(Bpk + (((int64_t)b * nbp + tn * kTileBlocks + seg) * kbp +
                                                       (int64_t)ks * kKStepBlocks) * 256);
#pragma unroll
    for (int j = 0; j < kVec; ++j) {
      ra[j] = pa[j * 64 + lane];
      rb[j] = pb[j * 64 + lane];
    }
  };
  auto store_stage = [&](int stage) {
    u4 *sa = reinterpret_cast<u4 *>(&lds[stage][0][seg * kSegElems]);
    u4 *sb = reinterpret_cast<u4 *>(&lds[stage][1][seg * kSegElems]);
#pragma unroll
    for (int j = 0; j < kVec; ++j) {
      sa[j * 64 + lane] = ra[j];
      sb[j * 64 + lane] = rb[j];
    }
  };
  auto advance = [&](int &a, int &b, int &ks) {
    if (++ks == nks) {
      ks = 0;
      if (single_pair < 0) {
        if (a + ++b > D - 1) {
          ++a;
          b = 0;
        }
      }
    }
  };

  acc_t acc[2][2];
  T sum[2][2][4][C + 1];
#pragma unroll
  for (int jb = 0; jb < 2; ++jb)
#pragma unroll
    for (int ib = 0; ib < 2; ++ib) {
      acc[jb][ib] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q <= C; ++q) sum[jb][ib][r][q] = T(0);
    }

  load_step(la, lb, lks);
  store_stage(0);
  advance(la, lb, lks);
  __syncthreads();

  int cks = 0;  // k step of the pair being computed
  for (int64_t step = 0; step < total; ++step) {
    const int stage = (int)(step & 1);
    const bool more = step + 1 < total;
    if (more) load_step(la, lb, lks);

    // matrix-core work on this stage: 2 k blocks x 4 instructions per 16 x 16 block
#pragma unroll
    for (int kb = 0; kb < kKStepBlocks; ++kb) {
      T fa[2][4], fb[2][4];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const T *pa = &lds[stage][0][((wm * 2 + x) * kKStepBlocks + kb) * 256];
        const T *pb = &lds[stage][1][((wn * 2 + x) * kKStepBlocks + kb) * 256];
        if constexpr (sizeof(T) == 8) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const d2 va = *reinterpret_cast<const d2 *>(pa + h * 128 + 2 * lane);
            const d2 vb = *reinterpret_cast<const d2 *>(pb + h * 128 + 2 * lane);
            fa[x][2 * h] = va[0];
            fa[x][2 * h + 1] = va[1];
            fb[x][2 * h] = vb[0];
            fb[x][2 * h + 1] = vb[1];
          }
        } else {
          const f4 va = *reinterpret_cast<const f4 *>(pa + 4 * lane);
          const f4 vb = *reinterpret_cast<const f4 *>(pb + 4 * lane);
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            fa[x][s] = va[s];
            fb[x][s] = vb[s];
          }
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
          for (int ib = 0; ib < 2; ++ib) acc[jb][ib] = M::run(fb[jb][s], fa[ib][s], acc[jb][ib]);
    }

    if (++cks == nks) {  // the pair's product is complete and exact: fold it in
      cks = 0;
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc_add<T, C + 1>(sum[jb][ib][r], acc[jb][ib][r]);
          acc[jb][ib] = acc_t{0, 0, 0, 0};
        }
    }

    if (more) {
      store_stage(stage ^ 1);
      advance(la, lb, lks);
    }
    __syncthreads();
  }

  // store: element (i, j) with i along the lanes (contiguous in column-major C)
#pragma unroll
  for (int jb = 0; jb < 2; ++jb)
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = tm * 64 + wm * 32 + ib * 16 + lane % 16;
        const int j = tn * 64 + wn * 32 + jb * 16 + M::out_row(lane, r);
        if (i >= m || j >= n) continue;
        if (single_pair >= 0) {
          Cdbg[i + (int64_t)j * lddbg] = (double)sum[jb][ib][r][0];
        } else {
          T v[C + 1];
#pragma unroll
          for (int q = 0; q <= C; ++q) v[q] = sum[jb][ib][r][q];
          renorm<T, C + 1>(v);
#pragma unroll
          for (int q = 0; q < C; ++q) Cout[q * c_stride + i + (int64_t)j * ldc] = v[q];
        }
      }
}

template <typename T, int C>
__global__ __launch_bounds__(kThreads) void k_gemm_plain(const T *__restrict__ Apk, const T *__restrict__ Bpk,
                                                         int64_t mbp, int64_t nbp, int64_t kbp, int m, int n, int D,
                                                         T *__restrict__ Cout, int ldc, int64_t c_stride,
                                                         int single_pair, double *__restrict__ Cdbg, int lddbg) {
  __shared__ __attribute__((aligned(16))) T lds[2][2][panel_elems<T>()];
  int tm, tn;
  tile_coords(blockIdx.x, gridDim.x, (int)(mbp / kTileBlocks), (int)(nbp / kTileBlocks), tm, tn);
  gemm_plain_tile<T, C>(Apk, Bpk, mbp, nbp, kbp, m, n, D, Cout, ldc, c_stride, single_pair, Cdbg, lddbg, tm, tn, lds);
}

// Persistent batched kernel: each workgroup takes (product, tile) work items
// from a shared counter until the list is exhausted (items are ordered by
// decreasing work, so the long tiles start first).
template <typename T, int C>
__global__ __launch_bounds__(kThreads) void k_gemm_plain_batched(const PlainGemmDesc *__restrict__ descs,
                                                                 const int2 *__restrict__ items, int nitems,
                                                                 int *__restrict__ counter) {
  __shared__ __attribute__((aligned(16))) T lds[2][2][panel_elems<T>()];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int it = next;
    __syncthreads();
    if (it >= nitems) break;
    const int2 w = items[it];
    const PlainGemmDesc &d = descs[w.x];
    const int tiles_m = (int)(d.mbp / kTileBlocks);
    gemm_plain_tile<T, C>(static_cast<const T *>(d.Apk), static_cast<const T *>(d.Bpk), d.mbp, d.nbp, d.kbp, d.m,
                          d.n, d.D, static_cast<T *>(d.C), d.ldc, d.c_stride, -1, nullptr, 0, w.y % tiles_m,
                          w.y / tiles_m, lds);
  }
}

}  // namespace

template <typename T, int C>
hipError_t launch_gemm_plain_batched(const PlainGemmDesc *descs, const int2 *items, int nitems, int *counter,
                                     int grid, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_gemm_plain_batched<T, C>), dim3((unsigned)grid), dim3(kThreads), 0, st, descs, items, nitems,
                     counter);
  return hipGetLastError();
}

template hipError_t launch_gemm_plain_batched<double, 2>(const PlainGemmDesc *, const int2 *, int, int *, int,
                                                         hipStream_t);
template hipError_t launch_gemm_plain_batched<double, 3>(const PlainGemmDesc *, const int2 *, int, int *, int,
                                                         hipStream_t);
template hipError_t launch_gemm_plain_batched<double, 4>(const PlainGemmDesc *, const int2 *, int, int *, int,
                                                         hipStream_t);
template hipError_t launch_gemm_plain_batched<float, 3>(const PlainGemmDesc *, const int2 *, int, int *, int,
                                                        hipStream_t);

template <typename T, int C>
hipError_t launch_gemm_plain(const void *Apk, const void *Bpk, int64_t mbp, int64_t nbp, int64_t kbp, int m, int n,
                             int D, T *Cout, int ldc, int64_t c_stride, int single_pair, double *Cdbg, int lddbg,
                             hipStream_t st) {
  const int64_t tiles = (mbp / kTileBlocks) * (nbp / kTileBlocks);
  if (tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_gemm_plain<T, C>), dim3((unsigned)tiles), dim3(kThreads), 0, st,
                     static_cast<const T *>(Apk), static_cast<const T *>(Bpk), mbp, nbp, kbp, m, n, D, Cout, ldc,
                     c_stride, single_pair, Cdbg, lddbg);
  return hipGetLastError();
}

template hipError_t launch_gemm_plain<double, 2>(const void *, const void *, int64_t, int64_t, int64_t, int, int, int,
                                                 double *, int, int64_t, int, double *, int, hipStream_t);
template hipError_t launch_gemm_plain<double, 3>(const void *, const void *, int64_t, int64_t, int64_t, int, int, int,
                                                 double *, int, int64_t, int, double *, int, hipStream_t);
template hipError_t launch_gemm_plain<double, 4>(const void *, const void *, int64_t, int64_t, int64_t, int, int, int,
                                                 double *, int, int64_t, int, double *, int, hipStream_t);
template hipError_t launch_gemm_plain<float, 3>(const void *, const void *, int64_t, int64_t, int64_t, int, int, int,
                                                float *, int, int64_t, int, double *, int, hipStream_t);

}  // namespace mp
