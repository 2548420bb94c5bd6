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

// Wave layouts of the 64 x 64 tile: WM x WN wavefronts, each owning
// (4 / WM) x (4 / WN) blocks of 16 x 16.
//   layout 1: 2 x 2 waves, 32 x 32 each (256 threads)
//   layout 2: 2 x 4 waves, 32 x 16 each (512 threads)
//   layout 3: 4 x 4 waves, 16 x 16 each (1024 threads)
// Fewer elements per lane means fewer accumulator registers and more
// wavefronts per SIMD to hide latency, at the price of more LDS reads per
// matrix-core instruction.
template <int L> struct Layout;
template <> struct Layout<1> { static constexpr int WM = 2, WN = 2; };
template <> struct Layout<2> { static constexpr int WM = 2, WN = 4; };
template <> struct Layout<3> { static constexpr int WM = 4, WN = 4; };

// Wavefronts per SIMD the register allocation must allow.  Layout 1 with
// three or four components is left free: forcing two wavefronts into 256
// registers made those schedules far slower than one wavefront that keeps its
// matrix-core accumulators in AGPRs.  Binary64 layout 2 is capped at 128
// registers so that two workgroups of eight wavefronts share a CU (their
// two-stage rings take 64 KiB of LDS each): while one waits on its loads the
// other keeps the matrix cores busy.
constexpr int waves_of(int layout, int C, int bytes) {
  return layout == 3 ? 4 : layout == 2 ? (bytes == 8 ? 4 : 2) : (C <= 2 ? 2 : 1);
}

// 16 bytes per lane from global memory straight into LDS: lane l's bytes land
// at lds_dst + 16 l (lds_dst is the same for the whole wavefront).
__device__ __forceinline__ void load_lds16(const void *src, void *lds_dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds_dst, 16, 0, 0);
}

// Waits until at most N vector-memory operations of this wavefront are in
// flight (the LDS-direct loads of later pipeline stages).
template <int N>
__device__ __forceinline__ void wait_vm() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Operand staging: every k step (32) of a pair needs a 64 x 32 panel of A_a and
// one of B_b; the panels arrive by global-to-LDS loads (16 bytes per lane,
// 1 KiB per wavefront instruction, no registers involved) into a ring of NS
// stages, issued NS - 1 steps ahead of the matrix-core work.  A step waits
// only for its own loads (s_waitcnt on the count of later loads still in
// flight), then one barrier makes every wavefront's loads visible.
template <typename T>
constexpr int stage_elems() {
  return 2 * panel_elems<T>();  // A panel, then B panel
}
// Ring depth: binary64 stages take 32 KiB, so two of them leave room for a
// second workgroup per CU (which hides latency better than a deeper ring);
// binary32 stages take 16 KiB and four of them still fit twice.
template <typename T>
constexpr int stages_of() {
  return sizeof(T) == 8 ? 2 : 4;
}

// Waits until this wavefront's loads of the step about to be computed have
// landed: with an NS-stage ring, min(NS - 2, later) later steps (kL loads
// each) may stay in flight.
template <int NS, int kL>
__device__ __forceinline__ void wait_step(int64_t later) {
  if constexpr (NS >= 4) {
    if (later >= 2)
      wait_vm<2 * kL>();
    else if (later == 1)
      wait_vm<kL>();
    else
      wait_vm<0>();
  } else if constexpr (NS == 3) {
    if (later >= 1)
      wait_vm<kL>();
    else
      wait_vm<0>();
  } else {
    wait_vm<0>();
  }
}

// A tile's pair staircase: count a (0..16) in byte a of two 64-bit words,
// held in scalar registers (no memory access on the pair walk).
struct Staircase {
  uint64_t lo, hi;
  __device__ __forceinline__ int operator()(int a) const {
    return (int)(((a < 8 ? lo >> (8 * a) : hi >> (8 * (a - 8)))) & 0xff);
  }
};

// All slice products of one 64 x 64 tile (tm, tn) of one product, folded into
// C.  `lds` is the workgroup's ring of stages_of<T>() staging buffers of
// stage_elems<T>() elements each.  The pairs are (a, b), 0-based, with
// b < lim(a): the triangle a + b <= D - 1 (lim(a) = D - a), or with PRUNE the
// tile's own staircase lim(a) = stair(a) (non-increasing in a, at most D).
template <typename T, int C, int LAYOUT, bool PRUNE = false>
__device__ __forceinline__ void gemm_plain_tile(const T *__restrict__ Apk, const T *__restrict__ Bpk, int64_t mbp, int64_t nbp,
                                int64_t kbp, int m, int n, int D, T *__restrict__ Cout, int ldc, int64_t c_stride,
                                int single_pair, double *__restrict__ Cdbg, int lddbg, int tm, int tn,
                                T *lds, Staircase stair = Staircase{0, 0}) {
  using M = Mma<T>;
  using acc_t = typename M::acc_t;
  constexpr int WM = Layout<LAYOUT>::WM, WN = Layout<LAYOUT>::WN;
  constexpr int BI = kTileBlocks / WM, BJ = kTileBlocks / WN;  // 16 x 16 blocks per wavefront
  constexpr int NW = WM * WN;
  constexpr int kSegElems = kKStepBlocks * 256;              // one row block x one k step
  constexpr int kPanelElems = panel_elems<T>();
  constexpr int kInstElems = 64 * 16 / (int)sizeof(T);       // elements one wavefront instruction moves
  constexpr int kInstPerSeg = kSegElems / kInstElems;
  constexpr int kInstPerPanel = kTileBlocks * kInstPerSeg;
  constexpr int kL = 2 * kInstPerPanel / NW;                 // instructions per wavefront per step
  constexpr int kStages = stages_of<T>();
  static_assert(kStages >= 2 && kStages <= 4, "wait chain covers rings of 2 to 4 stages");
  static_assert(2 * kInstPerPanel % NW == 0, "staging split");

  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  // wavefront -> (wm, wn).  With 2 x 4 wavefronts (two per SIMD: w and w + 4)
  // the two of a SIMD differ in both wm and wn, so that a tile padded in m or
  // in n leaves each SIMD a wavefront with work.
  int wm, wn;
  if constexpr (WM == 2 && WN == 4) {
    const int sw = wave & 3, hw = wave >> 2;
    wm = (sw & 1) ^ hw;
    wn = (sw >> 1) + 2 * hw;
  } else {
    wm = wave % WM;
    wn = wave / WM;
  }

  const int nks = (int)(kbp / kKStepBlocks);
  auto lim = [&](int a) -> int {
    if constexpr (PRUNE)
      return stair(a);
    else
      return D - a;
  };
  int npairs = single_pair >= 0 ? 1 : D * (D + 1) / 2;
  if constexpr (PRUNE) {
    npairs = 0;
    for (int a = 0; a < D; ++a) npairs += stair(a);
  }
  const int64_t total = (int64_t)npairs * nks;

  // this wavefront's share of a step: operand op_w and kL consecutive 1 KiB
  // pieces of its panel, starting at piece r0.  Piece j sits at a fixed
  // offset from the step's panel base: g0 (per lane) plus a uniform term, so a
  // load costs one 64-bit add.
  static_assert(kInstPerPanel % kL == 0, "a wavefront's loads of a step come from one operand");
  constexpr bool kOneSeg = kL <= kInstPerSeg;
  static_assert(kOneSeg ? kInstPerSeg % kL == 0 : kL % kInstPerSeg == 0, "pieces tile the segments");
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  const int op_w = (wave_u * kL) / kInstPerPanel;
  const int r0 = (wave_u * kL) % kInstPerPanel;
  const int sg0 = r0 / kInstPerSeg, part0 = r0 % kInstPerSeg;
  const int64_t seg_bytes = kbp * 256 * (int64_t)sizeof(T);  // one row block to the next (k <= 2^20: < 2^32 / 4)
  const uint32_t g0 = (uint32_t)(sg0 * seg_bytes + part0 * 1024) + 16u * (uint32_t)lane;
  const int l0 = op_w * kPanelElems + sg0 * kSegElems + part0 * kInstElems;
  auto goff = [&](int j) -> int64_t {
    return kOneSeg ? (int64_t)j * 1024 : (int64_t)(j / kInstPerSeg) * seg_bytes + (j % kInstPerSeg) * 1024;
  };
  auto loff = [&](int j) -> int {
    return kOneSeg ? j * kInstElems : (j / kInstPerSeg) * kSegElems + (j % kInstPerSeg) * kInstElems;
  };

  int la = single_pair >= 0 ? single_pair / D : 0, lb = single_pair >= 0 ? single_pair % D : 0, lks = 0;
  int64_t issued = 0;
  // panel base (bytes, uniform) of the step at the load cursor: A_la or B_lb
  auto panel_base = [&]() -> const char * {
    return op_w == 0
               ? reinterpret_cast<const char *>(Apk + (((int64_t)la * mbp + tm * kTileBlocks) * kbp +
                                                       (int64_t)lks * kKStepBlocks) * 256)
               : reinterpret_cast<const char *>(Bpk + (((int64_t)lb * nbp + tn * kTileBlocks) * kbp +
                                                       (int64_t)lks * kKStepBlocks) * 256);
  };
  auto advance = [&]() {
    ++issued;
    if (++lks == nks) {
      lks = 0;
      if (single_pair < 0 && ++lb >= lim(la)) {
        ++la;
        lb = 0;
      }
    }
  };

  acc_t acc[BJ][BI];
  T sum[BJ][BI][4][C + 1];
#pragma unroll
  for (int y = 0; y < BJ; ++y)
#pragma unroll
    for (int x = 0; x < BI; ++x) {
      acc[y][x] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q <= C; ++q) sum[y][x][r][q] = T(0);
    }

  wait_vm<0>();  // nothing older than this tile's loads stays in flight
#pragma unroll
  for (int s0 = 0; s0 < kStages - 1; ++s0)
    if (issued < total) {
      const char *src = panel_base();
      T *dst = lds + (issued % kStages) * stage_elems<T>();
#pragma unroll
      for (int j = 0; j < kL; ++j) load_lds16(src + goff(j) + g0, dst + l0 + loff(j));
      advance();
    }

  // matrix-core instructions per wavefront per step.  The loads of the step
  // kStages - 1 ahead are issued either spread, one after every kEvery of them
  // (binary64 with 4 wavefronts of 32 x 32, where each wavefront issues many
  // loads and a burst would stall its matrix cores), or all at once at the
  // step's first instruction (the other layouts and binary32, where a wavefront
  // issues few loads and grouping them measured faster with less L2 traffic)
  constexpr int kMma = kKStepBlocks * 4 * BI * BJ;
  static_assert(kMma % kL == 0, "one load per fixed number of matrix-core instructions");
  constexpr int kEvery = kMma / kL;
  constexpr bool kSpread = sizeof(T) == 8 && LAYOUT == 1;

  // A wavefront whose blocks are all padding (rows from m or columns from n
  // on) has no matrix-core work and nothing to store: it only moves its share
  // of the panels, at the places and about the pace (one 64-cycle sleep per
  // instruction slot where loads are spread) of the others, and passes the same
  // barriers.
  if (__builtin_amdgcn_readfirstlane(tm * 64 + wm * BI * 16 >= m || tn * 64 + wn * BJ * 16 >= n ? 1 : 0)) {
    for (int64_t step = 0; step < total; ++step) {
      wait_step<kStages, kL>(total - 1 - step);
      __builtin_amdgcn_s_barrier();
      const bool more = issued < total;
      const char *nsrc = more ? panel_base() : reinterpret_cast<const char *>(Apk);
      T *ndst = lds + (issued % kStages) * stage_elems<T>();
      if constexpr (kSpread) {
#pragma unroll
        for (int mma = 0; mma < kMma; ++mma) {
          if (mma % kEvery == 0 && more) load_lds16(nsrc + goff(mma / kEvery) + g0, ndst + l0 + loff(mma / kEvery));
          __builtin_amdgcn_s_sleep(1);
          __builtin_amdgcn_sched_barrier(0);
        }
      } else if (more) {
#pragma unroll
        for (int j = 0; j < kL; ++j) load_lds16(nsrc + goff(j) + g0, ndst + l0 + loff(j));
      }
      if (more) advance();
    }
    __builtin_amdgcn_s_barrier();
    return;
  }

  int cks = 0;  // k step of the pair being computed
  for (int64_t step = 0; step < total; ++step) {
    wait_step<kStages, kL>(total - 1 - step);
    __builtin_amdgcn_s_barrier();
    // the step kStages - 1 ahead goes into the slot computed in the previous step
    const bool more = issued < total;
    const char *nsrc = more ? panel_base() : reinterpret_cast<const char *>(Apk);
    T *ndst = lds + (issued % kStages) * stage_elems<T>();

    const T *stage = lds + (step % kStages) * stage_elems<T>();
    // raised wave priority while this wave issues its matrix-core work, so the
    // sequencer favours waves that can feed the matrix cores over those about to
    // wait at the barrier (TS 108 -> 100 ms, DD 41.6 -> 41.0 ms at n = 4096)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int kb = 0; kb < kKStepBlocks; ++kb) {
      // binary64 fragments arrive in two halves (k substeps q = 0,1 and 2,3),
      // each loaded just before its matrix-core instructions; binary32 in one
      constexpr int kH = sizeof(T) == 8 ? 2 : 1, kQ = 4 / kH;
#pragma unroll
      for (int h = 0; h < kH; ++h) {
        T fa[BI][kQ], fb[BJ][kQ];
#pragma unroll
        for (int x = 0; x < BI; ++x) {
          const T *pa = stage + ((wm * BI + x) * kKStepBlocks + kb) * 256;
          if constexpr (sizeof(T) == 8) {
            const d2 va = *reinterpret_cast<const d2 *>(pa + h * 128 + 2 * lane);
            fa[x][0] = va[0];
            fa[x][1] = va[1];
          } else {
            const f4 va = *reinterpret_cast<const f4 *>(pa + 4 * lane);
#pragma unroll
            for (int q = 0; q < 4; ++q) fa[x][q] = va[q];
          }
        }
#pragma unroll
        for (int y = 0; y < BJ; ++y) {
          const T *pb = stage + kPanelElems + ((wn * BJ + y) * kKStepBlocks + kb) * 256;
          if constexpr (sizeof(T) == 8) {
            const d2 vb = *reinterpret_cast<const d2 *>(pb + h * 128 + 2 * lane);
            fb[y][0] = vb[0];
            fb[y][1] = vb[1];
          } else {
            const f4 vb = *reinterpret_cast<const f4 *>(pb + 4 * lane);
#pragma unroll
            for (int q = 0; q < 4; ++q) fb[y][q] = vb[q];
          }
        }
#pragma unroll
        for (int qq = 0; qq < kQ; ++qq)
#pragma unroll
          for (int y = 0; y < BJ; ++y)
#pragma unroll
            for (int x = 0; x < BI; ++x) {
              const int mma = ((kb * 4 + h * kQ + qq) * BJ + y) * BI + x;
              if constexpr (kSpread) {
                if (mma % kEvery == 0 && more)
                  load_lds16(nsrc + goff(mma / kEvery) + g0, ndst + l0 + loff(mma / kEvery));
              } else if (mma == 0 && more) {
#pragma unroll
                for (int j = 0; j < kL; ++j) load_lds16(nsrc + goff(j) + g0, ndst + l0 + loff(j));
              }
              acc[y][x] = M::run(fb[y][qq], fa[x][qq], acc[y][x]);
              __builtin_amdgcn_sched_barrier(0);  // keep the loads where they were placed
            }
      }
    }
    __builtin_amdgcn_s_setprio(0);
    if (more) advance();

    if (++cks == nks) {  // the pair's product is complete and exact: fold it in
      cks = 0;
#pragma unroll
      for (int y = 0; y < BJ; ++y)
#pragma unroll
        for (int x = 0; x < BI; ++x) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc_add<T, C + 1>(sum[y][x][r], acc[y][x][r]);
          acc[y][x] = acc_t{0, 0, 0, 0};
        }
    }
  }
  __builtin_amdgcn_s_barrier();  // every wavefront is done with the ring

  // store: element (i, j) with i along the lanes (contiguous in column-major C)
#pragma unroll
  for (int y = 0; y < BJ; ++y)
#pragma unroll
    for (int x = 0; x < BI; ++x)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = tm * 64 + (wm * BI + x) * 16 + lane % 16;
        const int j = tn * 64 + (wn * BJ + y) * 16 + M::out_row(lane, r);
        if (i >= m || j >= n) continue;
        if (single_pair >= 0) {
          Cdbg[i + (int64_t)j * lddbg] = (double)sum[y][x][r][0];
        } else {
          T v[C + 1];
#pragma unroll
          for (int q = 0; q <= C; ++q) v[q] = sum[y][x][r][q];
          renorm<T, C + 1>(v);
#pragma unroll
          for (int q = 0; q < C; ++q) Cout[q * c_stride + i + (int64_t)j * ldc] = v[q];
        }
      }
}

template <typename T, int C, int LAYOUT>
__global__ __launch_bounds__(64 * Layout<LAYOUT>::WM * Layout<LAYOUT>::WN, waves_of(LAYOUT, C, (int)sizeof(T))) void k_gemm_plain(
    const T *__restrict__ Apk, const T *__restrict__ Bpk, int64_t mbp, int64_t nbp, int64_t kbp, int m, int n, int D,
    T *__restrict__ Cout, int ldc, int64_t c_stride, int single_pair, double *__restrict__ Cdbg, int lddbg) {
  __shared__ __attribute__((aligned(16))) T lds[stages_of<T>()][stage_elems<T>()];
  int tm, tn;
  tile_coords(blockIdx.x, gridDim.x, (int)(mbp / kTileBlocks), (int)(nbp / kTileBlocks), tm, tn);
  gemm_plain_tile<T, C, LAYOUT>(Apk, Bpk, mbp, nbp, kbp, m, n, D, Cout, ldc, c_stride, single_pair, Cdbg, lddbg, tm,
                                tn, &lds[0][0]);
}

// The same with the pairs of each tile chosen from the data: tile (tm, tn)
// takes pairs (a, b) with b < lims[(tn * tiles_m + tm) * D + a] (a staircase
// written by launch_tile_pairs).
template <typename T, int C, int LAYOUT>
__global__ __launch_bounds__(64 * Layout<LAYOUT>::WM * Layout<LAYOUT>::WN, waves_of(LAYOUT, C, (int)sizeof(T))) void k_gemm_plain_pruned(
    const T *__restrict__ Apk, const T *__restrict__ Bpk, int64_t mbp, int64_t nbp, int64_t kbp, int m, int n, int D,
    T *__restrict__ Cout, int ldc, int64_t c_stride, const int8_t *__restrict__ lims) {
  __shared__ __attribute__((aligned(16))) T lds[stages_of<T>()][stage_elems<T>()];
  int tm, tn;
  const int tiles_m = (int)(mbp / kTileBlocks);
  tile_coords(blockIdx.x, gridDim.x, tiles_m, (int)(nbp / kTileBlocks), tm, tn);
  // the tile's D counts (uniform), packed a byte each
  const int8_t *src = lims + ((int64_t)tn * tiles_m + tm) * D;
  uint64_t lo = 0, hi = 0;
  for (int a = 0; a < D; ++a) {
    const uint64_t v = (uint64_t)(uint8_t)src[a];
    if (a < 8)
      lo |= v << (8 * a);
    else
      hi |= v << (8 * (a - 8));
  }
  lo = ((uint64_t)__builtin_amdgcn_readfirstlane((int)(lo >> 32)) << 32) |
       (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)lo);
  hi = ((uint64_t)__builtin_amdgcn_readfirstlane((int)(hi >> 32)) << 32) |
       (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)hi);
  gemm_plain_tile<T, C, LAYOUT, true>(Apk, Bpk, mbp, nbp, kbp, m, n, D, Cout, ldc, c_stride, -1, nullptr, 0, tm, tn,
                                      &lds[0][0], Staircase{lo, hi});
}

// Persistent batched kernel: each workgroup takes (product, tile) work items
// from a shared counter until the list is exhausted (items are ordered by
// decreasing work, so the long tiles start first).
template <typename T, int C, int LAYOUT>
__global__ __launch_bounds__(64 * Layout<LAYOUT>::WM * Layout<LAYOUT>::WN, waves_of(LAYOUT, C, (int)sizeof(T))) void k_gemm_plain_batched(
    const PlainGemmDesc *__restrict__ descs, const int2 *__restrict__ items, const int *__restrict__ bounds,
    int *__restrict__ counters) {
  __shared__ __attribute__((aligned(16))) T lds[stages_of<T>()][stage_elems<T>()];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = take_item(counters, bounds, blockIdx.x);
    __syncthreads();
    const int it = next;
    __syncthreads();
    if (it < 0) break;
    const int2 w = items[it];
    const PlainGemmDesc &d = descs[w.x];
    const int tiles_m = (int)(d.mbp / kTileBlocks);
    gemm_plain_tile<T, C, LAYOUT>(static_cast<const T *>(d.Apk), static_cast<const T *>(d.Bpk), d.mbp, d.nbp, d.kbp,
                                  d.m, d.n, d.D, static_cast<T *>(d.C), d.ldc, d.c_stride, -1, (double *)nullptr,
                                  0, w.y % tiles_m, w.y / tiles_m, &lds[0][0]);
  }
}

constexpr int threads_of(int layout) { return layout == 1 ? 256 : layout == 2 ? 512 : 1024; }

}  // namespace

template <typename T, int C>
hipError_t launch_gemm_plain(const void *Apk, const void *Bpk, int64_t mbp, int64_t nbp, int64_t kbp, int m, int n,
                             int D, T *Cout, int ldc, int64_t c_stride, int single_pair, double *Cdbg, int lddbg,
                             int layout, hipStream_t st) {
  const int64_t tiles = (mbp / kTileBlocks) * (nbp / kTileBlocks);
  if (tiles <= 0) return hipSuccess;
  const T *a = static_cast<const T *>(Apk);
  const T *b = static_cast<const T *>(Bpk);
  switch (layout) {
    case 2:
      hipLaunchKernelGGL((k_gemm_plain<T, C, 2>), dim3((unsigned)tiles), dim3(threads_of(2)), 0, st, a, b, mbp, nbp,
                         kbp, m, n, D, Cout, ldc, c_stride, single_pair, Cdbg, lddbg);
      break;
    case 3:
      hipLaunchKernelGGL((k_gemm_plain<T, C, 3>), dim3((unsigned)tiles), dim3(threads_of(3)), 0, st, a, b, mbp, nbp,
                         kbp, m, n, D, Cout, ldc, c_stride, single_pair, Cdbg, lddbg);
      break;
    default:
      hipLaunchKernelGGL((k_gemm_plain<T, C, 1>), dim3((unsigned)tiles), dim3(threads_of(1)), 0, st, a, b, mbp, nbp,
                         kbp, m, n, D, Cout, ldc, c_stride, single_pair, Cdbg, lddbg);
  }
  return hipGetLastError();
}

template <typename T, int C>
hipError_t launch_gemm_plain_pruned(const void *Apk, const void *Bpk, int64_t mbp, int64_t nbp, int64_t kbp, int m,
                                    int n, int D, T *Cout, int ldc, int64_t c_stride, const int8_t *lims, int layout,
                                    hipStream_t st) {
  const int64_t tiles = (mbp / kTileBlocks) * (nbp / kTileBlocks);
  if (tiles <= 0) return hipSuccess;
  if (D < 1 || D > kMaxPairLim) return hipErrorInvalidValue;
  const T *a = static_cast<const T *>(Apk);
  const T *b = static_cast<const T *>(Bpk);
  switch (layout) {
    case 2:
      hipLaunchKernelGGL((k_gemm_plain_pruned<T, C, 2>), dim3((unsigned)tiles), dim3(threads_of(2)), 0, st, a, b, mbp,
                         nbp, kbp, m, n, D, Cout, ldc, c_stride, lims);
      break;
    case 3:
      hipLaunchKernelGGL((k_gemm_plain_pruned<T, C, 3>), dim3((unsigned)tiles), dim3(threads_of(3)), 0, st, a, b, mbp,
                         nbp, kbp, m, n, D, Cout, ldc, c_stride, lims);
      break;
    default:
      hipLaunchKernelGGL((k_gemm_plain_pruned<T, C, 1>), dim3((unsigned)tiles), dim3(threads_of(1)), 0, st, a, b, mbp,
                         nbp, kbp, m, n, D, Cout, ldc, c_stride, lims);
  }
  return hipGetLastError();
}

template <typename T, int C>
hipError_t launch_gemm_plain_batched(const PlainGemmDesc *descs, const int2 *items, const int *bounds,
                                     int *counters, int grid, int layout, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  switch (layout) {
    case 2:
      hipLaunchKernelGGL((k_gemm_plain_batched<T, C, 2>), dim3((unsigned)grid), dim3(threads_of(2)), 0, st, descs,
                         items, bounds, counters);
      break;
    case 3:
      hipLaunchKernelGGL((k_gemm_plain_batched<T, C, 3>), dim3((unsigned)grid), dim3(threads_of(3)), 0, st, descs,
                         items, bounds, counters);
      break;
    default:
      hipLaunchKernelGGL((k_gemm_plain_batched<T, C, 1>), dim3((unsigned)grid), dim3(threads_of(1)), 0, st, descs,
                         items, bounds, counters);
  }
  return hipGetLastError();
}

#define MP_GEMM_INST(T, C)                                                                                            \
  template hipError_t launch_gemm_plain<T, C>(const void *, const void *, int64_t, int64_t, int64_t, int, int, int, \
                                              T *, int, int64_t, int, double *, int, int, hipStream_t);              \
  template hipError_t launch_gemm_plain_batched<T, C>(const PlainGemmDesc *, const int2 *, const int *, int *, int, \
                                                      int, hipStream_t);                                            \
  template hipError_t launch_gemm_plain_pruned<T, C>(const void *, const void *, int64_t, int64_t, int64_t, int, int, \
                                                     int, T *, int, int64_t, const int8_t *, int, hipStream_t);
MP_GEMM_INST(double, 2)
MP_GEMM_INST(double, 3)
MP_GEMM_INST(double, 4)
MP_GEMM_INST(float, 3)
#undef MP_GEMM_INST

}  // namespace mp
