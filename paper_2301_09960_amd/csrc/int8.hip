// INT8-slice form (the precision form; not in the paper): digit slices on the
// INT8 matrix cores with exact 32-bit integer sums.
//
// With digit units u_s = 2^(E - 6 - 7 (s - 1)) (split.hip), every product
// A_s B_t on the anti-diagonal s + t = g + 1 has the same unit
// 2^(E_i + F_j + 2 - 7 (g + 1)), so the D (D + 1) / 2 slice products collapse
// into D exact integer diagonal sums S_g = sum_{s + t = g + 1} A_s B_t, each a
// GEMM with the k loops of its g pairs concatenated.  |digit| <= 64, so a
// 32-bit sum of up to 2^31 / 4096 digit products is exact; k is cut into
// chunks short enough for that bound, each chunk writing its own partial S_g.
//
// k_gemm_int8: one workgroup per tile of C (128 x 128 or 256 x 256), k chunk
// and group of diagonals (the diagonal sums are independent, so a small
// product spreads its diagonals over the grid); each wavefront owns a grid of
// 32 x 32 blocks of v_mfma_i32_32x32x32_i8.  Panels of A_s and B_t (64 or 128
// k per step) move global -> LDS by direct loads into a ring of 2 to 4
// stages, as in the floating-point kernel.  After the last pair of a diagonal
// the 32-bit tile is written to the S_g plane in a blocked layout (16-byte
// stores per lane).  k_gemm_int8_batched runs the same tiles as items of a
// persistent launch over many products.
//
// k_int8_combine: per element, C = sum_g S_g 2^(E_i + F_j + 2 - 7 (g + 1)):
// runs of consecutive diagonals summed exactly in 64-bit integers, each run
// split exactly into two binary64 values, added with TwoSum into a (c+1)-term
// accumulator and renormalized into the c components of C (it reads D 32-bit
// sums per element per chunk and writes C once).
#include <algorithm>

#include "internal.h"
#include "layout.h"
#include "mp_device.h"

namespace mp {
namespace {

constexpr int kGroupM = 8;

typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

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

__device__ __forceinline__ void load_lds16(const void *src, void *lds_dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds_dst, 16, 0, 0);
}
template <int N>
__device__ __forceinline__ void wait_vm() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Waits until this wavefront's loads of the step about to be computed have
// landed: with an NS-stage ring, min(NS - 2, later) later steps (kL loads
// each) may stay in flight.
template <int NS, int kL>
__device__ __forceinline__ void wait_step(int64_t later) {
  static_assert(NS >= 2 && NS <= 4, "wait chain covers rings of 2 to 4 stages");
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

// Tile configurations (in 32 x 32 blocks): TB x TB tile of C, WM x WN
// wavefronts, KSB 32-wide k blocks per pipeline step, NS LDS stages.
//   config 1: 128 x 128 tile, 4 wavefronts of 64 x 64 (small products), k
//             steps of 128 in a 2-stage ring (two workgroups per CU), each
//             step's loads over its first half
//   config 2: 256 x 256 tile, 4 wavefronts of 128 x 128 (accumulators in AGPRs;
//             LDS traffic per instruction halved)
//   config 4: 256 x 256 tile, 16 wavefronts of 64 x 64 (more wavefronts to
//             hide latency, more LDS reads per instruction), k steps of 128
//   config 3: 256 x 256 tile, 8 wavefronts of 128 x 64, k steps of 128 in a
//             2-stage ring (half the barriers of 64-wide steps, and 64 KiB
//             requested per step)
// KSB is 1 or 2 times kKStepBlocks8, the k padding unit of the INT8 slices (64
// k): with 4-block steps a pair's last step in a k chunk may hold 2 blocks.
template <int CFG> struct Int8Cfg;
template <> struct Int8Cfg<1> { static constexpr int TB = 4, WM = 2, WN = 2, KSB = 4, NS = 2, SPACING = 1; };
template <> struct Int8Cfg<2> { static constexpr int TB = 8, WM = 2, WN = 2, KSB = 2, NS = 4, SPACING = 0; };
template <> struct Int8Cfg<3> { static constexpr int TB = 8, WM = 2, WN = 4, KSB = 4, NS = 2, SPACING = 3; };
template <> struct Int8Cfg<4> { static constexpr int TB = 8, WM = 4, WN = 4, KSB = 4, NS = 2, SPACING = 0; };

// Matrix-core instructions between two loads of the next step: spread over the
// whole step by default, fewer where a configuration issues its loads earlier.
template <typename G>
constexpr int load_spacing(int even) {
  return G::SPACING > 0 ? G::SPACING : even;
}

template <int CFG>
constexpr int int8_stage_bytes() {
  return 2 * Int8Cfg<CFG>::TB * Int8Cfg<CFG>::KSB * 1024;  // A panel, then B panel
}

// Diagonal sums S_g of one tile (tm, tn) and k chunk, as in the file comment:
// operand panels (TB blocks x KSB k blocks of A_s and of B_t) move
// global -> LDS by direct loads into a ring of NS stages, NS - 1 steps ahead;
// each step waits for its own loads and passes one barrier.
//
// Each wavefront moves kL 1 KiB pieces of one operand per step.  Their global
// offsets from the step's panel base and their LDS offsets are fixed for the
// whole tile, so a load costs one 64-bit add; and the loads of the next step
// are spread between this step's matrix-core instructions (one per kEvery),
// which keeps the matrix cores fed where a burst of LDS-direct loads would
// stall them.  The 256 x 256 configuration with its 2-stage ring issues them
// over the first three quarters of the step (one per 3 instructions instead of
// one per 4), so that the last ones land before the step ends.
template <int CFG>
__device__ __forceinline__ void gemm_int8_tile(const int8_t *__restrict__ Apk, const int8_t *__restrict__ Bpk,
                                               int64_t mbp, int64_t nbp, int64_t kbp, int64_t kb0, int nks, int last,
                                               int D, int m, int n, int32_t *__restrict__ S, int64_t plane, int chunk,
                                               int nchunks, int tm, int tn, int g0, int g1, int8_t *lds) {
  using G = Int8Cfg<CFG>;
  constexpr int TB = G::TB, WM = G::WM, WN = G::WN, KSB = G::KSB, NS = G::NS;
  constexpr int BI = TB / WM, BJ = TB / WN;
  constexpr int NW = WM * WN;
  constexpr int kPanel = TB * KSB * 1024;
  constexpr int kInst = 2 * TB * KSB;  // 1 KiB wavefront instructions per step
  constexpr int kL = kInst / NW;
  constexpr int kMma = KSB * BI * BJ;  // matrix-core instructions per wavefront per step
  constexpr int kEvery = load_spacing<G>(kMma / kL);
  static_assert(kInst % NW == 0, "staging split");
  static_assert((TB * KSB) % kL == 0, "a wavefront's loads of a step come from one operand");
  static_assert(kMma % kL == 0, "one load per fixed number of matrix-core instructions");
  static_assert(kEvery * kL <= kMma, "every load of the next step is issued within this step");
  // a pair's k blocks in the chunk are a multiple of kKStepBlocks8: its steps
  // are full but the last, which holds `last` blocks (KSB / 2 or KSB)
  static_assert(KSB % kKStepBlocks8 == 0 && KSB <= 2 * kKStepBlocks8, "k steps and the k padding unit");

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
  // diagonals g0 .. g1 - 1 (g pairs each)
  const int64_t total = ((int64_t)(g1 - 1) * g1 / 2 - (int64_t)(g0 - 1) * g0 / 2) * nks;

  // this wavefront's share of a step: operand op_w, pieces j = 0..kL-1
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  const int op_w = (wave_u * kL) / (TB * KSB);
  uint32_t goff[kL];  // byte offset from the step's panel base (per lane; k <= 2^20 keeps it below 2^32)
  int loff[kL];       // byte offset in the stage (uniform)
  uint32_t beyond[kL];  // in a pair's short last step the piece lies past the pair's k: load piece kb - KSB / 2
#pragma unroll
  for (int j = 0; j < kL; ++j) {
    const int r = (wave_u * kL + j) % (TB * KSB);
    const int blk = r / KSB, kb = r % KSB;
    goff[j] = (uint32_t)(((int64_t)blk * kbp + kb) * 1024) + 16u * (uint32_t)lane;
    loff[j] = op_w * kPanel + (blk * KSB + kb) * 1024;
    beyond[j] = kb >= KSB / 2 ? (uint32_t)(KSB / 2) * 1024u : 0u;
  }
  // every step loads kL pieces (the wait counts assume it): a pair's short
  // last step re-loads pieces of its own range into stage slots that no
  // matrix-core instruction reads
  auto piece = [&](int j, int ks) -> uint32_t { return goff[j] - (ks == nks - 1 && last < KSB ? beyond[j] : 0u); };

  int lg = g0, ls = 1, lks = 0;  // load cursor: diagonal, pair within it, k step
  int64_t issued = 0;
  // panel base of the step at the load cursor (A_ls or B_(lg+1-ls)), and its ring slot
  auto panel_base = [&]() -> const int8_t * {
    return op_w == 0 ? Apk + (((int64_t)(ls - 1) * mbp + (int64_t)tm * TB) * kbp + kb0 + (int64_t)lks * KSB) * 1024
                     : Bpk + (((int64_t)(lg - ls) * nbp + (int64_t)tn * TB) * kbp + kb0 + (int64_t)lks * KSB) * 1024;
  };
  auto advance = [&]() {
    ++issued;
    if (++lks == nks) {
      lks = 0;
      if (++ls > lg) {
        ++lg;
        ls = 1;
      }
    }
  };

  i16v acc[BJ][BI];
#pragma unroll
  for (int y = 0; y < BJ; ++y)
#pragma unroll
    for (int x = 0; x < BI; ++x)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[y][x][r] = 0;

  wait_vm<0>();
#pragma unroll
  for (int s0 = 0; s0 < NS - 1; ++s0)
    if (issued < total) {
      const int8_t *src = panel_base();
      int8_t *dst = lds + (issued % NS) * int8_stage_bytes<CFG>();
#pragma unroll
      for (int j = 0; j < kL; ++j) load_lds16(src + piece(j, lks), dst + loff[j]);
      advance();
    }

  // A wavefront whose blocks are all padding (rows from m or columns from n
  // on) has no matrix-core work: it only moves its share of the panels, at the
  // places and about the pace (64 cycles per two instructions) of the others,
  // and passes the same barriers.  It leaves its blocks of the S_g planes
  // unwritten; the combine reads no element outside m x n.
  if (__builtin_amdgcn_readfirstlane(((int64_t)tm * TB + wm * BI) * 32 >= m || ((int64_t)tn * TB + wn * BJ) * 32 >= n
                                         ? 1
                                         : 0)) {
    for (int64_t step = 0; step < total; ++step) {
      wait_step<NS, kL>(total - 1 - step);
      __builtin_amdgcn_s_barrier();
      const bool more = issued < total;
      const int8_t *nsrc = more ? panel_base() : Apk;
      int8_t *ndst = lds + (issued % NS) * int8_stage_bytes<CFG>();
      const uint32_t next_short = lks == nks - 1 && last < KSB ? 1u : 0u;
#pragma unroll
      for (int mma = 0; mma < kMma; ++mma) {
        if (mma % kEvery == 0 && mma / kEvery < kL && more)
          load_lds16(nsrc + (goff[mma / kEvery] - next_short * beyond[mma / kEvery]), ndst + loff[mma / kEvery]);
        if (mma % 2 == 1) __builtin_amdgcn_s_sleep(1);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (more) advance();
    }
    __builtin_amdgcn_s_barrier();
    return;
  }

  int cg = g0, cs = 1, cks = 0;  // compute cursor
  for (int64_t step = 0; step < total; ++step) {
    wait_step<NS, kL>(total - 1 - step);
    __builtin_amdgcn_s_barrier();
    // the step NS - 1 ahead goes into the slot computed in the previous step
    const bool more = issued < total;
    const int8_t *nsrc = more ? panel_base() : Apk;
    int8_t *ndst = lds + (issued % NS) * int8_stage_bytes<CFG>();

    const int8_t *stage = lds + (step % NS) * int8_stage_bytes<CFG>();
    // a pair's short last step holds the first KSB / 2 k blocks (the only
    // short length): its second half is skipped, on a uniform branch
    const bool short_step = cks == nks - 1 && last < KSB;
    const uint32_t next_short = lks == nks - 1 && last < KSB ? 1u : 0u;  // the step being loaded is short
#pragma unroll
    for (int kb = 0; kb < KSB; ++kb) {
      const bool run = kb < KSB / 2 || !short_step;
      i4v fa[BI], fb[BJ];
      if (run) {
#pragma unroll
        for (int x = 0; x < BI; ++x)
          fa[x] = *reinterpret_cast<const i4v *>(stage + ((wm * BI + x) * KSB + kb) * 1024 + 16 * lane);
#pragma unroll
        for (int y = 0; y < BJ; ++y)
          fb[y] = *reinterpret_cast<const i4v *>(stage + kPanel + ((wn * BJ + y) * KSB + kb) * 1024 + 16 * lane);
      }
#pragma unroll
      for (int y = 0; y < BJ; ++y)
#pragma unroll
        for (int x = 0; x < BI; ++x) {
          const int mma = (kb * BJ + y) * BI + x;
          if (mma % kEvery == 0 && mma / kEvery < kL && more)
            load_lds16(nsrc + (goff[mma / kEvery] - next_short * beyond[mma / kEvery]), ndst + loff[mma / kEvery]);
          if (run) acc[y][x] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fb[y], fa[x], acc[y][x], 0, 0, 0);
          __builtin_amdgcn_sched_barrier(0);  // keep the loads where they were placed
        }
    }
    if (more) advance();
    if (++cks == nks) {
      cks = 0;
      if (++cs > cg) {  // diagonal cg complete: write its exact partial sum (blocked layout)
        int32_t *out = S + ((int64_t)(cg - 1) * nchunks + chunk) * plane;
#pragma unroll
        for (int y = 0; y < BJ; ++y)
#pragma unroll
          for (int x = 0; x < BI; ++x) {
            const int64_t bi = (int64_t)tm * TB + wm * BI + x, bj = (int64_t)tn * TB + wn * BJ + y;
            i4v *dst = reinterpret_cast<i4v *>(out + ((bj * mbp + bi) * 64 + lane) * 16);
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[v] = i4v{acc[y][x][4 * v], acc[y][x][4 * v + 1], acc[y][x][4 * v + 2],
                                                     acc[y][x][4 * v + 3]};
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[y][x][r] = 0;
          }
        ++cg;
        cs = 1;
      }
    }
  }
  __builtin_amdgcn_s_barrier();
}

// Diagonals [g0, g1) of group z of `groups`: the D (D + 1) / 2 pairs cut into
// nearly equal parts at diagonal boundaries (a group may be empty).
__device__ __forceinline__ void diagonal_group(int D, int z, int groups, int &g0, int &g1) {
  g0 = 1;
  g1 = D + 1;
  if (groups <= 1) return;
  const int64_t pairs = (int64_t)D * (D + 1) / 2;
  auto first_reaching = [&](int64_t target) {  // smallest g with g (g + 1) / 2 >= target
    int g = 0;
    while ((int64_t)g * (g + 1) / 2 < target) ++g;
    return g;
  };
  g0 = first_reaching(pairs * z / groups) + 1;
  g1 = first_reaching(pairs * (z + 1) / groups) + 1;
}

template <int CFG>
__global__ __launch_bounds__(64 * Int8Cfg<CFG>::WM * Int8Cfg<CFG>::WN, 1) void k_gemm_int8(
    const int8_t *__restrict__ Apk, const int8_t *__restrict__ Bpk, int64_t mbp, int64_t nbp, int64_t kbp,
    int kb_chunk, int D, int m, int n, int32_t *__restrict__ S, int64_t plane) {
  __shared__ __attribute__((aligned(16))) int8_t lds[Int8Cfg<CFG>::NS * int8_stage_bytes<CFG>()];
  constexpr int TB = Int8Cfg<CFG>::TB;
  int tm, tn;
  tile_coords(blockIdx.x, gridDim.x, (int)(mbp / TB), (int)(nbp / TB), tm, tn);
  const int chunk = blockIdx.y, nchunks = gridDim.y;
  const int64_t kb0 = (int64_t)chunk * kb_chunk;
  const int64_t kb1 = kb0 + kb_chunk < kbp ? kb0 + kb_chunk : kbp;
  constexpr int KSB = Int8Cfg<CFG>::KSB;
  const int nks = (int)ceil_div(kb1 - kb0, KSB), last = (int)(kb1 - kb0) - (nks - 1) * KSB;
  // diagonal group blockIdx.z of gridDim.z
  int g0, g1;
  diagonal_group(D, blockIdx.z, gridDim.z, g0, g1);
  gemm_int8_tile<CFG>(Apk, Bpk, mbp, nbp, kbp, kb0, nks, last, D, m, n, S, plane, chunk, nchunks, tm, tn, g0, g1,
                      lds);
}

// Diagonal-sum planes are blocked: the 32 x 32 block (bi, bj) of C holds, for
// lane l and accumulator r of the 32x32x32 instruction, element
// (32 bi + l % 32, 32 bj + 8 (r / 4) + 4 (l / 32) + r % 4) at
// ((bj * mbp + bi) * 64 + l) * 16 + r.  A combine thread takes four
// consecutive r of one (block, lane): one 16-byte load per diagonal and chunk.
//
// Consecutive diagonals differ in weight by 2^7, so a run of L of them is
// summed exactly in a 64-bit integer, T = sum_j S_(g0 + j) 2^(7 (L - 1 - j)),
// at the weight of its last diagonal, and enters the accumulator as the two
// binary64 values hi = RN(T) and lo = T - hi (exact: |lo| < 2^9 while
// |T| < 2^62).  With digits of at most 64 in magnitude, |S_g| <= g K 2^12 <=
// D K 2^12 (K the padded k); for 2^B >= D K 2^12, |T| < 2^(B + 7 (L - 1) + 1),
// so L = 1 + (61 - B) / 7 keeps |T| below 2^62 (L = 5 for QD at k = 4096).
// Two accumulator additions per run instead of one per diagonal: the combine
// is bound by its binary64 additions, not by its loads.
__host__ __device__ inline int combine_run(int D, int64_t kbp) {
  int64_t x = (int64_t)(D > 0 ? D : 1) * (kbp > 0 ? kbp : 1) * kKBlk8;  // D K
  int b = 12;
  while (x > 1) {  // b = 12 + ceil(log2(D K))
    x = (x + 1) / 2;
    ++b;
  }
  return b <= 61 ? 1 + (61 - b) / 7 : 1;
}

// Combine thread t (0 <= t < mbp * nbp * 256) of one product: four
// consecutive accumulator entries r of one (block, lane).
template <int C>
__device__ __forceinline__ void combine_one(int64_t t, const int32_t *__restrict__ S, int64_t plane, int nchunks,
                                            int D, int run, const int *__restrict__ EA, const int *__restrict__ EB,
                                            int64_t mbp, int m, int n, double *__restrict__ Cout, int ldc,
                                            int64_t c_stride, int debug_g, int64_t *__restrict__ Sdbg, int lddbg) {
  const int q = (int)(t % 4);
  const int lane = (int)((t / 4) % 64);
  const int64_t blk = t / 256;
  const int64_t bi = blk % mbp, bj = blk / mbp;
  const int i = (int)(bi * 32 + lane % 32);
  const int j0 = (int)(bj * 32 + 8 * q + 4 * (lane / 32));
  if (i >= m || j0 >= n) return;
  const int64_t off = (blk * 64 + lane) * 16 + 4 * q;
  const int Ei = EA[i];
  double acc[4][C + 1];
  int Fj[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    Fj[e] = j0 + e < n ? EB[j0 + e] : kZeroExp;
#pragma unroll
    for (int c = 0; c <= C; ++c) acc[e][c] = 0.0;
  }
  for (int g0 = 1; g0 <= D; g0 += run) {
    const int g1 = g0 + run <= D + 1 ? g0 + run : D + 1;  // diagonals g0 .. g1 - 1
    int64_t T[4] = {0, 0, 0, 0};
    for (int g = g0; g < g1; ++g) {
      int64_t s[4] = {0, 0, 0, 0};
      for (int c = 0; c < nchunks; ++c) {
        const i4v v = *reinterpret_cast<const i4v *>(S + ((int64_t)(g - 1) * nchunks + c) * plane + off);
#pragma unroll
        for (int e = 0; e < 4; ++e) s[e] += v[e];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (debug_g == g && j0 + e < n) Sdbg[i + (int64_t)(j0 + e) * lddbg] = s[e];
        T[e] = T[e] * 128 + s[e];
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (j0 + e >= n || Ei == kZeroExp || Fj[e] == kZeroExp || T[e] == 0) continue;
      const double hi = (double)T[e];
      const double lo = (double)(T[e] - (int64_t)hi);
      const int w = Ei + Fj[e] + 2 - 7 * g1;  // the weight of diagonal g1 - 1
      acc_add<double, C + 1>(acc[e], ldexp(hi, w));
      acc_add<double, C + 1>(acc[e], ldexp(lo, w));
    }
  }
  if (debug_g > 0) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (j0 + e >= n) continue;
    renorm<double, C + 1>(acc[e]);
#pragma unroll
    for (int c = 0; c < C; ++c) Cout[c * c_stride + i + (int64_t)(j0 + e) * ldc] = acc[e][c];
  }
}

template <int C>
__global__ __launch_bounds__(256) void k_int8_combine(const int32_t *__restrict__ S, int64_t plane, int nchunks, int D,
                                                      int run, const int *__restrict__ EA, const int *__restrict__ EB,
                                                      int64_t mbp, int64_t nbp, int m, int n,
                                                      double *__restrict__ Cout, int ldc, int64_t c_stride,
                                                      int debug_g, int64_t *__restrict__ Sdbg, int lddbg) {
  const int64_t total = mbp * nbp * 64 * 4;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x)
    combine_one<C>(t, S, plane, nchunks, D, run, EA, EB, mbp, m, n, Cout, ldc, c_stride, debug_g, Sdbg, lddbg);
}

// Persistent INT8 GEMM of a batch in tile configuration CFG: each workgroup
// takes (product, tile, k chunk, diagonal group) items from a shared counter;
// items are ordered by decreasing work.
template <int CFG>
__global__ __launch_bounds__(64 * Int8Cfg<CFG>::WM * Int8Cfg<CFG>::WN, 1) void k_gemm_int8_batched(
    const Int8GemmDesc *__restrict__ descs, const int4 *__restrict__ items, const int *__restrict__ bounds,
    int *__restrict__ counters) {
  __shared__ __attribute__((aligned(16))) int8_t lds[Int8Cfg<CFG>::NS * int8_stage_bytes<CFG>()];
  __shared__ int next;
  constexpr int TB = Int8Cfg<CFG>::TB;
  for (;;) {
    if (threadIdx.x == 0) next = take_item(counters, bounds, blockIdx.x);
    __syncthreads();
    const int it = next;
    __syncthreads();
    if (it < 0) break;
    const int4 w = items[it];
    const Int8GemmDesc &d = descs[w.x];
    const int tiles_m = (int)(d.mbp / TB);
    const int tm = w.y % tiles_m, tn = w.y / tiles_m;
    const int chunk = w.z;
    const int64_t kb0 = (int64_t)chunk * d.kbc;
    const int64_t kb1 = kb0 + d.kbc < d.kbp ? kb0 + d.kbc : d.kbp;
    constexpr int KSB = Int8Cfg<CFG>::KSB;
    const int nks = (int)ceil_div(kb1 - kb0, KSB), last = (int)(kb1 - kb0) - (nks - 1) * KSB;
    int g0, g1;
    diagonal_group(d.D, w.w, d.groups, g0, g1);
    gemm_int8_tile<CFG>(d.Apk, d.Bpk, d.mbp, d.nbp, d.kbp, kb0, nks, last, d.D, d.m, d.n, d.S, d.plane, chunk,
                        d.nchunks, tm, tn, g0, g1, lds);
  }
}

// Combine of a batch: workgroup b takes 32 x 32 block b - prefix[p] of product p.
template <int C>
__global__ __launch_bounds__(256) void k_int8_combine_batched(const Int8GemmDesc *__restrict__ descs,
                                                              const int *__restrict__ prefix, int nprod) {
  int lo = 0, hi = nprod - 1;  // last p with prefix[p] <= blockIdx.x
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (prefix[mid] <= (int)blockIdx.x)
      lo = mid;
    else
      hi = mid - 1;
  }
  const Int8GemmDesc &d = descs[lo];
  const int64_t t = ((int64_t)blockIdx.x - prefix[lo]) * 256 + threadIdx.x;
  combine_one<C>(t, d.S, d.plane, d.nchunks, d.D, combine_run(d.D, d.kbp), d.EA, d.EB, d.mbp, d.m, d.n, d.C, d.ldc,
                 d.c_stride, 0, nullptr, 0);
}

}  // namespace

// Longest k chunk (in 32-wide k blocks, a multiple of the k step) whose
// diagonal sums stay within 32 bits: D * k_chunk * 64 * 64 < 2^31.
int int8_kblocks_per_chunk(int D) {
  int64_t kc = ((int64_t(1) << 31) - 1) / (int64_t(4096) * (D > 0 ? D : 1));
  int64_t blocks = kc / (kKBlk8 * kKStepBlocks8) * kKStepBlocks8;
  return (int)(blocks > kKStepBlocks8 ? blocks : kKStepBlocks8);
}

// Tile configuration for an m x n product (cfg > 0 forces one): the 256 x 256
// tiles unless padding to them more than doubles the padded area of 128 x 128
// tiles.  Small grids are filled by spreading the diagonals over the grid, and
// the larger tile ran 1.6 to 2 times faster from n = 1024 up
// (DD and QD at n = 1024, 2048, 3072).
int int8_tile_config(int64_t m, int64_t n, int cfg) {
  if (cfg >= 1 && cfg <= 4) return cfg;
  const int64_t area3 = ceil_div(m, 256) * ceil_div(n, 256) * 4, area1 = ceil_div(m, 128) * ceil_div(n, 128);
  return area3 <= 2 * area1 ? 3 : 1;
}

template <int C>
hipError_t launch_gemm_int8(const void *Apk, const void *Bpk, const int *EA, const int *EB, int32_t *Sws, int64_t mbp,
                            int64_t nbp, int64_t kbp, int m, int n, int D, double *Cout, int ldc, int64_t c_stride,
                            int debug_g, int64_t *Sdbg, int lddbg, int cfg, hipStream_t st) {
  if (mbp <= 0 || nbp <= 0 || m <= 0 || n <= 0) return hipSuccess;
  const int kbc = int8_kblocks_per_chunk(D);
  const int nchunks = (int)ceil_div(kbp, kbc);
  const int64_t plane = mbp * nbp * 1024;  // blocked, padded diagonal-sum plane
  const auto *a = static_cast<const int8_t *>(Apk);
  const auto *b = static_cast<const int8_t *>(Bpk);
  const int use = int8_tile_config(m, n, cfg);
  const int tb = int8_tile_blocks(use);
  if (mbp % tb != 0 || nbp % tb != 0) return hipErrorInvalidValue;  // slices padded for another tile
  // small products: diagonals (independent sums, each with its own plane) spread
  // over gridDim.z so the grid still fills the chip (256 workgroups of the
  // 256 x 256 configuration, 512 of the smaller ones)
  const int64_t wgs = (mbp / tb) * (nbp / tb) * nchunks;
  const int64_t want = use >= 3 ? 256 : 512;
  const int groups = wgs >= want ? 1 : (int)std::min<int64_t>(D, ceil_div(want, wgs));
  if (use == 2) {
    const int64_t tiles = (mbp / 8) * (nbp / 8);
    hipLaunchKernelGGL((k_gemm_int8<2>), dim3((unsigned)tiles, (unsigned)nchunks, (unsigned)groups), dim3(64 * Int8Cfg<2>::WM * Int8Cfg<2>::WN), 0, st, a, b, mbp, nbp,
                       kbp, kbc, D, m, n, Sws, plane);
  } else if (use == 4) {
    const int64_t tiles = (mbp / 8) * (nbp / 8);
    hipLaunchKernelGGL((k_gemm_int8<4>), dim3((unsigned)tiles, (unsigned)nchunks, (unsigned)groups), dim3(64 * Int8Cfg<4>::WM * Int8Cfg<4>::WN), 0, st,
                       a, b, mbp, nbp, kbp, kbc, D, m, n, Sws, plane);
  } else if (use == 3) {
    const int64_t tiles = (mbp / 8) * (nbp / 8);
    hipLaunchKernelGGL((k_gemm_int8<3>), dim3((unsigned)tiles, (unsigned)nchunks, (unsigned)groups), dim3(64 * Int8Cfg<3>::WM * Int8Cfg<3>::WN), 0, st, a, b, mbp, nbp,
                       kbp, kbc, D, m, n, Sws, plane);
  } else {
    const int64_t tiles = (mbp / 4) * (nbp / 4);
    hipLaunchKernelGGL((k_gemm_int8<1>), dim3((unsigned)tiles, (unsigned)nchunks, (unsigned)groups), dim3(64 * Int8Cfg<1>::WM * Int8Cfg<1>::WN), 0, st, a, b, mbp, nbp,
                       kbp, kbc, D, m, n, Sws, plane);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int64_t blocks = ceil_div(mbp * nbp * 256, 256);
  hipLaunchKernelGGL((k_int8_combine<C>), dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, st, Sws,
                     plane, nchunks, D, combine_run(D, kbp), EA, EB, mbp, nbp, m, n, Cout, ldc, c_stride, debug_g,
                     Sdbg, lddbg);
  return hipGetLastError();
}

template <int C>
hipError_t launch_int8_batched(const Int8GemmDesc *descs, const int4 *items, int nitems1, int nitems3,
                               const int *bounds, int *counters, const int *prefix_blocks, int nprod, int64_t blocks,
                               hipStream_t st) {
  // items [0, nitems1): 128 x 128 tiles, two workgroups per CU; then the 256 x 256 ones, one per CU
  if (nitems1 > 0) {
    hipLaunchKernelGGL(k_gemm_int8_batched<1>, dim3(std::min(nitems1, 512)),
                       dim3(64 * Int8Cfg<1>::WM * Int8Cfg<1>::WN), 0, st, descs, items, bounds, counters);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  if (nitems3 > 0) {
    hipLaunchKernelGGL(k_gemm_int8_batched<3>, dim3(std::min(nitems3, 256)),
                       dim3(64 * Int8Cfg<3>::WM * Int8Cfg<3>::WN), 0, st, descs, items + nitems1, bounds + kXcds + 1,
                       counters + kXcds);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  if (blocks > 0) {
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_int8_combine_batched<C>), dim3((unsigned)blocks), dim3(256), 0, st, descs, prefix_blocks,
                       nprod);
    return hipGetLastError();
  }
  return hipSuccess;
}

#define MP_INT8_INST(C)                                                                                     \
  template hipError_t launch_gemm_int8<C>(const void *, const void *, const int *, const int *, int32_t *, int64_t, \
                                          int64_t, int64_t, int, int, int, double *, int, int64_t, int, int64_t *, \
                                          int, int, hipStream_t);
MP_INT8_INST(2)
MP_INT8_INST(3)
MP_INT8_INST(4)
MP_INT8_INST(5)
MP_INT8_INST(6)
MP_INT8_INST(7)
MP_INT8_INST(8)
MP_INT8_INST(9)
MP_INT8_INST(10)
MP_INT8_INST(11)
MP_INT8_INST(12)
MP_INT8_INST(13)
MP_INT8_INST(14)
template hipError_t launch_int8_batched<2>(const Int8GemmDesc *, const int4 *, int, int, const int *, int *,
                                           const int *, int, int64_t, hipStream_t);
template hipError_t launch_int8_batched<3>(const Int8GemmDesc *, const int4 *, int, int, const int *, int *,
                                           const int *, int, int64_t, hipStream_t);
template hipError_t launch_int8_batched<4>(const Int8GemmDesc *, const int4 *, int, int, const int *, int *,
                                           const int *, int, int64_t, hipStream_t);
#undef MP_INT8_INST

}  // namespace mp
