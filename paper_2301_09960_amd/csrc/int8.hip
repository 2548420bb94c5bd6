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
// k_gemm_int8: one workgroup (4 wavefronts) per 128 x 128 tile of C and k
// chunk; each wavefront owns 64 x 64 as 2 x 2 blocks of
// v_mfma_i32_32x32x32_i8; 16 KiB panels (A_s and B_t, 128 x 64 digits each)
// are staged through two LDS buffers as in the floating-point kernel.  After
// the last pair of a diagonal the 32-bit tile is written to the S_g plane.
//
// k_int8_combine: per element, C = sum_g S_g 2^(E_i + F_j + 2 - 7 (g + 1)),
// every term exact in binary64, added with TwoSum into a (c+1)-term
// accumulator and renormalized into the c components of C (HBM-bound: it
// reads D 32-bit sums per element per chunk and writes C once).
#include "internal.h"
#include "layout.h"
#include "mp_device.h"

namespace mp {
namespace {

constexpr int kThreads = 256;
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

__global__ __launch_bounds__(kThreads) void k_gemm_int8(const int8_t *__restrict__ Apk, const int8_t *__restrict__ Bpk,
                                                        int64_t mbp, int64_t nbp, int64_t kbp, int kb_chunk, int D,
                                                        int m, int n, int32_t *__restrict__ S, int64_t plane) {
  constexpr int kSegBytes = kKStepBlocks8 * 1024;       // one 32-row block x one k step
  constexpr int kPanelBytes = kTileBlocks8 * kSegBytes;  // 128 rows x 64 k
  __shared__ __attribute__((aligned(16))) int8_t lds[2][2][kPanelBytes];

  const int tiles_m = (int)(mbp / kTileBlocks8), tiles_n = (int)(nbp / kTileBlocks8);
  int tm, tn;
  tile_coords(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
  const int chunk = blockIdx.y, nchunks = gridDim.y;
  const int64_t kb0 = (int64_t)chunk * kb_chunk;
  const int64_t kb1 = kb0 + kb_chunk < kbp ? kb0 + kb_chunk : kbp;
  const int nks = (int)((kb1 - kb0) / kKStepBlocks8);
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int wm = wave % 2, wn = wave / 2;
  const int seg = tid / 64;
  const int64_t total = (int64_t)D * (D + 1) / 2 * nks;

  // load cursor: diagonal g (1-based), pair index s (1..g), k step
  int lg = 1, ls = 1, lks = 0;
  u4 ra[2], rb[2];
  auto load_step = [&](int g, int s, int ks) {
    const int t = g + 1 - s;
    const u4 *pa = reinterpret_cast<const u4 *>(
        Apk + (((int64_t)(s - 1) * mbp + tm * kTileBlocks8 + seg) * kbp + kb0 + (int64_t)ks * kKStepBlocks8) * 1024);
    const u4 *pb = reinterpret_cast<const u4 *>(
        Bpk + (((int64_t)(t - 1) * nbp + tn * kTileBlocks8 + seg) * kbp + kb0 + (int64_t)ks * kKStepBlocks8) * 1024);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      ra[j] = pa[j * 64 + lane];
      rb[j] = pb[j * 64 + lane];
    }
  };
  auto store_stage = [&](int stage) {
    u4 *sa = reinterpret_cast<u4 *>(&lds[stage][0][seg * kSegBytes]);
    u4 *sb = reinterpret_cast<u4 *>(&lds[stage][1][seg * kSegBytes]);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      sa[j * 64 + lane] = ra[j];
      sb[j * 64 + lane] = rb[j];
    }
  };
  auto advance = [&](int &g, int &s, int &ks) {
    if (++ks == nks) {
      ks = 0;
      if (++s > g) {
        ++g;
        s = 1;
      }
    }
  };

  i16v acc[2][2];
#pragma unroll
  for (int jb = 0; jb < 2; ++jb)
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[jb][ib][r] = 0;

  if (total > 0) {
    load_step(lg, ls, lks);
    store_stage(0);
    advance(lg, ls, lks);
  }
  __syncthreads();

  int cg = 1, cs = 1, cks = 0;  // compute cursor
  for (int64_t step = 0; step < total; ++step) {
    const int stage = (int)(step & 1);
    const bool more = step + 1 < total;
    if (more) load_step(lg, ls, lks);
#pragma unroll
    for (int kb = 0; kb < kKStepBlocks8; ++kb) {
      i4v fa[2], fb[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        fa[x] = *reinterpret_cast<const i4v *>(&lds[stage][0][((wm * 2 + x) * kKStepBlocks8 + kb) * 1024 + 16 * lane]);
        fb[x] = *reinterpret_cast<const i4v *>(&lds[stage][1][((wn * 2 + x) * kKStepBlocks8 + kb) * 1024 + 16 * lane]);
      }
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
          acc[jb][ib] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fb[jb], fa[ib], acc[jb][ib], 0, 0, 0);
    }
    if (++cks == nks) {
      cks = 0;
      if (++cs > cg) {  // diagonal cg complete: write its exact partial sum
        int32_t *out = S + ((int64_t)(cg - 1) * nchunks + chunk) * plane;
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
          for (int ib = 0; ib < 2; ++ib) {
            const int i = tm * 128 + wm * 64 + ib * 32 + lane % 32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int j = tn * 128 + wn * 64 + jb * 32 + 8 * (r / 4) + 4 * (lane / 32) + r % 4;
              if (i < m && j < n) out[i + (int64_t)j * m] = acc[jb][ib][r];
              acc[jb][ib][r] = 0;
            }
          }
        ++cg;
        cs = 1;
      }
    }
    if (more) {
      store_stage(stage ^ 1);
      advance(lg, ls, lks);
    }
    __syncthreads();
  }
}

template <int C>
__global__ __launch_bounds__(256) void k_int8_combine(const int32_t *__restrict__ S, int64_t plane, int nchunks, int D,
                                                      const int *__restrict__ EA, const int *__restrict__ EB, int m,
                                                      int n, double *__restrict__ Cout, int ldc, int64_t c_stride,
                                                      int debug_g, int64_t *__restrict__ Sdbg, int lddbg) {
  const int64_t total = (int64_t)m * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    const int Ei = EA[i], Fj = EB[j];
    const bool live = Ei != kZeroExp && Fj != kZeroExp;
    double acc[C + 1];
#pragma unroll
    for (int q = 0; q <= C; ++q) acc[q] = 0.0;
    for (int g = 1; g <= D; ++g) {
      int64_t s = 0;
      for (int c = 0; c < nchunks; ++c) s += S[((int64_t)(g - 1) * nchunks + c) * plane + e];
      if (debug_g == g) Sdbg[i + (int64_t)j * lddbg] = s;
      if (live && s != 0) acc_add<double, C + 1>(acc, ldexp((double)s, Ei + Fj + 2 - 7 * (g + 1)));
    }
    if (debug_g > 0) continue;
    renorm<double, C + 1>(acc);
#pragma unroll
    for (int q = 0; q < C; ++q) Cout[q * c_stride + i + (int64_t)j * ldc] = acc[q];
  }
}

}  // namespace

// Longest k chunk (in 32-wide k blocks, a multiple of the k step) whose
// diagonal sums stay within 32 bits: D * k_chunk * 64 * 64 < 2^31.
int int8_kblocks_per_chunk(int D) {
  int64_t kc = ((int64_t(1) << 31) - 1) / (int64_t(4096) * (D > 0 ? D : 1));
  int64_t blocks = kc / (kKBlk8 * kKStepBlocks8) * kKStepBlocks8;
  return (int)(blocks > kKStepBlocks8 ? blocks : kKStepBlocks8);
}

template <int C>
hipError_t launch_gemm_int8(const void *Apk, const void *Bpk, const int *EA, const int *EB, int32_t *Sws, int64_t mbp,
                            int64_t nbp, int64_t kbp, int m, int n, int D, double *Cout, int ldc, int64_t c_stride,
                            int debug_g, int64_t *Sdbg, int lddbg, hipStream_t st) {
  const int64_t tiles = (mbp / kTileBlocks8) * (nbp / kTileBlocks8);
  if (tiles <= 0 || m <= 0 || n <= 0) return hipSuccess;
  const int kbc = int8_kblocks_per_chunk(D);
  const int nchunks = (int)ceil_div(kbp, kbc);
  const int64_t plane = (int64_t)m * n;
  hipLaunchKernelGGL(k_gemm_int8, dim3((unsigned)tiles, (unsigned)nchunks), dim3(kThreads), 0, st,
                     static_cast<const int8_t *>(Apk), static_cast<const int8_t *>(Bpk), mbp, nbp, kbp, kbc, D, m, n,
                     Sws, plane);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int64_t blocks = ceil_div(plane, 256);
  hipLaunchKernelGGL((k_int8_combine<C>), dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, st, Sws,
                     plane, nchunks, D, EA, EB, m, n, Cout, ldc, c_stride, debug_g, Sdbg, lddbg);
  return hipGetLastError();
}

template hipError_t launch_gemm_int8<2>(const void *, const void *, const int *, const int *, int32_t *, int64_t,
                                        int64_t, int64_t, int, int, int, double *, int, int64_t, int, int64_t *, int,
                                        hipStream_t);
template hipError_t launch_gemm_int8<3>(const void *, const void *, const int *, const int *, int32_t *, int64_t,
                                        int64_t, int64_t, int, int, int, double *, int, int64_t, int, int64_t *, int,
                                        hipStream_t);
template hipError_t launch_gemm_int8<4>(const void *, const void *, const int *, const int *, int32_t *, int64_t,
                                        int64_t, int64_t, int, int, int, double *, int, int64_t, int, int64_t *, int,
                                        hipStream_t);

}  // namespace mp
