// Split kernels: Algorithm 1 (Section 3) of Utsugiri & Kouya, the loop that
// cuts A into slices A_1..A_D row by row and B into B_1..B_D column by column.
//
// Pass a (0-based) of a vector (a row of A or a column of B):
//   mu   = max |lead| over the vector          (lead: component 0 of the residual)
//   e    = ceil(log2 mu),  tau = 2^(e + rho),   rho = ceil((S + log2 k) / 2)
//   X_a  = (lead + tau) - tau                  (S-bit arithmetic: binary64 or binary32)
//   lead = lead - X_a                          (exact), then renormalize the residual
// The maximum for pass a + 1 is taken while pass a writes its residual, so the
// D passes cost D + 1 sweeps over the operand.  mu = 0 gives a zero slice.
// The residual after the last pass is dropped, so every slice product is exact.
//
// Each block handles a 64 x 64 tile of (vector, k) elements with 256 threads;
// lanes run along the contiguous memory index (the row index of a column-major
// A, the k index of a column-major B) so loads are coalesced.  Row maxima of A
// are combined across the block in LDS, column maxima of B with wavefront
// shuffles, then one integer atomic max per vector per block.
#include "internal.h"
#include "layout.h"
#include "mp_device.h"

namespace mp {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 64;
constexpr int kPerThread = kTile * kTile / kThreads;  // 16

struct TileCoord {
  int v0, p0;
};

// Tile of linear index idx for an operand covering nvec_cover x len_cover.
template <int ORIENT>
__device__ __forceinline__ TileCoord tile_of(int idx, int nvec_cover, int len_cover) {
  if (ORIENT == 0) {
    const int tc = (nvec_cover + kTile - 1) / kTile;
    return {(idx % tc) * kTile, (idx / tc) * kTile};
  } else {
    const int tc = (len_cover + kTile - 1) / kTile;
    return {(idx / tc) * kTile, (idx % tc) * kTile};
  }
}

// Element t (0..15) of this thread inside the tile.
template <int ORIENT>
__device__ __forceinline__ void elem_of(const TileCoord &tc, int t, int &v, int &p) {
  const int lane = threadIdx.x % 64, ty = threadIdx.x / 64;
  if (ORIENT == 0) {
    v = tc.v0 + lane;
    p = tc.p0 + ty + 4 * t;
  } else {
    p = tc.p0 + lane;
    v = tc.v0 + ty + 4 * t;
  }
}

__device__ __forceinline__ unsigned long long shfl_max(unsigned long long x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    unsigned long long y = __shfl_xor(x, off, 64);
    x = y > x ? y : x;
  }
  return x;
}
__device__ __forceinline__ unsigned int shfl_max(unsigned int x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    unsigned int y = __shfl_xor(x, off, 64);
    x = y > x ? y : x;
  }
  return x;
}

// Combine per-element maxima m[t] (bit patterns) into one atomic max per vector.
template <int ORIENT, typename U>
__device__ __forceinline__ void reduce_max(const TileCoord &tc, const U (&m)[kPerThread], U *mu, int nvec) {
  const int lane = threadIdx.x % 64, ty = threadIdx.x / 64;
  if (ORIENT == 0) {
    // all 16 elements of a thread share v = v0 + lane
    U best = 0;
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) best = m[t] > best ? m[t] : best;
    __shared__ U red[4][64];
    red[ty][lane] = best;
    __syncthreads();
    if (ty == 0) {
      U b = red[0][lane];
#pragma unroll
      for (int q = 1; q < 4; ++q) b = red[q][lane] > b ? red[q][lane] : b;
      const int v = tc.v0 + lane;
      if (v < nvec && b != 0) atomicMax(mu + v, b);
    }
  } else {
    // element t of the wavefront: one vector v = v0 + ty + 4 t, lanes along k
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const U b = shfl_max(m[t]);
      const int v = tc.v0 + ty + 4 * t;
      if (lane == 0 && v < nvec && b != 0) atomicMax(mu + v, b);
    }
  }
}

template <typename T, int C, int ORIENT>
__device__ void max0_body(const SplitOperand<T> &op, int idx) {
  using U = typename bits_of<T>::type;
  const TileCoord tc = tile_of<ORIENT>(idx, op.nvec, op.len);
  U m[kPerThread];
#pragma unroll
  for (int t = 0; t < kPerThread; ++t) {
    int v, p;
    elem_of<ORIENT>(tc, t, v, p);
    m[t] = (v < op.nvec && p < op.len) ? abs_bits(op.X[(int64_t)v * op.sv + (int64_t)p * op.sp]) : U(0);
  }
  reduce_max<ORIENT>(tc, m, static_cast<U *>(op.mu), op.nvec);
}

template <typename T, int C>
__global__ __launch_bounds__(kThreads) void k_split_max0(SplitOperand<T> a, SplitOperand<T> b, int blocks_a) {
  if ((int)blockIdx.x < blocks_a)
    max0_body<T, C, 0>(a, blockIdx.x);
  else
    max0_body<T, C, 1>(b, blockIdx.x - blocks_a);
}

template <typename T, int C, int ORIENT>
__device__ void pass_body(const SplitOperand<T> &op, int idx, int pass, int rho, bool first, bool last) {
  using U = typename bits_of<T>::type;
  const int nvec_cover = (int)(op.nbp * kBlk), len_cover = (int)(op.kbp * kKBlk);
  const TileCoord tc = tile_of<ORIENT>(idx, nvec_cover, len_cover);
  const U *mu_cur = static_cast<const U *>(op.mu) + (int64_t)pass * op.nvec;
  U *mu_next = static_cast<U *>(op.mu) + (int64_t)(pass + 1) * op.nvec;
  T *packed = static_cast<T *>(op.packed);
  const int64_t plane = (int64_t)op.nvec * op.len;
  // compact residual strides (same orientation as the input)
  const int64_t rsv = ORIENT == 0 ? 1 : op.len, rsp = ORIENT == 0 ? op.nvec : 1;
  U m[kPerThread];
#pragma unroll
  for (int t = 0; t < kPerThread; ++t) {
    int v, p;
    elem_of<ORIENT>(tc, t, v, p);
    m[t] = 0;
    if (v >= nvec_cover || p >= len_cover) continue;
    const bool valid = v < op.nvec && p < op.len;
    T sl = T(0);
    int e = kZeroExp;
    if (v < op.nvec) {
      const U mub = mu_cur[v];
      if (mub != 0) e = ceil_log2(from_bits(mub, T(0)));
    }
    if (valid) {
      T R[C];
      if (first) {
#pragma unroll
        for (int r = 0; r < C; ++r) R[r] = op.X[r * op.comp_stride + (int64_t)v * op.sv + (int64_t)p * op.sp];
      } else {
#pragma unroll
        for (int r = 0; r < C; ++r) R[r] = op.resid[r * plane + (int64_t)v * rsv + (int64_t)p * rsp];
      }
      if (e != kZeroExp) {
        const T tau = pow2(e + rho, T(0));
        const T lead = R[0];
        // Algorithm 1 as printed takes the residual's leading component as the
        // last slice (op.last_literal); by default it is extracted like the rest
        sl = last && op.last_literal ? lead : (lead + tau) - tau;
        R[0] = lead - sl;  // exact
        renorm<T, C>(R);
      }
      if (!last) {
#pragma unroll
        for (int r = 0; r < C; ++r) op.resid[r * plane + (int64_t)v * rsv + (int64_t)p * rsp] = R[r];
        m[t] = abs_bits(R[0]);
      }
    }
    packed[packed_index<sizeof(T) == 8>(pass, v, p, op.nbp, op.kbp)] = sl;
    // the thread holding k index 0 of vector v records the exponent of this pass
    if (p == 0 && v < op.nvec) op.exps[(int64_t)pass * op.nvec + v] = e;
  }
  if (!last) reduce_max<ORIENT>(tc, m, mu_next, op.nvec);
}

template <typename T, int C>
__global__ __launch_bounds__(kThreads) void k_split_pass(SplitOperand<T> a, SplitOperand<T> b, int blocks_a, int pass,
                                                         int rho, int first, int last) {
  if ((int)blockIdx.x < blocks_a)
    pass_body<T, C, 0>(a, blockIdx.x, pass, rho, first != 0, last != 0);
  else
    pass_body<T, C, 1>(b, blockIdx.x - blocks_a, pass, rho, first != 0, last != 0);
}

int tiles(int64_t nvec, int64_t len) { return (int)(ceil_div(nvec, kTile) * ceil_div(len, kTile)); }

// Operand owning global tile index b: the last i with prefix[i] <= b.
__device__ __forceinline__ int find_operand(const int *prefix, int nops, int b) {
  int lo = 0, hi = nops - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (prefix[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <typename T, int C>
__global__ __launch_bounds__(kThreads) void k_split_max0_batched(const SplitOperand<T> *ops, const int *prefix,
                                                                 int nops) {
  const int i = find_operand(prefix, nops, blockIdx.x);
  const SplitOperand<T> &op = ops[i];
  const int local = blockIdx.x - prefix[i];
  if (op.orient == 0)
    max0_body<T, C, 0>(op, local);
  else
    max0_body<T, C, 1>(op, local);
}

template <typename T, int C>
__global__ __launch_bounds__(kThreads) void k_split_pass_batched(const SplitOperand<T> *ops, const int *prefix,
                                                                 int nops, int pass) {
  const int i = find_operand(prefix, nops, blockIdx.x);
  const SplitOperand<T> &op = ops[i];
  if (pass >= op.D) return;  // uniform over the block
  const int local = blockIdx.x - prefix[i];
  const bool first = pass == 0, last = pass == op.D - 1;
  if (op.orient == 0)
    pass_body<T, C, 0>(op, local, pass, op.rho, first, last);
  else
    pass_body<T, C, 1>(op, local, pass, op.rho, first, last);
}

// ---------------------------------------------------------------------------
// Fused plain split.  While whole vectors fit in one workgroup's registers, a
// workgroup of NT threads (512 or 1024) takes nv vectors (nv of the 16 of one
// packed row/column block) over their full padded length and runs all D
// passes itself.  The maximum of each pass is reduced inside the workgroup, so
// the operand is read once and only the slices are written, instead of D + 1
// sweeps that read and write the residual.  Every element goes through the
// arithmetic of pass_body, step for step, so the slices and exponents are the
// same as those of the pass kernels.
//
// Thread t holds the strip elements t + NT j, numbered in packed
// order.  Each slice store is then a run of 2 nv (binary64) or 4 nv (binary32)
// consecutive elements per group of lanes, and every element of a thread lies
// in the same vector (that run length divides 64).
// ---------------------------------------------------------------------------
template <typename U>
__device__ __forceinline__ U umax(U a, U b) {
  return a > b ? a : b;
}

// Workgroups are dealt to the 8 XCDs in turn (b % 8); renumber them so that
// each XCD takes one contiguous range of strips.  Neighbouring strips of A
// share cache lines (a line holds 16 rows at one k), and this keeps those
// lines in one L2.  A bijection of [0, total).
__device__ __forceinline__ int xcd_contiguous(int b, int total) {
  const int per = total / 8, rem = total % 8, x = b % 8;
  return x * per + (x < rem ? x : rem) + b / 8;
}

template <typename T, int C, int NT>
__device__ void fused_strip(const SplitOperand<T> &op, int strip, int D, int rho) {
  using U = typename bits_of<T>::type;
  constexpr int kPer = fused_per_thread<T, C>();
  constexpr int kRunPer = sizeof(T) == 8 ? 2 : 4;  // consecutive packed elements of one vector
  constexpr int kWaves = NT / 64;
  const int64_t len_cover = op.kbp * kKBlk;
  const int nv = fused_vectors(len_cover, kPer, NT);
  const int run = kRunPer * nv, per_block = kBlk * nv;
  const int v0 = strip * nv, vb = v0 / kBlk, vl0 = v0 % kBlk;
  const int nl = (int)(nv * len_cover);
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int vo = (lane % run) / kRunPer;
  const int v = v0 + vo;
  const bool vec_ok = v < op.nvec;

  T R[kPer][C];
  int off[kPer];  // offset inside the strip's part of a slice plane; -1: beyond the strip
  bool valid[kPer];
  bool has_p0 = false;
  U m = 0;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int idx = tid + NT * j;
    off[j] = -1;
    valid[j] = false;
#pragma unroll
    for (int r = 0; r < C; ++r) R[j][r] = T(0);
    if (idx < nl) {
      const int kb = idx / per_block, rr = idx % per_block, g = rr / run, q = rr % run;
      int kl, within;
      if constexpr (sizeof(T) == 8) {
        const int st = 2 * (g / 4) + (q & 1);
        kl = 4 * st + g % 4;
        within = (g / 4) * 128 + 2 * ((g % 4) * 16 + vl0 + vo) + (q & 1);
      } else {
        const int st = q % 4;
        kl = 4 * st + g;
        within = 4 * (g * 16 + vl0 + vo) + st;
      }
      const int p = kb * kKBlk + kl;
      off[j] = kb * 256 + within;
      has_p0 = has_p0 || p == 0;
      valid[j] = vec_ok && p < op.len;
      if (valid[j]) {
#pragma unroll
        for (int r = 0; r < C; ++r) R[j][r] = op.X[r * op.comp_stride + (int64_t)v * op.sv + (int64_t)p * op.sp];
        m = umax(m, abs_bits(R[j][0]));
      }
    }
  }

  __shared__ U red[2][kWaves][kBlk];
  T *packed = static_cast<T *>(op.packed);
#pragma unroll 1
  for (int a = 0; a < D; ++a) {
    // maximum of the leading components of this vector's residual: lanes of
    // one vector first (xor over the bits below the run and from the run up),
    // then the waves through LDS (two buffers, so one barrier per pass)
    U mw = m;
#pragma unroll
    for (int o = 1; o < kRunPer; o <<= 1) mw = umax(mw, (U)__shfl_xor(mw, o, 64));
    for (int o = run; o < 64; o <<= 1) mw = umax(mw, (U)__shfl_xor(mw, o, 64));
    if (lane < run && lane % kRunPer == 0) red[a & 1][wave][vo] = mw;
    __syncthreads();
    U mu = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) mu = umax(mu, red[a & 1][w][vo]);
    int e = kZeroExp;
    if (vec_ok && mu != 0) e = ceil_log2(from_bits(mu, T(0)));
    const T tau = e != kZeroExp ? pow2(e + rho, T(0)) : T(0);
    const bool literal = op.last_literal && a == D - 1;
    T *dst = packed + ((int64_t)a * op.nbp + vb) * op.kbp * 256;
    m = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      if (off[j] < 0) continue;
      T sl = T(0);
      if (valid[j] && e != kZeroExp) {
        const T lead = R[j][0];
        sl = literal ? lead : (lead + tau) - tau;
        R[j][0] = lead - sl;  // exact
        renorm<T, C>(R[j]);
      }
      dst[off[j]] = sl;
      if (valid[j]) m = umax(m, abs_bits(R[j][0]));
    }
    if (has_p0 && vec_ok) op.exps[(int64_t)a * op.nvec + v] = e;
  }
}

template <typename T, int C, int NT>
__global__ __launch_bounds__(NT) void k_split_fused(SplitOperand<T> a, SplitOperand<T> b, int strips_a, int D,
                                                    int rho) {
  const int w = xcd_contiguous(blockIdx.x, gridDim.x);
  if (w < strips_a)
    fused_strip<T, C, NT>(a, w, D, rho);
  else
    fused_strip<T, C, NT>(b, w - strips_a, D, rho);
}

// Batched: workgroup b takes strip b - prefix[i] of operand i (operands split
// by the pass kernels own no strips).
template <typename T, int C, int NT>
__global__ __launch_bounds__(NT) void k_split_fused_batched(const SplitOperand<T> *ops, const int *prefix, int nops) {
  const int w = xcd_contiguous(blockIdx.x, gridDim.x);
  const int i = __builtin_amdgcn_readfirstlane(find_operand(prefix, nops, w));
  const SplitOperand<T> op = ops[i];  // uniform: kept in scalar registers
  fused_strip<T, C, NT>(op, w - prefix[i], op.D, op.rho);
}

__global__ void k_fill32(uint32_t *p, int64_t n, uint32_t value) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

}  // namespace

hipError_t launch_fill32(void *p, int64_t nwords, uint32_t value, hipStream_t st) {
  if (nwords <= 0) return hipSuccess;
  const int64_t blocks = ceil_div(nwords, 256);
  hipLaunchKernelGGL(k_fill32, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, st, (uint32_t *)p,
                     nwords, value);
  return hipGetLastError();
}

template <typename T, int C>
hipError_t launch_split_plain(const SplitOperand<T> &a, const SplitOperand<T> &b, int D, int rho, bool fused,
                              hipStream_t st) {
  using U = typename bits_of<T>::type;
  const int ta = fused_threads<T, C>(a.kbp * kKBlk), tb = fused_threads<T, C>(b.kbp * kKBlk);
  if (fused && ta > 0 && tb > 0) {
    const int nt = ta > tb ? ta : tb;
    const int sa = fused_strips<T, C>(a, nt), sb = fused_strips<T, C>(b, nt);
    if (sa + sb > 0 && D > 0) {
      if (nt == 512)
        hipLaunchKernelGGL((k_split_fused<T, C, 512>), dim3(sa + sb), dim3(512), 0, st, a, b, sa, D, rho);
      else
        hipLaunchKernelGGL((k_split_fused<T, C, 1024>), dim3(sa + sb), dim3(1024), 0, st, a, b, sa, D, rho);
      return hipGetLastError();
    }
    return hipSuccess;
  }
  // zero the per-pass maxima (a and b own separate arrays)
  hipError_t err = launch_fill32(a.mu, (int64_t)D * a.nvec * sizeof(U) / 4, 0u, st);
  if (err != hipSuccess) return err;
  err = launch_fill32(b.mu, (int64_t)D * b.nvec * sizeof(U) / 4, 0u, st);
  if (err != hipSuccess) return err;
  const int ba0 = a.nvec > 0 && a.len > 0 ? tiles(a.nvec, a.len) : 0;
  const int bb0 = b.nvec > 0 && b.len > 0 ? tiles(b.nvec, b.len) : 0;
  if (ba0 + bb0 > 0) {
    hipLaunchKernelGGL((k_split_max0<T, C>), dim3(ba0 + bb0), dim3(kThreads), 0, st, a, b, ba0);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  const int ba = a.nvec > 0 ? tiles(a.nbp * kBlk, a.kbp * kKBlk) : 0;
  const int bb = b.nvec > 0 ? tiles(b.nbp * kBlk, b.kbp * kKBlk) : 0;
  for (int pass = 0; pass < D; ++pass) {
    hipLaunchKernelGGL((k_split_pass<T, C>), dim3(ba + bb), dim3(kThreads), 0, st, a, b, ba, pass, rho,
                       pass == 0 ? 1 : 0, pass == D - 1 ? 1 : 0);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  return hipSuccess;
}

template <typename T, int C>
hipError_t launch_split_plain_batched(const SplitOperand<T> *ops, const int *prefix_max0, const int *prefix_pass,
                                      const int *prefix_fused, int nops, int tiles_max0, int tiles_pass,
                                      int strips_fused, int fused_nt, int dmax, void *mu_all, int64_t mu_words,
                                      hipStream_t st) {
  hipError_t err = hipSuccess;
  if (nops <= 0) return err;
  if (strips_fused > 0) {
    if (fused_nt == 512)
      hipLaunchKernelGGL((k_split_fused_batched<T, C, 512>), dim3(strips_fused), dim3(512), 0, st, ops, prefix_fused,
                         nops);
    else
      hipLaunchKernelGGL((k_split_fused_batched<T, C, 1024>), dim3(strips_fused), dim3(1024), 0, st, ops,
                         prefix_fused, nops);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  if (tiles_max0 <= 0 && tiles_pass <= 0) return hipSuccess;
  if ((err = launch_fill32(mu_all, mu_words, 0u, st)) != hipSuccess) return err;
  if (tiles_max0 > 0) {
    hipLaunchKernelGGL((k_split_max0_batched<T, C>), dim3(tiles_max0), dim3(kThreads), 0, st, ops, prefix_max0, nops);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  for (int pass = 0; pass < dmax && tiles_pass > 0; ++pass) {
    hipLaunchKernelGGL((k_split_pass_batched<T, C>), dim3(tiles_pass), dim3(kThreads), 0, st, ops, prefix_pass, nops,
                       pass);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  return hipSuccess;
}

#define MP_SPLIT_BATCHED(T, C)                                                                                 \
  template hipError_t launch_split_plain_batched<T, C>(const SplitOperand<T> *, const int *, const int *,         \
                                                       const int *, int, int, int, int, int, int, void *,     \
                                                       int64_t, hipStream_t);
MP_SPLIT_BATCHED(double, 2)
MP_SPLIT_BATCHED(double, 3)
MP_SPLIT_BATCHED(double, 4)
MP_SPLIT_BATCHED(float, 3)
#undef MP_SPLIT_BATCHED

template hipError_t launch_split_plain<double, 2>(const SplitOperand<double> &, const SplitOperand<double> &, int, int,
                                                  bool, hipStream_t);
template hipError_t launch_split_plain<double, 3>(const SplitOperand<double> &, const SplitOperand<double> &, int, int,
                                                  bool, hipStream_t);
template hipError_t launch_split_plain<double, 4>(const SplitOperand<double> &, const SplitOperand<double> &, int, int,
                                                  bool, hipStream_t);
template hipError_t launch_split_plain<float, 3>(const SplitOperand<float> &, const SplitOperand<float> &, int, int,
                                                 bool, hipStream_t);

// ---------------------------------------------------------------------------
// INT8 digit split (the precision form).  Per vector: E = 1 + ilogb(max |x_0|)
// (the frexp exponent of the maximum, so |x| < 2^E), then digit s (s = 1..D)
// is the extraction step of Algorithm 1 on the fixed grid
// u_s = 2^(E - 6 - 7 (s - 1)) applied to the exact residual: with
// W_s = RN(x / u_s) (nearest, ties to even) and W_0 = 0, d_s = W_s - 128 W_{s-1},
// so |d_s| <= 64 and sum_{t <= s} d_t u_t = W_s u_s.
//
// No floating-point step is taken.  The element's value is formed exactly as
// the two's complement integer N = floor(x / 2^P) in NW 32-bit words, with
// P = E - 7 Dw (Dw >= D: the digits the window holds), and a flag for a
// nonzero remainder below 2^P.  For a normalized expansion only the first
// component whose last bit lies below 2^P has bits there, and the components
// after it add less than that last bit, so the remainder is that component's
// cut-off bits moved by the sign of the first nonzero component after it.
// In window bits, digit s has its 7 bits b_s at 7 (Dw - s) + 1, its half bit
// h_s at 7 (Dw - s), and rounds up (r_s = 1) when h_s is set and anything
// below it is nonzero or b_s is odd; then d_s = b_s + r_s - 128 r_{s-1}, with
// r_0 the sign bit (bit 7 Dw).
//
// One workgroup per 32 x 32 block of one operand.  Thread T owns bytes
// 4T .. 4T+3 of the block in every digit plane: with l = T / 4 and q = T % 4
// these are row/column l % 32 of the block and k = 16 (l / 32) + 4 q + j,
// j = 0..3 (the packed INT8 layout), so each digit plane of the block is
// written by one coalesced 4-byte store per thread.
// ---------------------------------------------------------------------------
namespace {

// Digits a window of NW words holds.
template <int NW>
constexpr int window_digits() {
  return (32 * NW - 1) / 7;
}

// Smallest window (of the instantiated sizes) for D digits: 4..9 words for the
// DD/TD/QD formats (D <= 41), 13 or 25 for longer expansions (D <= 114).
int window_words(int D) {
  for (int nw : {4, 5, 6, 7, 8, 9, 13, 25})
    if ((32 * nw - 1) / 7 >= D) return nw;
  return 0;
}

// x = M 2^q exactly, |M| < 2^53 (zero gives M = 0).
__device__ __forceinline__ void binary64_parts(double x, int64_t &M, int &q) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const int ef = (int)((b >> 52) & 0x7ff);
  const int64_t f = (int64_t)(b & 0xfffffffffffffULL);
  const int64_t m = ef == 0 ? f : (f | (int64_t(1) << 52));
  q = ef == 0 ? -1074 : ef - 1075;
  M = (b >> 63) ? -m : m;
}

// w += M 2^off over all NW words (two's complement; off >= 0).  With
// off = 32 q + sh, M 2^sh spans three words x0, x1, x2 (the sign beyond), and
// word i receives the one of them numbered i - q: selects, no branches.
template <int NW>
__device__ __forceinline__ void window_add(uint32_t (&w)[NW], int64_t M, int off) {
  const int q = off >> 5, sh = off & 31;
  const uint64_t u = (uint64_t)M << sh;
  const uint32_t sign = (uint32_t)(M >> 63);
  const uint32_t x0 = (uint32_t)u, x1 = (uint32_t)(u >> 32);
  const uint32_t x2 = sh ? (uint32_t)(M >> (64 - sh)) : sign;
  uint32_t carry = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const int d = i - q;
    const uint32_t part = d < 0 ? 0u : d == 0 ? x0 : d == 1 ? x1 : d == 2 ? x2 : sign;
    const uint64_t sum = (uint64_t)w[i] + part + carry;
    w[i] = (uint32_t)sum;
    carry = (uint32_t)(sum >> 32);
  }
}

// N = floor(x / 2^P) of the c components x[r * stride] (a normalized
// expansion) into w, and whether x - N 2^P is nonzero.  The loop over the
// components is unrolled for the DD/TD/QD formats (CMAX <= 4) only.
template <int CMAX, int NW>
__device__ __forceinline__ void value_window(const double *x, int64_t stride, int c, int P, uint32_t (&w)[NW],
                                             bool &below) {
#pragma unroll
  for (int i = 0; i < NW; ++i) w[i] = 0u;
  bool cut = false, cut_bits = false;
  int tail = 0;  // sign of the first nonzero component after the cut one
  constexpr int kUnroll = CMAX <= 4 ? CMAX : 1;
#pragma unroll kUnroll
  for (int r = 0; r < c; ++r) {
    const double xr = x[r * stride];
    if (xr == 0.0) continue;
    if (cut) {
      if (tail == 0) tail = xr < 0.0 ? -1 : 1;
      continue;
    }
    int64_t M;
    int q;
    binary64_parts(xr, M, q);
    int off = q - P;
    if (off < 0) {  // bits below 2^P: floor, and whether any was cut off
      const int sh = -off;
      cut_bits = sh >= 64 ? true : (M & ((int64_t(1) << sh) - 1)) != 0;
      M = sh >= 64 ? (M < 0 ? -1 : 0) : (M >> sh);
      off = 0;
      cut = true;
    }
    window_add<NW>(w, M, off);
  }
  below = false;
  if (cut) {
    if (!cut_bits && tail < 0) {  // a remainder of 0 moved below zero: borrow
      window_add<NW>(w, -1, 0);
      below = true;
    } else {
      below = cut_bits || tail != 0;
    }
  }
}

template <int NW>
__device__ __forceinline__ uint32_t window_bit(const uint32_t (&w)[NW], int j) {
  return (w[j >> 5] >> (j & 31)) & 1u;
}

// bits j .. j + 6
template <int NW>
__device__ __forceinline__ uint32_t window_bits7(const uint32_t (&w)[NW], int j) {
  const int i = j >> 5, o = j & 31;
  uint32_t v = w[i] >> o;
  if (o > 25 && i + 1 < NW) v |= w[i + 1] << (32 - o);
  return v & 127u;
}

// LIVE: blk numbers only the blocks that hold an element of the operand (the
// padding blocks of the packed planes were cleared once and are not written);
// otherwise every packed block, padding included.
template <int CMAX, int NW, int ORIENT, bool LIVE = false>
__device__ void int8_block(const SplitOperand<double> &op, int64_t blk, int D, int c) {
  constexpr int Dw = window_digits<NW>();
  const int64_t nb = LIVE ? ceil_div((int64_t)op.nvec, (int64_t)kBlk8) : op.nbp;
  const int64_t kbn = LIVE ? ceil_div((int64_t)op.len, (int64_t)kKBlk8) : op.kbp;
  // A (rows, contiguous along the row index): walk row blocks fastest;
  // B (columns, contiguous along k): walk k blocks fastest.
  const int64_t vb = ORIENT == 0 ? blk % nb : blk / kbn;
  const int64_t kb = ORIENT == 0 ? blk / nb : blk % kbn;
  const int T = threadIdx.x, l = T >> 2, q = T & 3;
  const int v = (int)(vb * kBlk8) + (l & 31);
  const int p0 = (int)(kb * kKBlk8) + 16 * (l >> 5) + 4 * q;
  const unsigned long long *mu = static_cast<const unsigned long long *>(op.mu);

  int E = kZeroExp;
  if (v < op.nvec && mu[v] != 0) {
    int ex;
    (void)frexp(from_bits(mu[v], 0.0), &ex);
    E = ex;
  }
  const int P = E != kZeroExp ? E - 7 * Dw : 0;
  int8_t *dst = static_cast<int8_t *>(op.packed) + (vb * op.kbp + kb) * 1024 + 4 * T;
  const int64_t plane = op.nbp * op.kbp * 1024;
  // the thread's 4 elements in groups of G (fewer for wide windows, whose
  // words would not all fit in registers); each group's digits are stored as
  // G consecutive bytes of every plane
  constexpr int G = NW <= 7 ? 4 : NW <= 13 ? 2 : 1;
#pragma unroll 1
  for (int j0 = 0; j0 < 4; j0 += G) {
    uint32_t w[G][NW];
    bool below[G];
    uint32_t anyw[G];  // bit i: a nonzero word below word i
    int rprev[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int p = p0 + j0 + j;
      const bool live = v < op.nvec && p < op.len && E != kZeroExp;
      value_window<CMAX, NW>(op.X + (live ? (int64_t)v * op.sv + (int64_t)p * op.sp : 0), op.comp_stride,
                             live ? (CMAX <= 4 ? CMAX : c) : 0, P, w[j], below[j]);
      uint32_t run = 0u, m = 0u;
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        m |= (run != 0u ? 1u : 0u) << i;
        run |= w[j][i];
      }
      anyw[j] = m;
      rprev[j] = (int)window_bit(w[j], 7 * Dw);  // the sign: W_0 = 0
    }
    // every digit the window holds is formed (the bit positions are then
    // constants); the first D are stored
#pragma unroll
    for (int s = 1; s <= Dw; ++s) {
      const int ph = 7 * (Dw - s);  // half bit of digit s
      unsigned int word = 0;
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const uint32_t b = window_bits7(w[j], ph + 1);
        const uint32_t h = window_bit(w[j], ph);
        const bool st = below[j] || ((anyw[j] >> (ph >> 5)) & 1u) || (w[j][ph >> 5] & ((1u << (ph & 31)) - 1u)) != 0u;
        const int r = (int)(h & ((st ? 1u : 0u) | (b & 1u)));
        const int d = (int)b + r - 128 * rprev[j];
        rprev[j] = r;
        word |= (unsigned int)(uint8_t)(int8_t)d << (8 * j);
      }
      if (s <= D) {
        int8_t *out = dst + (int64_t)(s - 1) * plane + j0;
        if constexpr (G == 4)
          *reinterpret_cast<unsigned int *>(out) = word;
        else if constexpr (G == 2)
          *reinterpret_cast<unsigned short *>(out) = (unsigned short)word;
        else
          *out = (int8_t)word;
      }
    }
  }
  if (p0 == 0 && v < op.nvec) op.exps[v] = E;
}

template <int CMAX, int NW>
__global__ __launch_bounds__(kThreads) void k_split_int8(SplitOperand<double> a, SplitOperand<double> b,
                                                         int64_t blocks_a, int D, int c) {
  const int64_t blk = (int64_t)blockIdx.x;
  if (blk < blocks_a)
    int8_block<CMAX, NW, 0>(a, blk, D, c);
  else
    int8_block<CMAX, NW, 1>(b, blk - blocks_a, D, c);
}

// Batched: workgroup b takes live block b - prefix[i] of operand i (ops[i].D
// digits; the window holds the batch's largest D).  The batch's packed planes
// are cleared when its plan is built, so padding blocks are never written.
template <int C, int NW>
__global__ __launch_bounds__(kThreads) void k_split_int8_batched(const SplitOperand<double> *ops, const int *prefix,
                                                                 int nops) {
  const int i = find_operand(prefix, nops, blockIdx.x);
  const SplitOperand<double> &op = ops[i];
  const int64_t local = (int64_t)blockIdx.x - prefix[i];
  if (op.orient == 0)
    int8_block<C, NW, 0, true>(op, local, op.D, C);
  else
    int8_block<C, NW, 1, true>(op, local, op.D, C);
}

// Digit kernel for c components and D digits: the DD/TD/QD formats in their own
// instantiations, longer expansions in one generic one (up to 14 components).
template <int C>
hipError_t launch_int8_digits(const SplitOperand<double> &a, const SplitOperand<double> &b, int64_t ba, int64_t bb,
                              int D, hipStream_t st) {
  constexpr int CM = C <= 4 ? C : 14;
  const dim3 grid((unsigned)(ba + bb)), block(kThreads);
  int nw = window_words(D);
  if (C > 4 && nw > 0 && nw < 9) nw = 9;
  switch (nw) {
#define MP_DIGITS_CASE(NW)                                                                                  \
  case NW:                                                                                                  \
    if constexpr ((C <= 4 && NW <= 9) || (C > 4 && NW >= 9)) {                                              \
      hipLaunchKernelGGL((k_split_int8<CM, NW>), grid, block, 0, st, a, b, ba, D, C);                       \
      return hipGetLastError();                                                                             \
    }                                                                                                       \
    break;
    MP_DIGITS_CASE(4)
    MP_DIGITS_CASE(5)
    MP_DIGITS_CASE(6)
    MP_DIGITS_CASE(7)
    MP_DIGITS_CASE(8)
    MP_DIGITS_CASE(9)
    MP_DIGITS_CASE(13)
    MP_DIGITS_CASE(25)
#undef MP_DIGITS_CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace

template <int C>
hipError_t launch_split_int8(const SplitOperand<double> &a, const SplitOperand<double> &b, int D, hipStream_t st) {
  hipError_t err = launch_fill32(a.mu, (int64_t)a.nvec * 2, 0u, st);
  if (err != hipSuccess) return err;
  if ((err = launch_fill32(b.mu, (int64_t)b.nvec * 2, 0u, st)) != hipSuccess) return err;
  const int ba0 = a.nvec > 0 && a.len > 0 ? tiles(a.nvec, a.len) : 0;
  const int bb0 = b.nvec > 0 && b.len > 0 ? tiles(b.nvec, b.len) : 0;
  if (ba0 + bb0 > 0) {
    hipLaunchKernelGGL((k_split_max0<double, C>), dim3(ba0 + bb0), dim3(kThreads), 0, st, a, b, ba0);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  // one workgroup of kThreads (= 1024 / 4) threads per 32 x 32 block
  static_assert(kThreads * 4 == kBlk8 * kKBlk8, "thread per 4 bytes of a block");
  const int64_t ba = a.nvec > 0 ? a.nbp * a.kbp : 0;
  const int64_t bb = b.nvec > 0 ? b.nbp * b.kbp : 0;
  if (ba + bb > 0) {
    if (ba + bb > 0x7fffffffLL) return hipErrorInvalidValue;
    return launch_int8_digits<C>(a, b, ba, bb, D, st);
  }
  return hipSuccess;
}

template <int C>
hipError_t launch_split_int8_batched(const SplitOperand<double> *ops, const int *prefix_max0, const int *prefix_blk,
                                     int nops, int tiles_max0, int64_t blocks, int dmax, void *mu_all,
                                     int64_t mu_words, hipStream_t st) {
  hipError_t err = launch_fill32(mu_all, mu_words, 0u, st);
  if (err != hipSuccess) return err;
  if (tiles_max0 > 0) {
    hipLaunchKernelGGL((k_split_max0_batched<double, C>), dim3(tiles_max0), dim3(kThreads), 0, st, ops, prefix_max0,
                       nops);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  if (blocks > 0) {
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    switch (window_words(dmax)) {
#define MP_DIGITS_BATCHED_CASE(NW)                                                                           \
  case NW:                                                                                                   \
    hipLaunchKernelGGL((k_split_int8_batched<C, NW>), dim3((unsigned)blocks), dim3(kThreads), 0, st, ops,     \
                       prefix_blk, nops);                                                                    \
    return hipGetLastError();
      MP_DIGITS_BATCHED_CASE(4)
      MP_DIGITS_BATCHED_CASE(5)
      MP_DIGITS_BATCHED_CASE(6)
      MP_DIGITS_BATCHED_CASE(7)
      MP_DIGITS_BATCHED_CASE(8)
      MP_DIGITS_BATCHED_CASE(9)
#undef MP_DIGITS_BATCHED_CASE
      default:
        return hipErrorInvalidValue;
    }
  }
  return hipSuccess;
}

template hipError_t launch_split_int8_batched<2>(const SplitOperand<double> *, const int *, const int *, int, int,
                                                 int64_t, int, void *, int64_t, hipStream_t);
template hipError_t launch_split_int8_batched<3>(const SplitOperand<double> *, const int *, const int *, int, int,
                                                 int64_t, int, void *, int64_t, hipStream_t);
template hipError_t launch_split_int8_batched<4>(const SplitOperand<double> *, const int *, const int *, int, int,
                                                 int64_t, int, void *, int64_t, hipStream_t);

#define MP_SPLIT_INT8_LONG(C) \
  template hipError_t launch_split_int8<C>(const SplitOperand<double> &, const SplitOperand<double> &, int, hipStream_t);
MP_SPLIT_INT8_LONG(5)
MP_SPLIT_INT8_LONG(6)
MP_SPLIT_INT8_LONG(7)
MP_SPLIT_INT8_LONG(8)
MP_SPLIT_INT8_LONG(9)
MP_SPLIT_INT8_LONG(10)
MP_SPLIT_INT8_LONG(11)
MP_SPLIT_INT8_LONG(12)
MP_SPLIT_INT8_LONG(13)
MP_SPLIT_INT8_LONG(14)
#undef MP_SPLIT_INT8_LONG
template hipError_t launch_split_int8<2>(const SplitOperand<double> &, const SplitOperand<double> &, int, hipStream_t);
template hipError_t launch_split_int8<3>(const SplitOperand<double> &, const SplitOperand<double> &, int, hipStream_t);
template hipError_t launch_split_int8<4>(const SplitOperand<double> &, const SplitOperand<double> &, int, hipStream_t);

// ---------------------------------------------------------------------------
// Debug unpacking of packed slices.
// ---------------------------------------------------------------------------
namespace {
__global__ void k_unpack(int elem_bytes, const void *packed, int64_t nbp, int64_t kbp, int D, int orient, int rows,
                         int cols, void *out) {
  const int64_t plane = (int64_t)rows * cols;
  const int64_t total = plane * D;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(i / plane);
    const int64_t rem = i % plane;
    const int r = (int)(rem % rows), c = (int)(rem / rows);
    // operand 0: rows = vectors (rows of A), cols = k; operand 1: rows = k, cols = vectors
    const int64_t v = orient == 0 ? r : c, p = orient == 0 ? c : r;
    if (elem_bytes == 8)
      static_cast<double *>(out)[i] = static_cast<const double *>(packed)[packed_index<true>(a, v, p, nbp, kbp)];
    else if (elem_bytes == 4)
      static_cast<float *>(out)[i] = static_cast<const float *>(packed)[packed_index<false>(a, v, p, nbp, kbp)];
    else
      static_cast<int8_t *>(out)[i] = static_cast<const int8_t *>(packed)[packed_index8(a, v, p, nbp, kbp)];
  }
}
}  // namespace

hipError_t launch_unpack(int elem_bytes, const void *packed, int64_t nbp, int64_t kbp, int D, int orient, int rows,
                         int cols, void *out, hipStream_t st) {
  const int64_t total = (int64_t)rows * cols * D;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = ceil_div(total, 256);
  hipLaunchKernelGGL(k_unpack, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), 0, st, elem_bytes, packed,
                     nbp, kbp, D, orient, rows, cols, out);
  return hipGetLastError();
}

}  // namespace mp
