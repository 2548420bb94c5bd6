// A-posteriori error certificate of the slice product (binary64/binary32 or INT8 slices).
//
// With D slices per row of A and column of B (Algorithm 1, Section 3), write
// A = A_s + RA and B = B_s + RB, where A_s is the sum of the slices and RA the
// remainder left by the D passes.  The product computed from the triangle
// a + b <= D + 1 (the pairs the statement after Fig. 1 keeps) differs from AB by
//   AB - C_tri = sum_{a,b <= D, a + b > D + 1} A_a B_b + A_s RB + RA B,
// and the computed C differs from C_tri by the rounding of the accumulation to
// c components.  Per entry (i, j) this file bounds each part from quantities
// the split already produced (in either slice form: an INT8 digit plane is a
// slice on the fixed grid of E - 6 - 7 (s - 1)), and bounds (|A||B|)_ij from below:
//   T1 = k sum_{dropped (a, b)} 2^(eA_a,i + eB_b,j)      |A_a,ip| <= 2^eA_a,i
//   T2 = rB_j (rsA_i + k rA_i)                             |A_s| <= |A| + |RA|
//   T3 = rA_i csB_j
//   T4 = 2^(4 - S c) UB_ij                                 final rounding of C
// with rA_i the bound on the remainder after the last slice (remainder_bound),
// rsA_i / csB_j upper bounds of the row sums of |A| and column sums of |B|, and
// UB_ij / LB_ij upper / lower bounds of (|A||B|)_ij
// from one binary64 product of the absolute leading components |A_0| |B_0|
// (run on the slice-product kernel as a single pair).  Entry (i, j) is
// certified when T1 + T2 + T3 + T4 <= 2^-t LB_ij.
#include "internal.h"
#include "layout.h"
#include "mp_device.h"

namespace mp {
namespace {

constexpr int kCertThreads = 256;

// |X_0| of one operand in the packed binary64 layout (slice plane 0), zero in
// the padding: thread per packed element, so stores are contiguous.
template <typename T>
__global__ __launch_bounds__(kCertThreads) void k_pack_abs_lead(SplitOperand<T> op, double *out) {
  const int64_t total = op.nbp * op.kbp * 256;
  for (int64_t idx = blockIdx.x * (int64_t)kCertThreads + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kCertThreads) {
    const int64_t blk = idx / 256, kb = blk % op.kbp, vb = blk / op.kbp;
    const int within = (int)(idx % 256);
    // invert the binary64 packed order: within = (s / 2) 128 + 2 lane + (s % 2)
    const int half = within / 128, r = within % 128, lane = r / 2, s = 2 * half + r % 2;
    const int64_t v = vb * kBlk + lane % 16, p = kb * kKBlk + 4 * s + lane / 16;
    double x = 0.0;
    if (v < op.nvec && p < op.len) x = fabs((double)op.X[v * op.sv + p * op.sp]);
    out[idx] = x;
  }
}

// Sum over p of |X_0(v, p)| for every vector v, in a fixed order.
// Rows of A (v contiguous in memory): a workgroup of 1024 threads takes 64
// rows; lane l of wavefront w adds p = w, w + 16, ... of row l (each wavefront
// reads 64 neighbouring rows at one p), and the 16 partial sums meet in LDS.
template <typename T>
__global__ __launch_bounds__(1024) void k_abs_row_sums(SplitOperand<T> op, double *sums) {
  __shared__ double part[16][64];
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int v = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (v < op.nvec)
    for (int p = w; p < op.len; p += 16) s += fabs((double)op.X[(int64_t)v * op.sv + (int64_t)p * op.sp]);
  part[w][lane] = s;
  __syncthreads();
  if (w == 0 && v < op.nvec) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += part[q][lane];
    sums[v] = t;
  }
}

// Columns of B (p contiguous): one wavefront per column, lanes along p, then a
// shuffle reduction.
template <typename T>
__global__ __launch_bounds__(kCertThreads) void k_abs_sums(SplitOperand<T> op, double *sums) {
  const int v = blockIdx.x * (kCertThreads / 64) + threadIdx.x / 64, lane = threadIdx.x % 64;
  if (v >= op.nvec) return;  // uniform over the wavefront
  double s = 0.0;
  for (int p = lane; p < op.len; p += 64) s += fabs((double)op.X[(int64_t)v * op.sv + (int64_t)p * op.sp]);
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) sums[v] = s;
}

__device__ __forceinline__ double pow2d(int e) { return ldexp(1.0, e); }

// Exponent bounding slice a (1-based) of vector v: FLOAT form, the pass's
// ceil(log2 mu) (exps holds D x nvec); INT8 form, E_v - 7 (a - 1), since a digit
// is at most 64 units u_a = 2^(E_v - 6 - 7 (a - 1)) (exps holds E per vector).
__device__ __forceinline__ int slice_exp(const int *exps, int nvec, int v, int a, bool int8) {
  if (!int8) return exps[(int64_t)(a - 1) * nvec + v];
  const int E = exps[v];
  return E == kZeroExp ? kZeroExp : E - 7 * (a - 1);
}

// Bound of the remainder after D slices: FLOAT form, 2^(e_D + rho - S)
// (1 + 2^(1 - rho)) (half a grid step of the last pass, and the rounding of the
// grid to the sum); INT8 form, u_D / 2 = 2^(E - 7 D), with a margin for the
// components below the leading one.
__device__ __forceinline__ double remainder_bound(const int *exps, int nvec, int v, int D, int rho, int S,
                                                  bool int8) {
  if (int8) {
    const int E = exps[v];
    return E == kZeroExp ? 0.0 : ldexp(1.0, E - 7 * D) * (1.0 + ldexp(1.0, -40));
  }
  const int e = exps[(int64_t)(D - 1) * nvec + v];
  return e == kZeroExp ? 0.0 : ldexp(1.0, e + rho - S) * (1.0 + ldexp(1.0, 1 - rho));
}

// Per entry: reads the single-pair product of |A_0| |B_0| from plane 0 of
// `cert`, writes the error bound there and the lower bound of (|A||B|)_ij to
// plane 1, and raises *worst to the largest ratio (bit patterns of
// non-negative doubles order like the values).
__global__ __launch_bounds__(kCertThreads) void k_certify(int m, int n, int k, int D, int rho, int S, int comps,
                                                          int int8, const int *__restrict__ eA,
                                                          const int *__restrict__ eB,
                                                          const double *__restrict__ rsA,
                                                          const double *__restrict__ csB, double *cert,
                                                          unsigned long long *worst,
                                                          const int8_t *__restrict__ lims, int tiles_m) {
  const int64_t mn = (int64_t)m * n;
  const double u = ldexp(1.0, -52);
  const double sum_up = 1.0 + (k + 2) * u;  // |computed sum - exact| <= (k - 1) u' (sum), u' = 2^-53
  const double lead_lo = 1.0 - ldexp(1.0, 2 - S), lead_hi = 1.0 + ldexp(1.0, 2 - S);  // |x_0| vs |x|
  unsigned long long local = 0;
  for (int64_t idx = blockIdx.x * (int64_t)kCertThreads + threadIdx.x; idx < mn;
       idx += (int64_t)gridDim.x * kCertThreads) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    const double raw = cert[idx];
    const double lb = raw * (1.0 - (k + 2) * u) * lead_lo * lead_lo;
    const double ub = raw * sum_up * lead_hi * lead_hi;
    // T1: the pairs left out: outside the triangle (both indices >= 2), or
    // outside the tile's pair set when the pairs were chosen per tile
    double t1 = 0.0;
    const int8_t *lim = lims ? lims + ((int64_t)(j / 64) * tiles_m + i / 64) * D : nullptr;
    for (int a = lims ? 1 : 2; a <= D; ++a) {
      const int ea = slice_exp(eA, m, i, a, int8 != 0);
      if (ea == kZeroExp) break;  // later slices are zero too
      for (int b = lims ? lim[a - 1] + 1 : D + 2 - a; b <= D; ++b) {
        const int eb = slice_exp(eB, n, j, b, int8 != 0);
        if (eb == kZeroExp) break;
        t1 += pow2d(ea + eb);
      }
    }
    t1 *= (double)k;
    const double rA = remainder_bound(eA, m, i, D, rho, S, int8 != 0);
    const double rB = remainder_bound(eB, n, j, D, rho, S, int8 != 0);
    const double rs = rsA[i] * sum_up * lead_hi, cs = csB[j] * sum_up * lead_hi;
    const double t2 = rB * (rs + (double)k * rA);
    const double t3 = rA * cs;
    const double t4 = ldexp(ub, 4 - S * comps);
    const double beta = (t1 + t2 + t3 + t4) * (1.0 + ldexp(1.0, -40));
    cert[idx] = beta;
    cert[mn + idx] = lb;
    const double ratio = lb > 0.0 ? beta / lb : (beta > 0.0 ? __builtin_inf() : 0.0);
    const unsigned long long bits = (unsigned long long)__double_as_longlong(ratio);
    local = bits > local ? bits : local;
  }
  // one atomic per wavefront
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long o = __shfl_xor(local, off, 64);
    local = o > local ? o : local;
  }
  if (threadIdx.x % 64 == 0 && local != 0) atomicMax(worst, local);
}

// Pair set of one 64 x 64 tile of C from the data (one workgroup per tile).
// With D slices made, the computed C of a pair set P misses AB by at most
//   k sum_{(a, b) not in P} 2^(eA_a,i + eB_b,j) + T2 + T3 + T4
// per entry (the certificate's terms, T1 over the pairs left out).  Relative
// to the first slices, eA_a,i = eA_1,i + dA_a,i and eB_b,j = eB_1,j + dB_b,j,
// where the drops dA, dB (about -(a - 1) b bits for b-bit slices) hardly vary
// over a tile even when the rows' or columns' scales do.  With the tile's
// largest drops DA_a = max_i dA_a,i and DB_b = max_j dB_b,j, every entry
// meets 2^-t LB_ij once
//   sum_{(a, b) not in P} 2^(DA_a + DB_b)
//       <= min_ij (2^-t LB_ij - T2 - T3 - T4) / (k 2^(eA_1,i + eB_1,j)).
// P = {(a, b): DA_a + DB_b >= L} for the largest integer L that satisfies it:
// a staircase (the drops fall with a and with b), written as the count of b
// per a.  Entries with LB_ij = 0 are left out of the minimum: |A||B| is zero
// there, so every slice product, and C, is exactly zero.  A tile whose
// remainder and rounding terms alone exceed the bound somewhere takes every
// pair of nonzero slices (the certificate then reports the excess).
__global__ __launch_bounds__(kCertThreads) void k_tile_pairs(int m, int n, int k, int D, int rho, int S, int comps,
                                                             int t, const int *__restrict__ eA,
                                                             const int *__restrict__ eB,
                                                             const double *__restrict__ rsA,
                                                             const double *__restrict__ csB,
                                                             const double *__restrict__ raw, int tiles_m,
                                                             int8_t *__restrict__ lims) {
  __shared__ int sDA[kMaxPairLim], sDB[kMaxPairLim];
  __shared__ double s_min[kCertThreads / 64];
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int tid = threadIdx.x;
  const double u = ldexp(1.0, -52);
  const double sum_up = 1.0 + (k + 2) * u;
  const double lead_lo = 1.0 - ldexp(1.0, 2 - S), lead_hi = 1.0 + ldexp(1.0, 2 - S);
  // the tile's largest drops (kZeroExp for slices zero on the whole tile)
  if (tid < D) {
    int e = kZeroExp;
    for (int r = 0; r < 64; ++r) {
      const int i = tm * 64 + r;
      if (i >= m) break;
      const int e1 = eA[i], ea = eA[(int64_t)tid * m + i];
      if (e1 != kZeroExp && ea != kZeroExp) e = max(e, ea - e1);
    }
    sDA[tid] = e;
  } else if (tid >= 64 && tid < 64 + D) {
    int e = kZeroExp;
    for (int c = 0; c < 64; ++c) {
      const int j = tn * 64 + c;
      if (j >= n) break;
      const int f1 = eB[j], fb = eB[(int64_t)(tid - 64) * n + j];
      if (f1 != kZeroExp && fb != kZeroExp) e = max(e, fb - f1);
    }
    sDB[tid - 64] = e;
  }
  // the smallest relative slack over the tile's entries with a positive lower bound
  double slack = __builtin_inf();
  for (int e = tid; e < 64 * 64; e += kCertThreads) {
    const int i = tm * 64 + e % 64, j = tn * 64 + e / 64;
    if (i >= m || j >= n) continue;
    const double r = raw[i + (int64_t)j * m];
    const double lb = r * (1.0 - (k + 2) * u) * lead_lo * lead_lo;
    if (!(lb > 0.0)) continue;
    const double ub = r * sum_up * lead_hi * lead_hi;
    const double rA = remainder_bound(eA, m, i, D, rho, S, false);
    const double rB = remainder_bound(eB, n, j, D, rho, S, false);
    const double rs = rsA[i] * sum_up * lead_hi, cs = csB[j] * sum_up * lead_hi;
    const double rest = (rB * (rs + (double)k * rA) + rA * cs + ldexp(ub, 4 - S * comps)) * (1.0 + ldexp(1.0, -40));
    const double sl = ldexp(lb, -t) * (1.0 - ldexp(1.0, -40)) - rest;
    // lb > 0 makes both first slices nonzero; the scale 2^(eA_1,i + eB_1,j) is exact
    slack = fmin(slack, sl > 0.0 ? ldexp(sl, -(eA[i] + eB[j])) / (double)k : -1.0);
  }
  for (int off = 32; off >= 1; off >>= 1) slack = fmin(slack, __shfl_xor(slack, off, 64));
  if (tid % 64 == 0) s_min[tid / 64] = slack;
  __syncthreads();
  if (tid != 0) return;
  for (int w = 1; w < kCertThreads / 64; ++w) slack = fmin(slack, s_min[w]);
  int8_t *out = lims + ((int64_t)tn * tiles_m + tm) * D;
  // sums of finite drops span [lo, hi]
  int lo = INT_MAX, hi = INT_MIN;
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b)
      if (sDA[a] != kZeroExp && sDB[b] != kZeroExp) {
        lo = min(lo, sDA[a] + sDB[b]);
        hi = max(hi, sDA[a] + sDB[b]);
      }
  int L = INT_MIN;  // every pair of nonzero slices
  if (lo <= hi && slack > 0.0 && slack < __builtin_inf()) {
    // the left-out sum below threshold L against the budget, both scaled by 2^-eb
    const int eb = ilogb(slack);
    const double cap = ldexp(slack, -eb) * (1.0 - ldexp(1.0, -30));
    auto fits = [&](int thr) {
      double sum = 0.0;
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b)
          if (sDA[a] != kZeroExp && sDB[b] != kZeroExp && sDA[a] + sDB[b] < thr)
            sum += ldexp(1.0, sDA[a] + sDB[b] - eb);
      return sum <= cap;
    };
    // the largest L in [lo, hi + 1] that fits (L = lo leaves nothing out)
    int a0 = lo, a1 = hi + 1;
    if (fits(a1)) {
      L = a1;
    } else {
      while (a1 - a0 > 1) {
        const int mid = a0 + (a1 - a0) / 2;
        if (fits(mid))
          a0 = mid;
        else
          a1 = mid;
      }
      L = a0;
    }
  } else if (lo <= hi && slack == __builtin_inf()) {
    L = hi + 1;  // |A||B| is zero on the whole tile: C is zero without any pair
  }
  for (int a = 0; a < D; ++a) {
    int c = 0;
    if (sDA[a] != kZeroExp)
      while (c < D && sDB[c] != kZeroExp && (L == INT_MIN || sDA[a] + sDB[c] >= L)) ++c;
    out[a] = (int8_t)c;
  }
}

}  // namespace

hipError_t launch_tile_pairs(int m, int n, int k, int D, int rho, int S, int comps, int t, const int *eA,
                             const int *eB, const double *rs_a, const double *cs_b, const double *raw,
                             int64_t tiles_m, int64_t tiles_n, int8_t *lims, hipStream_t st) {
  if (D < 1 || D > kMaxPairLim) return hipErrorInvalidValue;
  if (tiles_m * tiles_n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_pairs, dim3((unsigned)(tiles_m * tiles_n)), dim3(kCertThreads), 0, st, m, n, k, D, rho, S,
                     comps, t, eA, eB, rs_a, cs_b, raw, (int)tiles_m, lims);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_abs_lead_product(const SplitOperand<T> &a, const SplitOperand<T> &b, int m, int n, double *raw,
                                   double *pack_a, double *pack_b, double *rs_a, double *cs_b, int layout,
                                   hipStream_t st) {
  const auto grid_of = [](int64_t work) { return (unsigned)std::min<int64_t>(ceil_div(work, kCertThreads), 8192); };
  hipLaunchKernelGGL((k_pack_abs_lead<T>), dim3(grid_of(a.nbp * a.kbp * 256)), dim3(kCertThreads), 0, st, a, pack_a);
  hipLaunchKernelGGL((k_pack_abs_lead<T>), dim3(grid_of(b.nbp * b.kbp * 256)), dim3(kCertThreads), 0, st, b, pack_b);
  hipLaunchKernelGGL((k_abs_row_sums<T>), dim3((unsigned)ceil_div(m, 64)), dim3(1024), 0, st, a, rs_a);
  hipLaunchKernelGGL((k_abs_sums<T>), dim3((unsigned)ceil_div(n, kCertThreads / 64)), dim3(kCertThreads), 0, st, b,
                     cs_b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // |A_0| |B_0| as one pair on the binary64 slice-product kernel, into two planes of raw
  return launch_gemm_plain<double, 2>(pack_a, pack_b, a.nbp, b.nbp, a.kbp, m, n, 1, raw, m, (int64_t)m * n, -1,
                                      nullptr, 0, layout, st);
}

template <typename T>
hipError_t launch_certify(const SplitOperand<T> &a, const SplitOperand<T> &b, int m, int n, int k, int D, int rho,
                          int comps, int int8, double *cert, double *worst, double *pack_a, double *pack_b,
                          double *rs_a, double *cs_b, int layout, hipStream_t st, const int8_t *lims,
                          bool raw_ready) {
  const int S = sizeof(T) == 8 ? 53 : 24;
  hipError_t e = launch_fill32(worst, 2, 0u, st);
  if (e != hipSuccess) return e;
  const auto grid_of = [](int64_t work) { return (unsigned)std::min<int64_t>(ceil_div(work, kCertThreads), 8192); };
  if (!raw_ready) {
    // |A_0| |B_0| into planes 0 and 1 of cert
    e = launch_abs_lead_product<T>(a, b, m, n, cert, pack_a, pack_b, rs_a, cs_b, layout, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_certify, dim3(grid_of((int64_t)m * n)), dim3(kCertThreads), 0, st, m, n, k, D, rho, S, comps,
                     int8, a.exps, b.exps, rs_a, cs_b, cert, reinterpret_cast<unsigned long long *>(worst), lims,
                     (int)(a.nbp / kTileBlocks));
  return hipGetLastError();
}

template hipError_t launch_certify<double>(const SplitOperand<double> &, const SplitOperand<double> &, int, int, int,
                                           int, int, int, int, double *, double *, double *, double *, double *,
                                           double *, int, hipStream_t, const int8_t *, bool);
template hipError_t launch_certify<float>(const SplitOperand<float> &, const SplitOperand<float> &, int, int, int, int,
                                          int, int, int, double *, double *, double *, double *, double *, double *,
                                          int, hipStream_t, const int8_t *, bool);
template hipError_t launch_abs_lead_product<double>(const SplitOperand<double> &, const SplitOperand<double> &, int,
                                                    int, double *, double *, double *, double *, double *, int,
                                                    hipStream_t);
template hipError_t launch_abs_lead_product<float>(const SplitOperand<float> &, const SplitOperand<float> &, int, int,
                                                   double *, double *, double *, double *, double *, int,
                                                   hipStream_t);

}  // namespace mp
