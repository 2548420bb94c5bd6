// Multi-component scalar arithmetic for the TD LU (Section 4.6 factorizes TD
// matrices as well as DD ones).  A value is C binary64 components, largest
// first.  Each operation gathers its exact terms (TwoSum / TwoProd), sorts
// them by decreasing magnitude, renormalizes them with `renorm` (mp_device.h:
// only TwoSum, so the sum is unchanged) and keeps the leading C components.
// Division takes C + 1 quotient digits, each from the remainder of the
// previous ones (the remainder formed in a single renormalization).  Must be
// compiled with -ffp-contract=off (only the explicit fma of TwoProd is fused).
#pragma once

#include <hip/hip_runtime.h>

#include "mp_device.h"

namespace mp {

template <int C>
struct mc {
  double x[C];
};

// Insertion sort by decreasing magnitude (fully unrolled, selects only).
template <int N>
__device__ __forceinline__ void sort_by_magnitude(double (&t)[N]) {
#pragma unroll
  for (int i = 1; i < N; ++i)
#pragma unroll
    for (int j = i; j > 0; --j) {
      const double a = t[j - 1], b = t[j];
      const bool swap = fabs(b) > fabs(a);
      t[j - 1] = swap ? b : a;
      t[j] = swap ? a : b;
    }
}

// The leading C components of the renormalized sum of N exact terms.
template <int C, int N>
__device__ __forceinline__ mc<C> mc_from_terms(double (&t)[N]) {
  sort_by_magnitude<N>(t);
  renorm<double, N>(t);
  mc<C> r;
#pragma unroll
  for (int i = 0; i < C; ++i) r.x[i] = t[i];
  return r;
}

template <int C>
__device__ __forceinline__ mc<C> mc_neg(mc<C> a) {
#pragma unroll
  for (int i = 0; i < C; ++i) a.x[i] = -a.x[i];
  return a;
}

template <int C>
__device__ __forceinline__ mc<C> mc_add(const mc<C> &a, const mc<C> &b) {
  double t[2 * C];
#pragma unroll
  for (int i = 0; i < C; ++i) {
    t[2 * i] = a.x[i];
    t[2 * i + 1] = b.x[i];
  }
  return mc_from_terms<C, 2 * C>(t);
}

template <int C>
__device__ __forceinline__ mc<C> mc_sub(const mc<C> &a, const mc<C> &b) {
  return mc_add<C>(a, mc_neg<C>(b));
}

// Products a_i b_j with i + j < C: exact (TwoProd) below the last order, plain
// on it; the terms beyond are below the precision kept.
template <int C>
__device__ __forceinline__ mc<C> mc_mul(const mc<C> &a, const mc<C> &b) {
  constexpr int kExact = (C - 1) * C / 2;  // pairs with i + j < C - 1
  constexpr int kPlain = C;                // pairs with i + j == C - 1
  double t[2 * kExact + kPlain];
  int w = 0;
#pragma unroll
  for (int i = 0; i < C; ++i)
#pragma unroll
    for (int j = 0; j + i < C; ++j) {
      if (i + j < C - 1) {
        const double p = a.x[i] * b.x[j];
        t[w++] = p;
        t[w++] = fma(a.x[i], b.x[j], -p);
      } else {
        t[w++] = a.x[i] * b.x[j];
      }
    }
  return mc_from_terms<C, 2 * kExact + kPlain>(t);
}

// r - q b for a binary64 q, in one renormalization: the terms of r, and q b_i
// exact (TwoProd) below the last order, plain on it.
template <int C>
__device__ __forceinline__ mc<C> mc_sub_scaled(const mc<C> &r, double q, const mc<C> &b) {
  double t[C + 2 * (C - 1) + 1];
  int w = 0;
#pragma unroll
  for (int i = 0; i < C; ++i) t[w++] = r.x[i];
#pragma unroll
  for (int i = 0; i < C - 1; ++i) {
    const double p = q * b.x[i];
    t[w++] = -p;
    t[w++] = -fma(q, b.x[i], -p);
  }
  t[w++] = -(q * b.x[C - 1]);
  return mc_from_terms<C, C + 2 * (C - 1) + 1>(t);
}

template <int C>
__device__ __forceinline__ mc<C> mc_div(const mc<C> &a, const mc<C> &b) {
  double q[C + 1];
  mc<C> r = a;
#pragma unroll
  for (int d = 0; d <= C; ++d) {
    q[d] = r.x[0] / b.x[0];
    if (d < C) r = mc_sub_scaled<C>(r, q[d], b);
  }
  return mc_from_terms<C, C + 1>(q);
}

}  // namespace mp
