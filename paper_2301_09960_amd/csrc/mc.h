// Multi-component scalar arithmetic for the TD LU (Section 4.6 factorizes TD
// matrices as well as DD ones) and the simple in-format matrix multiplication
// of TS, TD and QD (Section 4.4).  A value is C components of type T (binary64,
// or binary32 for TS), largest first.  Each operation gathers its terms (exact ones from TwoSum / TwoProd,
// and for a product a plain tail at the lowest order kept), sorts them by
// decreasing magnitude, renormalizes them with `renorm` (mp_device.h:
// only TwoSum, so the sum is unchanged) and keeps the leading C components.
// Division takes C quotient digits, each from the remainder of the previous
// ones (the remainder formed in a single renormalization).  Must be
// compiled with -ffp-contract=off (only the explicit fma of TwoProd is fused).
#pragma once

#include <hip/hip_runtime.h>

#include "mp_device.h"
#include "sortnet.h"

namespace mp {

template <int C, typename T = double>
struct mc {
  T x[C];
};

// Sort by decreasing magnitude with the comparator network of sortnet.h
// (fully unrolled: compile-time indices, selects only).
template <int N, typename T>
__device__ __forceinline__ void sort_by_magnitude(T (&t)[N]) {
  constexpr SortNet<N> net{};
#pragma unroll
  for (int c = 0; c < net.count; ++c) {
    const int lo = net.lo[c], hi = net.hi[c];
    const T a = t[lo], b = t[hi];
    const bool swap = fabs(b) > fabs(a);
    t[lo] = swap ? b : a;
    t[hi] = swap ? a : b;
  }
}

// The leading C components of the renormalized sum of N exact terms.
template <int C, int N, typename T>
__device__ __forceinline__ mc<C, T> mc_from_terms(T (&t)[N]) {
  sort_by_magnitude<N>(t);
  renorm<T, N>(t);
  mc<C, T> r;
#pragma unroll
  for (int i = 0; i < C; ++i) r.x[i] = t[i];
  return r;
}

template <int C, typename T>
__device__ __forceinline__ mc<C, T> mc_neg(mc<C, T> a) {
#pragma unroll
  for (int i = 0; i < C; ++i) a.x[i] = -a.x[i];
  return a;
}

template <int C, typename T>
__device__ __forceinline__ mc<C, T> mc_add(const mc<C, T> &a, const mc<C, T> &b) {
  T t[2 * C];
#pragma unroll
  for (int i = 0; i < C; ++i) {
    t[2 * i] = a.x[i];
    t[2 * i + 1] = b.x[i];
  }
  return mc_from_terms<C, 2 * C>(t);
}

template <int C, typename T>
__device__ __forceinline__ mc<C, T> mc_sub(const mc<C, T> &a, const mc<C, T> &b) {
  return mc_add<C>(a, mc_neg<C>(b));
}

// The terms of a b, from the products a_i b_j with i + j < C.  Below order
// C - 2 they are exact (TwoProd); on order C - 2 the product is kept and its
// error joins a plain binary64 tail with the products of order C - 1, which
// lie about 2^-106 |ab| below the lead (for C = 3), so the tail's rounding is
// near 2^-159 |ab|.  The terms beyond are below the precision kept.  C = 3
// gives 5 terms instead of the 9 of an exact gathering.
template <int C>
constexpr int mul_terms() {
  return 2 * ((C - 2) * (C - 1) / 2) + (C - 1) + 1;
}

template <int C, typename T>
__device__ __forceinline__ void gather_mul_terms(const mc<C, T> &a, const mc<C, T> &b, T (&t)[mul_terms<C>()]) {
  T tail = T(0);
  int w = 0;
#pragma unroll
  for (int i = 0; i < C; ++i)
#pragma unroll
    for (int j = 0; j + i < C; ++j) {
      const T p = a.x[i] * b.x[j];
      if (i + j < C - 2) {
        t[w++] = p;
        t[w++] = fma(a.x[i], b.x[j], -p);
      } else if (i + j == C - 2) {
        t[w++] = p;
        tail += fma(a.x[i], b.x[j], -p);
      } else {
        tail += p;
      }
    }
  t[w] = tail;
}

template <int C, typename T>
__device__ __forceinline__ mc<C, T> mc_mul(const mc<C, T> &a, const mc<C, T> &b) {
  T t[mul_terms<C>()];
  gather_mul_terms<C>(a, b, t);
  return mc_from_terms<C, mul_terms<C>()>(t);
}

// s - a b in one renormalization: the terms of s and of -(a b) as above.
template <int C, typename T>
__device__ __forceinline__ mc<C, T> mc_fms(const mc<C, T> &s, const mc<C, T> &a, const mc<C, T> &b) {
  constexpr int M = mul_terms<C>();
  T p[M];
  gather_mul_terms<C>(a, b, p);
  T t[C + M];
#pragma unroll
  for (int i = 0; i < C; ++i) t[i] = s.x[i];
#pragma unroll
  for (int i = 0; i < M; ++i) t[C + i] = -p[i];
  return mc_from_terms<C, C + M>(t);
}

// s + a b in one renormalization: the terms of s and of a b as above.
template <int C, typename T>
__device__ __forceinline__ mc<C, T> mc_fma(const mc<C, T> &s, const mc<C, T> &a, const mc<C, T> &b) {
  constexpr int M = mul_terms<C>();
  T t[C + M];
#pragma unroll
  for (int i = 0; i < C; ++i) t[i] = s.x[i];
  T p[M];
  gather_mul_terms<C>(a, b, p);
#pragma unroll
  for (int i = 0; i < M; ++i) t[C + i] = p[i];
  return mc_from_terms<C, C + M>(t);
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

// C quotient digits: after them the remainder is near 2^(-53 C) |a|, so the
// next digit would only move the result by about the rounding of its last
// component.  For C = 3 the relative error stays below 2^-155 (a host test
// checks it against exact rationals; 2^-158.7 at worst on random operands,
// against about 2^-105 with two digits).
template <int C>
__device__ __forceinline__ mc<C> mc_div(const mc<C> &a, const mc<C> &b) {
  double q[C];
  mc<C> r = a;
#pragma unroll
  for (int d = 0; d < C; ++d) {
    q[d] = r.x[0] / b.x[0];
    if (d < C - 1) r = mc_sub_scaled<C>(r, q[d], b);
  }
  return mc_from_terms<C, C>(q);
}

}  // namespace mp
