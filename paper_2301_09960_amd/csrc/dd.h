// Double-double (DD) scalar arithmetic for the LU application (Section 4.6
// factorizes DD matrices with the slice-product GEMM doing the Schur updates).
// A DD number is hi + lo with |lo| <= ulp(hi) / 2.  The operations are the
// classical ones built from the error-free transformations: TwoSum
// (mp_device.h), the exact product TwoProd via a fused multiply-add, and a
// normalizing FastTwoSum.  Must be compiled with -ffp-contract=off (only the
// explicit fma below is fused).
#pragma once

#include <hip/hip_runtime.h>

#include "mp_device.h"

namespace mp {

struct dd {
  double hi, lo;
};

// s + e == a + b exactly, given |a| >= |b| or a == 0.
__device__ __forceinline__ double fast_two_sum(double a, double b, double &e) {
  const double s = a + b;
  e = b - (s - a);
  return s;
}

// p + e == a * b exactly (barring underflow).
__device__ __forceinline__ double two_prod(double a, double b, double &e) {
  const double p = a * b;
  e = fma(a, b, -p);
  return p;
}

__device__ __forceinline__ dd dd_make(double hi, double lo) { return dd{hi, lo}; }
__device__ __forceinline__ dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }

// a + b: both parts added with TwoSum, the errors folded in, renormalized twice.
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  double e, f;
  double s = two_sum(a.hi, b.hi, e);
  const double t = two_sum(a.lo, b.lo, f);
  e += t;
  s = fast_two_sum(s, e, e);
  e += f;
  s = fast_two_sum(s, e, e);
  return dd{s, e};
}

__device__ __forceinline__ dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

// a * b: the exact product of the high parts plus the cross terms.
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  double e;
  const double p = two_prod(a.hi, b.hi, e);
  e += a.hi * b.lo + a.lo * b.hi;
  double lo;
  const double hi = fast_two_sum(p, e, lo);
  return dd{hi, lo};
}

// a / b: three quotient digits, each from the remainder of the previous ones.
__device__ __forceinline__ dd dd_div(dd a, dd b) {
  const double q1 = a.hi / b.hi;
  dd r = dd_sub(a, dd_mul(dd{q1, 0.0}, b));
  const double q2 = r.hi / b.hi;
  r = dd_sub(r, dd_mul(dd{q2, 0.0}, b));
  const double q3 = r.hi / b.hi;
  double lo;
  const double hi = fast_two_sum(q1, q2, lo);
  return dd_add(dd{hi, lo}, dd{q3, 0.0});
}

}  // namespace mp
