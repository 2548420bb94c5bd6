// Device building blocks for the Ozaki-scheme kernels on gfx950.
//
// Error-free transformations (Knuth's TwoSum), the renormalization used for
// the split residual and the final result, and the packed slice layout that
// the split kernels write and the matrix-core kernels read.
//
// All of this must be compiled with -ffp-contract=off: a contracted
// multiply-add or a reassociated sum would break the error-free steps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mp {

// ---------------------------------------------------------------------------
// Error-free transformations.
// ---------------------------------------------------------------------------

// s + e == a + b exactly, s = fl(a + b); no precondition on the magnitudes.
template <typename T>
__device__ __forceinline__ T two_sum(T a, T b, T &e) {
  T s = a + b;
  T bb = s - a;
  e = (a - (s - bb)) + (b - bb);
  return s;
}

// Renormalization of an N-term expansion, in place.  A bottom-up TwoSum pass
// gathers the sum into the top term and leaves N - 1 error terms; a top-down
// TwoSum pass then emits a term each time the running error is nonzero,
// continuing with that error (zeros are padded at the end).  Only TwoSum is
// used, so the value of the expansion is unchanged, and the first term is
// nonzero whenever the value is.  Fully unrolled: the compaction is done with
// selects so that the term index stays a compile-time constant.
template <typename T, int N>
__device__ __forceinline__ void renorm(T (&x)[N]) {
  T e[N];
  T s = x[N - 1];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) s = two_sum(x[i], s, e[i + 1]);
  T out[N];
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = T(0);
  int w = 0;
  T t = s;
#pragma unroll
  for (int i = 1; i < N; ++i) {
    T err;
    T nt = two_sum(t, e[i], err);
    const bool emit = err != T(0);
    // before step i at most i - 1 terms were emitted, so w < i
#pragma unroll
    for (int q = 0; q < i; ++q)
      if (emit && q == w) out[q] = nt;
    t = emit ? err : nt;
    w += emit ? 1 : 0;
  }
#pragma unroll
  for (int q = 0; q < N; ++q)
    if (q == w) out[q] = t;
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = out[i];
}

// Adds an exact term x into an (N)-term accumulator: TwoSum down the chain of
// terms; the last error (below half an ulp of the last term) is dropped.
template <typename T, int N>
__device__ __forceinline__ void acc_add(T (&acc)[N], T x) {
  T s = x;
#pragma unroll
  for (int r = 0; r < N; ++r) acc[r] = two_sum(acc[r], s, s);
}

// ---------------------------------------------------------------------------
// ceil(log2 mu) for finite mu > 0 and the power of two 2^e.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ceil_log2(double mu) {
  int ex;
  double f = frexp(mu, &ex);  // mu = f 2^ex, f in [0.5, 1)
  return f == 0.5 ? ex - 1 : ex;
}
__device__ __forceinline__ int ceil_log2(float mu) {
  int ex;
  float f = frexpf(mu, &ex);
  return f == 0.5f ? ex - 1 : ex;
}
__device__ __forceinline__ double pow2(int e, double) { return ldexp(1.0, e); }
__device__ __forceinline__ float pow2(int e, float) { return ldexpf(1.0f, e); }

// Bit pattern of |x| as an unsigned integer: for nonnegative IEEE values the
// integer order is the numeric order, so maxima can use integer atomics.
__device__ __forceinline__ unsigned long long abs_bits(double x) {
  return (unsigned long long)__double_as_longlong(fabs(x));
}
__device__ __forceinline__ unsigned int abs_bits(float x) { return (unsigned int)__float_as_uint(fabsf(x)); }
__device__ __forceinline__ double from_bits(unsigned long long b, double) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ float from_bits(unsigned int b, float) { return __uint_as_float(b); }

template <typename T> struct bits_of;
template <> struct bits_of<double> { using type = unsigned long long; };
template <> struct bits_of<float> { using type = unsigned int; };

}  // namespace mp
