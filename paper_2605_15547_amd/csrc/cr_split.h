// cr_split.h -- float-float ("double-float", split binary32) arithmetic and
// the final rounding of the binary32-only kernels (device).
//
// The paper's binary32 kernels compute internally in binary64 (Sec. II-A) and
// note that this is costly where binary64 runs slowly (its second GPU,
// Sec. III-C).  The split path computes with binary32 operations only: a value
// is an unevaluated pair hi + lo of binary32 numbers (about 48 significant
// bits), built from the exact error-free transformations (Knuth's TwoSum,
// Dekker's Fast2Sum, and TwoProd through a fused multiply-add).  The code is
// compiled without contraction (-ffp-contract=off): every fmaf below is
// written out and no other operation is fused, so each transformation is
// exact as stated.
#pragma once
#include "cr_dd.h"

namespace cr {

struct ff {
  float hi, lo;
};

// s + e = a + b exactly
__device__ __forceinline__ ff ff_two_sum(float a, float b) {
  float s = a + b;
  float bb = s - a;
  float e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

// s + e = a + b exactly, provided a == 0 or exponent(a) >= exponent(b)
__device__ __forceinline__ ff ff_fast_two_sum(float a, float b) {
  float s = a + b;
  return {s, b - (s - a)};
}

// p + e = a b exactly (barring underflow)
__device__ __forceinline__ ff ff_two_prod(float a, float b) {
  float p = a * b;
  return {p, fmaf(a, b, -p)};
}

// 2^e as a binary32 number, -149 <= e <= 127
__device__ __forceinline__ float pow2f_i(int e) {
  return e >= -126 ? __uint_as_float((unsigned)(e + 127) << 23)
                   : __uint_as_float(1u << (e + 149));
}

// a / b for float-float a, b (b != 0): quotient estimate from the hardware
// reciprocal, float-float residual, two corrections (relative error ~2^-46)
__device__ __forceinline__ ff ff_div(ff a, ff b) {
  float ic = __builtin_amdgcn_rcpf(b.hi);
  float q1 = a.hi * ic;
  ff p = ff_two_prod(q1, b.hi);
  float rem = ((a.hi - p.hi) - p.lo) + fmaf(-q1, b.lo, a.lo);
  float q2 = rem * ic;
  q2 = fmaf(fmaf(-q2, b.hi, rem), ic, q2);
  return ff_fast_two_sum(q1, q2);
}

// Final rounding of a split result.  The exact value lies within err of
// h + l (h, l binary32, |l| small against h; err >= 0 covers every error,
// including the two roundings below).  RN_32 is monotone, so when
// RN(h + RN(l - err)) == RN(h + RN(l + err)) every real in between -- the
// exact value included -- rounds to that same float.  The result must be
// normal (or exactly representable): callers scale by powers of two only
// after this step, or use round_split_q for the subnormal range.
__device__ __forceinline__ float round_split(float h, float l, float err, bool& ok) {
  float a = h + (l - err);
  float b = h + (l + err);
  ok = a == b;
  return b;
}

// Rounding on the fixed quantum of the subnormal range: the exact value is
// (h + l) * 2^-149 (h + l in [0, 2^24), l not necessarily below ulp(h))
// within err * 2^-149, err covering the rounding of f below (|f| < 4: 2^-22).
// Returns the correctly rounded multiple of 2^-149; ok = false when the value
// lies within err of a half-integer.
__device__ __forceinline__ float round_split_q(float h, float l, float err, bool& ok) {
  float n = rintf(h);
  float f = (h - n) + l;  // h - n is exact; one rounding
  float g = rintf(f);
  float d = f - g;        // exact, |d| <= 1/2
  ok = fabsf(d) < 0.5f - err;
  return (n + g) * 0x1p-149f;  // n + g < 2^24: exact
}

}  // namespace cr
