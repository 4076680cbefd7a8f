// cr_dd.h -- error-free transformations and double-double arithmetic (device).
//
// The kernels are compiled with -ffp-contract=off so that no a*b+c is fused
// behind our back; every fused multiply-add below is an explicit fma().
// Algorithms: Knuth's TwoSum, Dekker's Fast2Sum, the FMA-based TwoProd, and
// the double-word additions/multiplications analysed by Joldes, Muller and
// Popescu (ACM TOMS 44(4), 2018): relative errors below 3u^2 (add) and
// 5u^2 (mul) with u = 2^-53.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cr {

struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

// requires |a| >= |b| (or a == 0)
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
  double s = a + b;
  double e = b - (s - a);
  return {s, e};
}

__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  return {p, fma(a, b, -p)};
}

// double-word + double
__device__ __forceinline__ dd dd_add_d(dd x, double y) {
  dd s = two_sum(x.hi, y);
  double v = x.lo + s.lo;
  return fast_two_sum(s.hi, v);
}

// double-word + double-word (accurate version, relative error <= 3u^2)
__device__ __forceinline__ dd dd_add(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  dd t = two_sum(x.lo, y.lo);
  double c = s.lo + t.hi;
  dd v = fast_two_sum(s.hi, c);
  double w = t.lo + v.lo;
  return fast_two_sum(v.hi, w);
}

// double-word + double-word when |x.hi| >= |y.hi| (or x.hi == 0) and the sum
// does not cancel: Fast2Sum of the high parts, the low parts added once
// (relative error a few u^2; 8 operations instead of 20)
__device__ __forceinline__ dd dd_add_ord(dd x, dd y) {
  dd s = fast_two_sum(x.hi, y.hi);
  return fast_two_sum(s.hi, s.lo + (x.lo + y.lo));
}

// double-word + double-word without an ordering condition, for sums that do
// not cancel: TwoSum of the high parts, the low parts added once
__device__ __forceinline__ dd dd_add_nc(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  return fast_two_sum(s.hi, s.lo + (x.lo + y.lo));
}

// double-word * double (relative error <= 2u^2)
__device__ __forceinline__ dd dd_mul_d(dd x, double y) {
  dd c = two_prod(x.hi, y);
  double cl = fma(x.lo, y, c.lo);
  return fast_two_sum(c.hi, cl);
}

// double-word * double-word (relative error <= 5u^2)
__device__ __forceinline__ dd dd_mul(dd x, dd y) {
  dd c = two_prod(x.hi, y.hi);
  double tl = x.hi * y.lo;
  double cl = fma(x.lo, y.hi, tl);
  cl = c.lo + cl;
  return fast_two_sum(c.hi, cl);
}

__device__ __forceinline__ dd dd_neg(dd x) { return {-x.hi, -x.lo}; }

__device__ __forceinline__ dd dd_mul_pow2(dd x, double s) { return {x.hi * s, x.lo * s}; }

// 2^m as a double for -1022 <= m <= 1023
__device__ __forceinline__ double pow2i(int m) {
  return __longlong_as_double((long long)(m + 1023) << 52);
}

__device__ __forceinline__ uint32_t f32_bits(float x) { return __float_as_uint(x); }
__device__ __forceinline__ float bits_f32(uint32_t b) { return __uint_as_float(b); }
// a / b from the hardware reciprocal and two corrections by exact residuals,
// each of which squares the relative error of the estimate: the quotient within
// 2^-52 |a/b| for b and a/b in the normal range.  Cheaper than the IEEE
// division sequence where the fast paths' error budgets allow 2^-52.
__device__ __forceinline__ double div_fast(double a, double b) {
  const double ib = __builtin_amdgcn_rcp(b);
  double q = a * ib;
  q = fma(fma(-q, b, a), ib, q);
  return fma(fma(-q, b, a), ib, q);
}

// x quieted (payload and sign kept) when x is a NaN, else v -- an integer
// select: as a float conditional the compiler branches around the bit operation
__device__ __forceinline__ float nan_or(float x, float v) {
  const uint32_t q = f32_bits(x) | 0x00400000u;
  return bits_f32(x != x ? q : f32_bits(v));
}

}  // namespace cr
