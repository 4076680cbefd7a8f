// cr_tf.h -- triple-float arithmetic and its final rounding (device), for the
// accurate step of the binary32-only implementation.
//
// The paper proposes binary32 arithmetic for GPUs with slow binary64 (Sec.
// II-A, IV).  The binary32-only kernels evaluate in float-float (cr_split.h,
// about 48 bits) and certify most results; the rare lanes that fail their
// rounding test need about 64 to 70 bits (the hardest binary32 inputs of the
// exhaustive scan lie 2^-56 .. 2^-66.8 from a rounding boundary, relative).
// A triple-float h + m + l carries about 70: every operation below is built
// from the error-free transformations of cr_split.h (TwoSum, Fast2Sum,
// TwoProd through fmaf), renormalised so that |m| <= ulp(h)/2 and
// |l| <= ulp(m)/2 (the construction of the triple-double arithmetic of
// cr_td.h, in binary32: Lauter, "Basic building blocks for a triple-double
// intermediate format", INRIA RR-5702, 2005).  Relative errors: tf_add a few
// 2^-70 of the result when it does not cancel, tf_mul below 2^-68.
// Components must stay in the normal binary32 range: callers keep values
// near 1 and scale by powers of two only after rounding.
#pragma once
#include "cr_split.h"

namespace cr {

struct tf {
  float h, m, l;
};

__device__ __forceinline__ tf tf_renorm(float a, float b, float c) {
  ff s = ff_two_sum(b, c);
  ff t = ff_two_sum(a, s.hi);
  ff u = ff_two_sum(t.lo, s.lo);
  ff v = ff_two_sum(t.hi, u.hi);
  ff w = ff_two_sum(v.lo, u.lo);
  return {v.hi, w.hi, w.lo};
}

// The same for |b|, |c| below 2^-20 |a| (or a = 0), as in a product whose
// leading part is a: b + c by TwoSum, a plus that sum's high part by Fast2Sum
// (exact: a's exponent is not below it), the two low parts by TwoSum.  Exact,
// and normalised as tf_renorm's result, in three transformations instead of
// five.
__device__ __forceinline__ tf tf_renorm_ord(float a, float b, float c) {
  ff s = ff_two_sum(b, c);
  ff t = ff_fast_two_sum(a, s.hi);
  ff u = ff_two_sum(t.lo, s.lo);
  return {t.hi, u.hi, u.lo};
}

__device__ __forceinline__ tf tf_from(float a) { return {a, 0.0f, 0.0f}; }
__device__ __forceinline__ tf tf_from_ff(ff a) { return {a.hi, a.lo, 0.0f}; }
__device__ __forceinline__ tf tf_neg(tf a) { return {-a.h, -a.m, -a.l}; }
// a * 2^k for a power of two s = 2^k (exact while the components stay normal)
__device__ __forceinline__ tf tf_scale(tf a, float s) { return {a.h * s, a.m * s, a.l * s}; }
__device__ __forceinline__ tf tf_ld(float4 v) { return {v.x, v.y, v.z}; }

__device__ __forceinline__ tf tf_add(tf x, tf y) {
  ff s0 = ff_two_sum(x.h, y.h);
  ff s1 = ff_two_sum(x.m, y.m);
  ff s2 = ff_two_sum(x.l, y.l);
  ff t1 = ff_two_sum(s0.lo, s1.hi);
  float t2 = (s1.lo + s2.hi) + (s2.lo + t1.lo);
  return tf_renorm(s0.hi, t1.hi, t2);
}

// x + y where y cannot cancel x: |y| <= |x|/2, or x = 0 (then the sum is y
// itself).  The leading parts add by Fast2Sum (x's exponent is not below y's)
// and the renormalisation needs only the ordered form; one rounding, of the
// lowest parts, as in tf_add.
__device__ __forceinline__ tf tf_add_ord(tf x, tf y) {
  ff s0 = ff_fast_two_sum(x.h, y.h);
  ff s1 = ff_two_sum(x.m, y.m);
  ff t1 = ff_two_sum(s0.lo, s1.hi);
  return tf_renorm_ord(s0.hi, t1.hi, (s1.lo + (x.l + y.l)) + t1.lo);
}

// x + y for a binary32 y: one rounding, below 2^-71 (|x| + |y|)
__device__ __forceinline__ tf tf_add_f(tf x, float y) {
  ff s0 = ff_two_sum(y, x.h);
  ff t1 = ff_two_sum(s0.lo, x.m);
  return tf_renorm(s0.hi, t1.hi, x.l + t1.lo);
}

// x + y for a float-float y
__device__ __forceinline__ tf tf_add_ff(tf x, ff y) {
  ff s0 = ff_two_sum(x.h, y.hi);
  ff s1 = ff_two_sum(x.m, y.lo);
  ff t1 = ff_two_sum(s0.lo, s1.hi);
  return tf_renorm(s0.hi, t1.hi, (s1.lo + x.l) + t1.lo);
}

__device__ __forceinline__ tf tf_mul(tf x, tf y) {
  ff p00 = ff_two_prod(x.h, y.h);
  ff p01 = ff_two_prod(x.h, y.m);
  ff p10 = ff_two_prod(x.m, y.h);
  float low = fmaf(x.h, y.l, fmaf(x.m, y.m, x.l * y.h)) + (p01.lo + p10.lo);
  ff m1 = ff_two_sum(p01.hi, p10.hi);
  ff m2 = ff_two_sum(p00.lo, m1.hi);
  return tf_renorm_ord(p00.hi, m2.hi, (m1.lo + m2.lo) + low);
}

__device__ __forceinline__ tf tf_mul_f(tf x, float d) {
  ff p0 = ff_two_prod(x.h, d);
  ff p1 = ff_two_prod(x.m, d);
  ff m2 = ff_two_sum(p0.lo, p1.hi);
  return tf_renorm_ord(p0.hi, m2.hi, fmaf(x.l, d, p1.lo + m2.lo));
}

// a / b: three quotient digits from the hardware reciprocal, each followed by
// an exact-product residual update (the residual is carried in triple-float)
__device__ __forceinline__ tf tf_div(tf a, tf b) {
  const float ic = __builtin_amdgcn_rcpf(b.h);
  float q1 = a.h * ic;
  q1 = fmaf(fmaf(-q1, b.h, a.h), ic, q1);
  tf r = tf_add(a, tf_neg(tf_mul_f(b, q1)));
  float q2 = r.h * ic;
  q2 = fmaf(fmaf(-q2, b.h, r.h), ic, q2);
  r = tf_add(r, tf_neg(tf_mul_f(b, q2)));
  float q3 = r.h * ic;
  return tf_renorm(q1, q2, q3);
}

// ---------------------------------------------------------------- rounding
// RN_32(h + t) for a finite binary32 h and a tail t = m + l with |t| about
// ulp(h) or less, given an absolute error bound e on h + t: the tail is
// compared with half the spacing of the binary32 numbers on its side of h
// (a quarter of ulp(h) below a power of two above the subnormal range; the
// spacing is 2^-149 throughout the subnormal range).  For |h| < 2^-100 the
// tail and the bound are scaled by 2^64 first (exact), so that these
// half-spacings do not underflow.  ok = false when a rounding boundary lies
// within e.
__device__ __forceinline__ float round32_tail(float h, float m, float l, float e, bool& ok) {
  const float sc = fabsf(h) < 0x1p-100f ? 0x1p64f : 1.0f;
  ff t = ff_two_sum(m * sc, l * sc);
  const uint32_t hb = __float_as_uint(h);
  const uint32_t ef = hb & 0x7f800000u;
  const float U = __uint_as_float(ef > 0x00800000u ? ef : 0x00800000u) * (0x1p-23f * sc);  // ulp(h)
  const bool down = (t.hi < 0.0f) != (h < 0.0f);
  const bool pow2 = (hb & 0x007fffffu) == 0 && ef > 0x00800000u;
  const float half = (down && pow2) ? 0.25f * U : 0.5f * U;
  const float at = fabsf(t.hi), atl = (t.hi < 0.0f) ? -t.lo : t.lo;
  ok = true;
  if (at < 0.5f * half) return h;
  const float d = (at - half) + atl;  // at - half is exact (Sterbenz)
  if (fabsf(d) <= e * sc) ok = false;
  if (d > 0.0f) return __uint_as_float(down ? hb - 1 : hb + 1);
  return h;
}

// Relative form: the error bound is erel |h|.
__device__ __forceinline__ float round32_tf(tf y, float erel, bool& ok) {
  return round32_tail(y.h, y.m, y.l, fabsf(y.h) * erel, ok);
}

// Rounding on the fixed quantum of the subnormal range: the exact value is
// v 2^-149 with v = h + m + l in [0, 2^24) known within e.  Returns the
// nearest multiple of 2^-149; ok = false when v lies within e of a
// half-integer.  The fractional part a + lo is kept in two pieces: near a
// half-integer a is +-1/2 or close to it, 1/2 - |a| is exact and the distance
// to the boundary keeps its relative accuracy.
__device__ __forceinline__ float round32_tf_q(tf v, float e, bool& ok) {
  const float n = rintf(v.h);
  const ff s = ff_two_sum(v.h - n, v.m);  // v.h - n is exact
  float g = rintf(s.hi);
  float a = s.hi - g;                     // exact, |a| <= 1/2
  const float lo = s.lo + v.l;            // far below ulp(a) unless a = 0
  if (a == 0.5f && lo > 0.0f) {
    g += 1.0f;
    a = -0.5f;
  } else if (a == -0.5f && lo < 0.0f) {
    g -= 1.0f;
    a = 0.5f;
  }
  const float d = (0.5f - fabsf(a)) - (a < 0.0f ? -lo : lo);  // distance to +-1/2
  ok = d > e;
  return (n + g) * 0x1p-149f;  // n + g <= 2^24: exact
}

}  // namespace cr
