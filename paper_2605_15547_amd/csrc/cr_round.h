// cr_round.h -- final correct rounding of binary32 results (device).
//
// The paper's CPU kernels compute in binary64 and finish with round-to-zero
// plus a sticky bit before the conversion to binary32 (Sec. II-A, Fig. 1), and
// their FP64 functions pair an accurate main path with a correct-rounding test
// and a slower path for the lanes that fail it (Sec. II-B).  On the GPU there
// is no static rounding, so both ideas are expressed with round-to-nearest:
//
//  * fast path: the approximation yh (binary64) is within E ulps of f(x).
//    RN_f32 is monotone, so if RN_f32(yh - E ulp) == RN_f32(yh + E ulp) every
//    real in between -- f(x) included -- rounds to that same float.
//  * accurate path: a double-double (h, l) within a relative bound drel of
//    f(x).  Both ends of the enclosure are formed as round-to-odd binary64
//    numbers (truncate, then force the last bit to 1 if inexact); converting a
//    round-to-odd value with >= 2 extra bits to binary32 gives the correctly
//    rounded binary32 value of the exact number (Boldo and Melquiond,
//    "Emulation of FMA and correctly rounded sums: proved algorithms using
//    rounding to odd", IEEE TC 57(4), 2008).  Equal ends => correct result.
#pragma once
#include "cr_dd.h"

namespace cr {

// result of an out-of-line accurate path: the rounded value and whether its
// rounding was certified (returned in registers)
struct AccResult {
  float r;
  int ok;
};

// ulp of |y| in binary64 (y normal, nonzero): 2^(exponent(y) - 52)
__device__ __forceinline__ double ulp53(double y) {
  uint32_t hi = (uint32_t)__double2hiint(y) & 0x7ff00000u;
  return __hiloint2double((int)hi, 0) * 0x1p-52;
}

// 2^(exponent(y) + k) for normal y and a small k (exponent field arithmetic;
// the result must stay normal, which holds for every use here)
__device__ __forceinline__ double pow2_of_exp(double y, int k) {
  int hi = (__double2hiint(y) & 0x7ff00000) + (k << 20);
  return __hiloint2double(hi, 0);
}

// y * 2^m by adding m to the exponent field (y normal, result normal)
__device__ __forceinline__ double scale_exp(double y, int m) {
  return __hiloint2double(__double2hiint(y) + (m << 20), __double2loint(y));
}

// Fast-path rounding: *ok is set when every real within 2^LOG2E ulps of yh
// rounds to the returned float.
template <int LOG2E>
__device__ __forceinline__ float round_f32_fast(double yh, bool& ok) {
  double d = pow2_of_exp(yh, LOG2E - 52);
  float a = (float)(yh - d);
  float b = (float)(yh + d);
  ok = a == b;
  return b;
}

// The same test read off the bits of yh, for results that round to a normal
// binary32 number or to zero (|yh| in [2^-126, 2^128), or yh = 0): within the
// binade of yh the binary32 rounding boundaries -- the midpoints between
// consecutive floats -- are exactly the binary64 numbers whose 29 low
// significand bits equal 2^28, and a binade edge is a float, not a boundary.
// Those bits and 2^28 are integers (in ulps of yh), so when they differ by
// more than E no boundary lies within E + 1 ulps of yh: the test is sound for
// an error bound below E + 1 ulps.
template <unsigned E>
__device__ __forceinline__ float round_f32_bits(double yh, bool& ok) {
  const uint32_t lo = (uint32_t)__double2loint(yh);
  ok = ((lo - (0x10000000u - E)) & 0x1fffffffu) > 2u * E;
  return (float)yh;
}

// Same, with an absolute error bound instead of a count of ulps.
__device__ __forceinline__ float round_f32_fast_abs(double yh, double err, bool& ok) {
  float a = (float)(yh - err);
  float b = (float)(yh + err);
  ok = a == b;
  return b;
}

// Round-to-odd of h + l into binary64, given h = RN(h + l).
__device__ __forceinline__ double ro53(double h, double l) {
  long long b = __double_as_longlong(h);
  if (l != 0.0) {
    if ((l < 0.0) != (h < 0.0)) b -= 1;
    b |= 1;
  }
  return __longlong_as_double(b);
}

// Accurate-path rounding of h + l (|l| <= ulp(h)/2) known to within a relative
// error drel (drel already includes a safety margin).
__device__ __forceinline__ float round_f32_dd(double h, double l, double drel, bool& ok) {
  double e = fabs(h) * drel;
  dd lo = fast_two_sum(h, l - e);
  dd hi = fast_two_sum(h, l + e);
  float a = (float)ro53(lo.hi, lo.lo);
  float b = (float)ro53(hi.hi, hi.lo);
  ok = a == b;
  return b;
}

// ---------------------------------------------------- directed rounding
// The rounding modes of IEEE 754-2019 Sec. 4.3 that the paper's CPU library
// offers besides round to nearest (Sec. II-A; its GPU runs were round to
// nearest only, Sec. III-C).  Here they are reached from round-to-nearest
// hardware: a binary64 value v is converted to binary32 to nearest, and the
// result is moved by one ulp when it lies on the wrong side of v.
enum { RM_RN = 0, RM_RZ = 1, RM_RU = 2, RM_RD = 3 };

// The next binary32 number above / below r (r finite or an infinity reached
// from the other side; from +-0 the smallest subnormal of that direction).
__device__ __forceinline__ float f32_next_up(float r) {
  const uint32_t b = f32_bits(r);
  if ((b & 0x7fffffffu) == 0) return bits_f32(1u);
  return bits_f32((b >> 31) ? b - 1 : b + 1);
}
__device__ __forceinline__ float f32_next_down(float r) {
  const uint32_t b = f32_bits(r);
  if ((b & 0x7fffffffu) == 0) return bits_f32(0x80000001u);
  return bits_f32((b >> 31) ? b + 1 : b - 1);
}

// v (binary64, not NaN) rounded to binary32 in mode RM, overflow included:
// RN(v) is exact in binary64, so comparing it with v tells on which side of
// v it lies.
template <int RM>
__device__ __forceinline__ float cvt_f32_mode(double v) {
  const float r = (float)v;
  if (RM == RM_RN) return r;
  const double back = (double)r;
  const bool above = back > v, below = back < v;  // r above / below v
  const bool toward_zero_up = v < 0.0;            // for RZ: the direction of zero
  if (RM == RM_RU) return below ? f32_next_up(r) : r;
  if (RM == RM_RD) return above ? f32_next_down(r) : r;
  // RZ
  if (toward_zero_up) return below ? f32_next_up(r) : r;
  return above ? f32_next_down(r) : r;
}

// Accurate-path rounding in mode RM of h + l (|l| <= ulp(h)/2) known to within
// a relative error drel: both ends as round-to-odd binary64 numbers, then the
// mode's conversion.  A binary32 number is an even binary64 number, so a
// round-to-odd value lies strictly between the same two binary32 numbers as
// the exact one, and any rounding of it to binary32 is the rounding of the
// exact value (Boldo and Melquiond, cited above).
template <int RM>
__device__ __forceinline__ float round_f32_dd_mode(double h, double l, double drel, bool& ok) {
  double e = fabs(h) * drel;
  dd lo = fast_two_sum(h, l - e);
  dd hi = fast_two_sum(h, l + e);
  float a = cvt_f32_mode<RM>(ro53(lo.hi, lo.lo));
  float b = cvt_f32_mode<RM>(ro53(hi.hi, hi.lo));
  ok = a == b;
  return b;
}

// The same with an absolute error bound e.
template <int RM>
__device__ __forceinline__ float round_f32_dd_abs_mode(double h, double l, double e, bool& ok) {
  dd lo = fast_two_sum(h, l - e);
  dd hi = fast_two_sum(h, l + e);
  float a = cvt_f32_mode<RM>(ro53(lo.hi, lo.lo));
  float b = cvt_f32_mode<RM>(ro53(hi.hi, hi.lo));
  ok = a == b;
  return b;
}

// The rounding in mode RM of base + d, for a binary32 base and a d of sign s
// (+1 or -1) smaller than a quarter ulp of base (tiny arguments: sin x just
// below x, cos x just below 1, ...).
template <int RM>
__device__ __forceinline__ float round_near_float(float base, int s) {
  if (RM == RM_RU) return s > 0 ? f32_next_up(base) : base;
  if (RM == RM_RD) return s < 0 ? f32_next_down(base) : base;
  if (RM == RM_RZ) {
    if (base > 0.0f) return s < 0 ? f32_next_down(base) : base;
    return s > 0 ? f32_next_up(base) : base;
  }
  return base;
}

}  // namespace cr
