// cr_td.h -- triple-double arithmetic and binary64 final rounding (device).
//
// The paper's binary64 kernels pair an accurate main path with a correct
// rounding test and a slower path for the lanes that fail it (Sec. II-B).
// Here the main path works in double-double (about 2^-70 after the
// approximations) and the slower path in triple-double (h + m + l, about
// 2^-140), enough for inputs far harder than any the project's own search
// found (hardness <= 56 bits beyond the rounding bit).  Triple-double sums and
// products follow the usual error-free-transform construction (e.g. Lauter,
// "Basic building blocks for a triple-double intermediate format", INRIA
// RR-5702, 2005); every step here uses TwoSum/TwoProd, so no magnitude
// ordering is assumed.
#pragma once
#include "cr_dd.h"

namespace cr {

struct td {
  double h, m, l;
};

// exact renormalisation of a + b + c into h + m + l with |m| <= ulp(h)/2
__device__ __forceinline__ td td_renorm(double a, double b, double c) {
  dd s = two_sum(b, c);
  dd t = two_sum(a, s.hi);
  dd u = two_sum(t.lo, s.lo);
  dd v = two_sum(t.hi, u.hi);
  dd w = two_sum(v.lo, u.lo);
  return {v.hi, w.hi, w.lo};
}

__device__ __forceinline__ td td_from(double a) { return {a, 0.0, 0.0}; }
__device__ __forceinline__ td td_from_dd(dd a) { return {a.hi, a.lo, 0.0}; }
__device__ __forceinline__ td td_neg(td a) { return {-a.h, -a.m, -a.l}; }
__device__ __forceinline__ td td_scale(td a, double s) { return {a.h * s, a.m * s, a.l * s}; }

__device__ __forceinline__ td td_add(td x, td y) {
  dd s0 = two_sum(x.h, y.h);
  dd s1 = two_sum(x.m, y.m);
  dd s2 = two_sum(x.l, y.l);
  dd t1 = two_sum(s0.lo, s1.hi);
  double t2 = (s1.lo + s2.hi) + (s2.lo + t1.lo);
  return td_renorm(s0.hi, t1.hi, t2);
}

__device__ __forceinline__ td td_mul(td x, td y) {
  dd p00 = two_prod(x.h, y.h);
  dd p01 = two_prod(x.h, y.m);
  dd p10 = two_prod(x.m, y.h);
  double low = fma(x.h, y.l, fma(x.m, y.m, x.l * y.h)) + (p01.lo + p10.lo);
  dd m1 = two_sum(p01.hi, p10.hi);
  dd m2 = two_sum(p00.lo, m1.hi);
  return td_renorm(p00.hi, m2.hi, (m1.lo + m2.lo) + low);
}

__device__ __forceinline__ td td_mul_d(td x, double d) {
  dd p0 = two_prod(x.h, d);
  dd p1 = two_prod(x.m, d);
  dd m2 = two_sum(p0.lo, p1.hi);
  return td_renorm(p0.hi, m2.hi, fma(x.l, d, p1.lo + m2.lo));
}

__device__ __forceinline__ td td_div(td a, td b) {
  double q1 = a.h / b.h;
  td r = td_add(a, td_neg(td_mul_d(b, q1)));
  double q2 = r.h / b.h;
  r = td_add(r, td_neg(td_mul_d(b, q2)));
  double q3 = r.h / b.h;
  return td_renorm(q1, q2, q3);
}

__device__ __forceinline__ td td_ld(double4 v) { return {v.x, v.y, v.z}; }

// ---------------------------------------------------------------- rounding
// RN_64(h + t) for a normal h and a tail t = (t1 + t2) with |t| <= ulp(h)
// (about), given an absolute error bound e on h + t.  Returns the rounded
// value; ok = false when a rounding boundary lies within e.
__device__ __forceinline__ double round64_tail(double h, double t1, double t2, double e,
                                               bool& ok) {
  dd t = two_sum(t1, t2);
  // grid spacing above |h| is U; below it is U/2 when h is a power of two
  long long hb = __double_as_longlong(h);
  double U = __longlong_as_double(hb & 0x7ff0000000000000ll) * 0x1p-52;
  bool down = (t.hi < 0.0) != (h < 0.0);  // the tail moves |h + t| below |h|
  bool pow2 = (hb & 0x000fffffffffffffll) == 0;
  double half = (down && pow2) ? 0.25 * U : 0.5 * U;
  double at = fabs(t.hi), atl = (t.hi < 0.0) ? -t.lo : t.lo;
  ok = true;
  if (at < 0.5 * half) return h;  // far from the midpoint on this side
  double d = (at - half) + atl;  // at - half is exact here (Sterbenz)
  if (fabs(d) <= e) ok = false;
  if (d > 0.0) {  // beyond the midpoint: step one grid point toward the tail
    return __longlong_as_double(down ? hb - 1 : hb + 1);
  }
  return h;
}

// Round an integer-scaled value Z = (z1 + z2 + z3), 0 <= Z < 2^54, to the
// nearest integer (ties cannot occur for the functions here: the result is
// never exactly a midpoint); ok = false when within e of a half-integer.
__device__ __forceinline__ double round_to_int(double z1, double z2, double z3, double e,
                                               bool& ok) {
  double n = rint(z1);
  dd t = two_sum(z1 - n, z2);  // z1 - n is exact
  t = two_sum(t.hi, t.lo + z3);
  double d = fabs(t.hi) - 0.5 + ((t.hi < 0.0) ? -t.lo : t.lo);
  ok = !(fabs(d) <= e);
  if (d > 0.0) n += (t.hi < 0.0) ? -1.0 : 1.0;
  return n;
}

// y * 2^m for a binary64 y in [2^-2, 2^2] with the product exact or
// overflowing to infinity (m up to 1025)
__device__ __forceinline__ double scale_pow2(double y, int m) {
  int m1 = m >> 1, m2 = m - m1;
  return (y * pow2i(m1)) * pow2i(m2);
}

}  // namespace cr
