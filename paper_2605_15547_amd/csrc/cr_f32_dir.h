// cr_f32_dir.h -- the binary32 functions in the directed rounding modes
// (device): round toward zero, toward +infinity, toward -infinity.
//
// The paper's CPU library supports every IEEE 754 rounding mode: its kernels
// end with round-to-zero + sticky so that the final conversion can round in
// the user's mode (Sec. II-A); its GPU runs were round to nearest only
// (Sec. III-C).  Here a directed mode runs each element through a double-
// double evaluation of about 2^-100 relative accuracy (the accurate paths of
// the round-to-nearest kernels, with the longer series where those were cut
// to the round-to-nearest hard cases) and rounds both ends of its error
// interval as round-to-odd binary64 numbers in the requested mode
// (cr_round.h).  In a directed mode the rounding boundaries are the binary32
// numbers themselves, so three kinds of input are decided before that:
//  * exact results (exp2f at integers, exp10f at 1..10, log2f at powers of
//    two, log10f at 10..10^10, and the special values): an error interval
//    around an exact binary32 result always straddles it;
//  * tiny arguments, |x| < 2^-26, where f(x) = x (1 + c x^2 + ...) or
//    1 + c x + ... lies within a quarter ulp of x or 1 on a known side;
//  * saturation that the evaluation clamps (expm1 near -1, infinite inputs).
// Every other result is certified by the rounding of both interval ends.
#pragma once
#include "cr_f32_atan.h"
#include "cr_f32_exp.h"
#include "cr_f32_hyp.h"
#include "cr_f32_log.h"
#include "cr_f32_rsqrt.h"
#include "cr_f32_trig.h"

namespace cr {

constexpr float DIR_TINY = 0x1p-26f;  // tiny-argument threshold
constexpr double DIR_DREL = 0x1p-90;  // relative bound used with the ~2^-100 evaluations

__device__ __forceinline__ float quiet_nan(float x) { return bits_f32(f32_bits(x) | 0x00400000u); }
__device__ __forceinline__ int sign_of(float x) { return x < 0.0f ? -1 : 1; }

// ------------------------------------------------------------ exp family
template <int K, int RM>
__device__ __noinline__ AccResult exp_dir(float xf, const ExpTab& tb) {
  if (xf != xf) return {quiet_nan(xf), 1};
  if (xf == INFINITY) return {INFINITY, 1};
  if (xf == -INFINITY) return {K == EXPK_EM1 ? -1.0f : 0.0f, 1};
  if (xf == 0.0f) return {K == EXPK_EM1 ? xf : 1.0f, 1};
  if (fabsf(xf) < DIR_TINY)  // b^x = 1 + x ln b + ..., expm1 x = x + x^2/2 + ...
    return {K == EXPK_EM1 ? round_near_float<RM>(xf, 1) : round_near_float<RM>(1.0f, sign_of(xf)),
            1};
  if (K == EXPK_EM1 && xf <= -18.0f)  // e^x - 1 in (-1, -1 + 2^-25.9)
    return {round_near_float<RM>(-1.0f, 1), 1};
  if (K == EXPK_2 && xf == rintf(xf) && xf >= -149.0f && xf <= 127.0f)
    return {__builtin_ldexpf(1.0f, (int)xf), 1};  // 2^k exactly
  if (K == EXPK_10 && xf == rintf(xf) && xf >= 1.0f && xf <= 10.0f) {
    double p = 10.0;  // 10^k exactly (k <= 10: below 2^34, 24 significant bits)
    for (int i = 1; i < (int)xf; i++) p *= 10.0;
    return {(float)p, 1};
  }
  ExpSetup<K> S = exp_setup<K>(xf, tb);  // clamped inputs keep their side of every threshold
  double s = pow2i(S.m);
  dd rr = exp_reduce_acc<K>(S.xc, S.kd);  // within 2^-98 relative
  dd qq = expm1_dd(rr);                    // Taylor to degree 14
  dd Td = {S.T.x, S.T.y};
  dd Tq = dd_mul(Td, qq);
  dd y;
  if (K == EXPK_EM1) {
    dd A = dd_add_d(dd_mul_pow2(Td, s), -1.0);
    y = dd_add(A, dd_mul_pow2(Tq, s));
  } else {
    y = dd_mul_pow2(dd_add(Td, Tq), s);
  }
  bool ok;
  float r = round_f32_dd_mode<RM>(y.hi, y.lo, DIR_DREL, ok);
  return {r, ok ? 1 : 0};
}

// ------------------------------------------------------------ log family
// log1p(t) = 2 atanh(t/(2 + t)) for a double-double |t| <= 1/16: s = t/(2+t)
// (|s| < 1/31) in double-double, the series to s^21 (remainder below 2^-105
// relative), terms 6..10 in binary64, 0..5 by double-double Horner steps:
// within 2^-100 |log1p t|.
__device__ __forceinline__ dd log1p_dd_long(dd t) {
  dd den = dd_add_d(t, 2.0);
  double q1 = t.hi / den.hi;
  dd rr = dd_add(t, dd_neg(dd_mul_d(den, q1)));
  dd s = fast_two_sum(q1, rr.hi / den.hi);
  dd s2 = dd_mul(s, s);
  double P = INV_ODD_DD[10].x;
#pragma unroll
  for (int k = 9; k >= 6; k--) P = fma(P, s2.hi, INV_ODD_DD[k].x);
  dd w = {P, 0.0};
#pragma unroll
  for (int k = 5; k >= 0; k--) w = dd_add_ord(dd{INV_ODD_DD[k].x, INV_ODD_DD[k].y}, dd_mul(s2, w));
  dd l = dd_mul(s, w);
  return {2.0 * l.hi, 2.0 * l.lo};
}

template <int K, int RM>
__device__ __noinline__ AccResult log_dir(float xf, const LogTab& tb) {
  float sp;
  if (log_special<K>(xf, sp)) return {sp, 1};  // every special result is exact
  if (K == LOGK_2 && (f32_bits(xf) & 0x007fffffu) == 0)  // normal powers of two
    return {(float)((int)(f32_bits(xf) >> 23) - 127), 1};
  if (K == LOGK_2 && f32_bits(xf) < 0x00800000u && __popc(f32_bits(xf)) == 1)  // subnormal ones
    return {(float)(__ffs(f32_bits(xf)) - 1 - 149), 1};
  if (K == LOGK_10) {
    float p = 10.0f;  // 10^k exactly for k <= 10
    for (int k = 1; k <= 10; k++, p *= 10.0f)
      if (xf == p) return {(float)k, 1};
  }
  if (K == LOGK_1P && fabsf(xf) < DIR_TINY) return {round_near_float<RM>(xf, -1), 1};
  LogSetup S = log_setup<K>(xf, tb);
  dd p = two_prod(S.m, S.c);
  dd t = fast_two_sum(p.hi - 1.0, p.lo);
  if (K == LOGK_1P) {
    // (1 + x) - u exactly (TwoSum), scaled like m; non-zero only for x >= 2^29
    const double ulo = two_sum(1.0, (double)xf).lo * pow2i(-S.e2);
    t = dd_add_d(t, ulo * S.c);
  }
  dd l = log1p_dd_long(t);
  if (K == LOGK_2) l = dd_mul(l, dd{INV_LN2_HI, INV_LN2_LO});
  if (K == LOGK_10) l = dd_mul(l, dd{INV_LN10_HI, INV_LN10_LO});
  dd C = K == LOGK_2 ? dd{1.0, 0.0}
                     : K == LOGK_10 ? dd{LOG10_2_HI, LOG10_2_LO} : dd{LN2_HI, LN2_LO};
  dd y = dd_add(dd_mul_d(C, (double)S.e2), log_table_dd(S));
  y = dd_add(y, l);
  bool ok;
  float r = round_f32_dd_mode<RM>(y.hi, y.lo, DIR_DREL, ok);
  return {r, ok ? 1 : 0};
}

// ------------------------------------------------------------------ rsqrt
// z = RN(x^-1/2) is decided exactly (cr_f32_rsqrt.h); the sign of z^2 x - 1
// (z^2 exact in binary64, one rounding in the fma) tells whether z lies above
// or below x^-1/2, and it is zero exactly when x^-1/2 is z.
template <int RM>
__device__ __noinline__ AccResult rsqrt_dir(float xf) {
  float sp;
  if (rsqrt_special(xf, sp)) return {sp, 1};
  const float z = rsqrt_eval(xf);
  const double zd = (double)z;
  const double d = fma(zd * zd, (double)xf, -1.0);
  if (d == 0.0) return {z, 1};
  return {round_near_float<RM>(z, d > 0.0 ? -1 : 1), 1};
}

// ------------------------------------------------------------------- trig
template <int KIND, int RM>
__device__ __noinline__ AccResult trig_dir(float xf, const TrigTab& tb) {
  float sp;
  if (trig_special(xf, sp, KIND)) return {sp, 1};
  if (fabsf(xf) < DIR_TINY) {  // sin x = x - x^3/6, cos x = 1 - x^2/2, tan x = x + x^3/3
    if (KIND == TRIGK_COS) return {round_near_float<RM>(1.0f, -1), 1};
    return {round_near_float<RM>(xf, KIND == TRIGK_SIN ? -sign_of(xf) : sign_of(xf)), 1};
  }
  TrigAcc A = trig_acc_core(xf, tb);
  const bool neg = xf < 0.0f;
  dd y;
  double e;
  if (KIND == TRIGK_COS) {
    y = A.c;
    e = fma(fabs(y.hi), 0x1p-95, A.eabs);
  } else if (KIND == TRIGK_SIN) {
    y = neg ? dd_neg(A.s) : A.s;
    e = fma(fabs(y.hi), 0x1p-95, A.eabs);
  } else {
    y = dd_div(A.s, A.c);
    if (neg) y = dd_neg(y);
    double ic = 1.0 / fabs(A.c.hi);
    e = fma(fabs(y.hi), 0x1p-93, A.eabs * ic * (1.0 + fabs(y.hi)) * 2.0);
  }
  bool ok;
  float r = round_f32_dd_abs_mode<RM>(y.hi, y.lo, e, ok);
  return {r, ok ? 1 : 0};
}

template <int RM>
__device__ __noinline__ AccResult2 sincos_dir(float xf, const TrigTab& tb) {
  float ss, cs;
  if (trig_special(xf, ss, TRIGK_SIN)) {
    trig_special(xf, cs, TRIGK_COS);
    return {ss, cs, 1};
  }
  if (fabsf(xf) < DIR_TINY)
    return {round_near_float<RM>(xf, -sign_of(xf)), round_near_float<RM>(1.0f, -1), 1};
  TrigAcc A = trig_acc_core(xf, tb);
  dd s = xf < 0.0f ? dd_neg(A.s) : A.s;
  bool ok1, ok2;
  float rs = round_f32_dd_abs_mode<RM>(s.hi, s.lo, fma(fabs(s.hi), 0x1p-95, A.eabs), ok1);
  float rc = round_f32_dd_abs_mode<RM>(A.c.hi, A.c.lo, fma(fabs(A.c.hi), 0x1p-95, A.eabs), ok2);
  return {rs, rc, (ok1 && ok2) ? 1 : 0};
}

// ------------------------------------------------------------------- atan
template <int KIND, int RM>
__device__ __noinline__ AccResult atan_dir(float xf, const AtanTab& tb) {
  float sp;
  if (atan_special(xf, KIND, sp)) return {sp, 1};
  if (KIND != ATANK_ACOS && fabsf(xf) < DIR_TINY)  // atan x = x - x^3/3, asin x = x + x^3/6
    return {round_near_float<RM>(xf, KIND == ATANK_ATAN ? -sign_of(xf) : sign_of(xf)), 1};
  double a = fmin(fabs((double)xf), 0x1p100);
  dd y;
  if (KIND == ATANK_ATAN) {
    y = atan_ratio_acc(dd{a, 0.0}, dd{1.0, 0.0}, tb);
    if (xf < 0.0f) y = dd_neg(y);
  } else {
    dd s = sqrt_1m_sq(a);
    if (KIND == ATANK_ASIN) {
      y = atan_ratio_acc(dd{a, 0.0}, s, tb);
      if (xf < 0.0f) y = dd_neg(y);
    } else {
      y = atan_ratio_acc(s, dd{a, 0.0}, tb);
      if (xf < 0.0f) y = dd_add(dd{PI_HI, PI_LO}, dd_neg(y));
    }
  }
  bool ok;
  float r = round_f32_dd_mode<RM>(y.hi, y.lo, 0x1p-85, ok);
  return {r, ok ? 1 : 0};
}

// ------------------------------------------------------------- hyperbolic
template <int KIND, int RM>
__device__ __noinline__ AccResult hyp_dir(float xf, const ExpTab& tb) {
  if (xf != xf) return {quiet_nan(xf), 1};
  if (xf == 0.0f) return {KIND == HYPK_COSH ? 1.0f : xf, 1};
  if (fabsf(xf) == INFINITY)  // sinh(+-inf) = +-inf, cosh(+-inf) = +inf, tanh(+-inf) = +-1
    return {KIND == HYPK_COSH ? INFINITY : (KIND == HYPK_SINH ? xf : copysignf(1.0f, xf)), 1};
  if (fabsf(xf) < DIR_TINY) {  // sinh x = x + x^3/6, cosh x = 1 + x^2/2, tanh x = x - x^3/3
    if (KIND == HYPK_COSH) return {round_near_float<RM>(1.0f, 1), 1};
    return {round_near_float<RM>(xf, KIND == HYPK_SINH ? sign_of(xf) : -sign_of(xf)), 1};
  }
  double a = fabs((double)xf);
  dd y;
  if (KIND == HYPK_SINH) {
    dd e = exp_core_acc<true>(fmin(a, 100.0), tb);
    y = dd_mul_pow2(dd_add(e, dd_div_h(e, dd_add_d(e, 1.0))), 0.5);
  } else if (KIND == HYPK_COSH) {
    dd E = exp_core_acc<false>(fmin(a, 100.0), tb);
    y = dd_mul_pow2(dd_add(E, dd_div_h(dd{1.0, 0.0}, E)), 0.5);
  } else {
    dd e = exp_core_acc<true>(2.0 * fmin(a, 20.0), tb);  // tanh(20) and beyond: in (1 - 2^-57, 1)
    y = dd_div_h(e, dd_add_d(e, 2.0));
  }
  if (KIND != HYPK_COSH && xf < 0.0f) y = dd_neg(y);
  bool ok;
  float r = round_f32_dd_mode<RM>(y.hi, y.lo, 0x1p-85, ok);
  return {r, ok ? 1 : 0};
}

}  // namespace cr
