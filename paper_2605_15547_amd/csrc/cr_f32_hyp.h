// cr_f32_hyp.h -- correctly rounded sinhf, coshf, tanhf (device).
//
// sinhf, coshf and tanhf are among the paper's functions (Sec. II-A; Table I
// gives a 16-entry table for cr_sinhf).  They reuse the exponential kernel's
// reduction and 16-entry 2^(j/16) table; with a = |x|:
//   sinh a = (e + e/(e + 1)) / 2,   e = expm1(a)
//   cosh a = (E + 1/E) / 2,         E = exp(a)
//   tanh a = e / (e + 2),           e = expm1(2a)
// Every term is positive, so nothing cancels: small arguments keep the
// relative accuracy of expm1, which needs no special small-argument branch.
#pragma once
#include "cr_f32_exp.h"

namespace cr {

enum { HYPK_SINH = 0, HYPK_COSH = 1, HYPK_TANH = 2 };

// exp(a) (EM1 = false) or expm1(a) (EM1 = true) in binary64, fast path
template <bool EM1>
__device__ __forceinline__ double exp_core_fast(float af, double a, const ExpTab& tb) {
  ExpSetup<EM1 ? EXPK_EM1 : EXPK_E> S;
  S.xc = a;  // caller clamps
  exp_reduce_fast<EXPK_E>(a, S.kd, S.r);
  int k = (int)S.kd;
  S.m = k >> 4;
  S.T = tb.t[k & 15];
  double r = S.r;
  double p = EXPM1_P[EXPM1_P_DEG];
#pragma unroll
  for (int i = EXPM1_P_DEG - 1; i >= 0; i--) p = fma(p, r, EXPM1_P[i]);
  double q = fma(r * r, p, r);
  double s = pow2i(S.m);
  if (EM1) return fma(s, fma(S.T.x, q, S.T.y), fma(s, S.T.x, -1.0));
  return (S.T.x + fma(S.T.x, q, S.T.y)) * s;
  (void)af;
}

// Fast-path error: expm1/exp carry <= 4 ulps; the division (div_fast, within
// 2 ulps) and the sums add <= 4: 8 ulps of y, 16 of yh when yh falls just
// below a power of two.  The bit test of cr_round.h rejects yh within 32 ulps
// of the midpoint pattern (sound below 33 ulps).  It needs results that round
// to normal binary32 numbers or overflow: the tiny arguments of sinh and tanh,
// whose results could be subnormal, are special cases of the fast path
// (hyp_special_fast); cosh is at least 1; results of 2^128 and above round to
// infinity on either side of the test.
constexpr unsigned HYP_TEST_E = 32;

// Branch-free: res is always written (meaningful only when true is returned).
__device__ __forceinline__ bool hyp_special(float xf, int kind, float& res) {
  const bool nan = xf != xf;
  const bool zero = kind != HYPK_COSH && xf == 0.0f;
  res = nan_or(xf, xf);
  return nan | zero;
}

template <int KIND>
__device__ __forceinline__ double hyp_value_fast(float xf, const ExpTab& tb) {
  double a = fabs((double)xf);
  if (KIND == HYPK_SINH) {
    a = fmin(a, 100.0);  // sinh(100) > 2^143 overflows binary32 like sinh(inf)
    double e = exp_core_fast<true>(xf, a, tb);
    return 0.5 * (e + div_fast(e, e + 1.0));
  } else if (KIND == HYPK_COSH) {
    a = fmin(a, 100.0);
    double E = exp_core_fast<false>(xf, a, tb);
    return 0.5 * (E + div_fast(1.0, E));
  } else {
    a = fmin(a, 20.0);  // tanh(20) = 1 - 2^-57.7 rounds to 1 like tanh(inf)
    double e = exp_core_fast<true>(xf, 2.0 * a, tb);
    return div_fast(e, e + 2.0);
  }
}

// The fast path's special cases: those of hyp_special and, for sinh and tanh,
// the tiny arguments |x| < 2^-13 (zeros and subnormals included), whose
// results round to x itself: sinh x lies within x^2/6 < 2^-28.6 of x above x
// (relative), tanh x within x^2/3 < 2^-27.6 below it, and half the spacing of
// the binary32 numbers next to x is at least 2^-25 |x| on either side (and the
// deviation is far below half the subnormal quantum for subnormal x).
template <int KIND>
__device__ __forceinline__ bool hyp_special_fast(float xf, float& res) {
  bool spc = hyp_special(xf, KIND, res);
  if (KIND != HYPK_COSH) {
    const bool tiny = fabsf(xf) < 0x1p-13f;
    res = tiny ? xf : res;
    spc |= tiny;
  }
  return spc;
}

template <int KIND>
__device__ __forceinline__ float hyp_fast(float xf, const ExpTab& tb, bool& ok) {
  double y = hyp_value_fast<KIND>(xf, tb);
  if (KIND != HYPK_COSH && xf < 0.0f) y = -y;
  float res = round_f32_bits<HYP_TEST_E>(y, ok);
  float sp;
  if (hyp_special_fast<KIND>(xf, sp)) {
    res = sp;
    ok = true;
  }
  return res;
}

// exp(a) or expm1(a) in double-double (relative error < 2^-98)
template <bool EM1>
__device__ __forceinline__ dd exp_core_acc(double a, const ExpTab& tb) {
  double kd = rint(a * INV_LN2_16);
  int k = (int)kd;
  int m = k >> 4;
  double2 T = tb.t[k & 15];
  dd rr = exp_reduce_acc<EXPK_E>(a, kd);
  dd qq = expm1_dd(rr);
  dd Td = {T.x, T.y};
  dd Tq = dd_mul(Td, qq);
  double s = pow2i(m);
  if (EM1) {
    dd A = dd_add_d(dd_mul_pow2(Td, s), -1.0);
    return dd_add(A, dd_mul_pow2(Tq, s));
  }
  return dd_mul_pow2(dd_add(Td, Tq), s);
}

__device__ __forceinline__ dd dd_div_h(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd p = dd_mul_d(b, q1);
  dd r = dd_add(a, dd_neg(p));
  double q2 = r.hi / b.hi;
  return fast_two_sum(q1, q2);
}

template <int KIND>
__device__ __noinline__ AccResult hyp_accurate(float xf, const ExpTab& tb) {
  float sp;
  if (hyp_special(xf, KIND, sp)) return {sp, 1};
  double a = fabs((double)xf);
  dd y;
  if (KIND == HYPK_SINH) {
    dd e = exp_core_acc<true>(fmin(a, 100.0), tb);
    y = dd_mul_pow2(dd_add(e, dd_div_h(e, dd_add_d(e, 1.0))), 0.5);
  } else if (KIND == HYPK_COSH) {
    dd E = exp_core_acc<false>(fmin(a, 100.0), tb);
    y = dd_mul_pow2(dd_add(E, dd_div_h(dd{1.0, 0.0}, E)), 0.5);
  } else {
    dd e = exp_core_acc<true>(2.0 * fmin(a, 20.0), tb);
    y = dd_div_h(e, dd_add_d(e, 2.0));
  }
  if (KIND != HYPK_COSH && xf < 0.0f) y = dd_neg(y);
  bool ok;
  float r = round_f32_dd(y.hi, y.lo, 0x1p-85, ok);
  return {r, ok ? 1 : 0};
}

}  // namespace cr
