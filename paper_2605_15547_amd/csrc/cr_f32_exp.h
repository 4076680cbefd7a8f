// cr_f32_exp.h -- correctly rounded expf, exp2f, exp10f, expm1f (device).
//
// Paper, Sec. II-A and Fig. 1 (cr_exp2f): the argument is split into an integer
// multiple of 1/8 (here 1/16) and a small remainder R; 2^(j/16) comes from a
// 16-entry table, e^R - 1 from a short polynomial, and the result is scaled by
// a power of two before the final rounding.  The paper's kernel computes in
// binary64 and ends with round-to-zero + sticky; here the binary64 fast path
// ends with the rounding test of cr_round.h and the rare lanes that fail it
// take an accurate double-double path (the paper's fast-path/fallback idea of
// Sec. II-A, future work, and Sec. II-B).
//
// Reduction (b = e, 2, 10):  b^x = 2^(k/16) e^r,  k = nearest(16 x log2 b),
// r = x ln b - k ln2/16,  |r| <= 0.02167.  With k = 16 m + j (0 <= j < 16):
//     b^x = 2^m * T[j] * (1 + q),   T[j] = 2^(j/16),   q = e^r - 1.
// expm1: e^x - 1 = (2^m T_hi - 1) + 2^m (T_lo + T_hi q) -- the first term is
// exact for -1 <= m <= 52 and k = 0 gives T = 1, so no cancellation occurs.
#pragma once
#include "cr_consts.h"
#include "cr_round.h"

namespace cr {

enum { EXPK_E = 0, EXPK_2 = 1, EXPK_10 = 2, EXPK_EM1 = 3 };

struct ExpTab {
  double2 t[16];
};

__device__ __forceinline__ void exp_tab_load(ExpTab& t, int tid) {
  if (tid < 16) t.t[tid] = EXP_T16[tid];
}

// Fast-path error bound, in ulps of the binary64 result, before the final
// rounding test.  Derivation: the table entry is a double-double (error 2^-106
// relative); q has absolute error <= 2^-58.3 (reduction 2^-58.6, polynomial
// 2^-64.8, evaluation < 2^-60); T_hi q + T_lo adds 2^-57.5; the last addition
// is one rounding (1/2 ulp).  With |e^r| >= 0.978 this is < 0.6 ulp; counting
// a factor 2 for the ulp taken from the computed value's binade gives 1.2.
// expm1 has up to 3.5 ulps (|result| >= 0.0214 when k != 0), 7 with the
// factor 2.  Every binary32 input is checked against the accurate path on the
// GPU.  The test uses 2^LOG2E ulps: 2 for exp/exp2/exp10, 8 for expm1.
template <int K>
struct ExpErr {
  static constexpr int LOG2E = (K == EXPK_EM1) ? 3 : 1;
};

// k (as a double) and the reduced argument for the fast path
template <int K>
__device__ __forceinline__ void exp_reduce_fast(double x, double& kd, double& r) {
  if (K == EXPK_E || K == EXPK_EM1) {
    kd = rint(x * INV_LN2_16);
    double rh = fma(-kd, LN2_16_C1, x);  // exact: |k| < 2^12, C1 has 41 bits
    r = fma(-kd, LN2_16_C2, rh);
  } else if (K == EXPK_2) {
    double t = x * 16.0;  // exact
    kd = rint(t);
    double f = t - kd;    // exact, |f| <= 1/2
    r = f * LN2_16_HI;
  } else {
    // 16 x log2(10) = x C1 + x C2: x C1 is exact (24 + 28 bits) and so is its
    // distance f to k; r = f ln2/16 + x C2 ln2/16 with one rounding (2^-59),
    // ln2/16's own rounding (< 2^-60.3 for |f| <= 1/2) and a negligible x C2 term
    const double p = x * LOG2_10_16_C1;
    kd = rint(p);
    r = fma(p - kd, LN2_16_HI, x * EXP10_C2_LN2_16);
  }
}

// Accurate reduction: r as a double-double with relative error < 2^-98.
template <int K>
__device__ __forceinline__ dd exp_reduce_acc(double x, double kd) {
  if (K == EXPK_E || K == EXPK_EM1) {
    double rh = fma(-kd, LN2_16_C1, x);
    dd p = two_prod(kd, LN2_16_C2);
    dd s = two_sum(rh, -p.hi);
    double lo = s.lo - p.lo - kd * LN2_16_C3;
    return fast_two_sum(s.hi, lo);
  } else if (K == EXPK_2) {
    double f = x * 16.0 - kd;
    dd p = two_prod(f, LN2_16_HI);
    return fast_two_sum(p.hi, fma(f, LN2_16_LO, p.lo));
  } else {
    double th = x * LOG2_10_16_HI;
    double tl = fma(x, LOG2_10_16_HI, -th) + x * LOG2_10_16_LO;
    dd f = fast_two_sum(th - kd, tl);
    dd p = two_prod(f.hi, LN2_16_HI);
    double lo = p.lo + fma(f.lo, LN2_16_HI, f.hi * LN2_16_LO);
    return fast_two_sum(p.hi, lo);
  }
}

// e^r - 1 in double-double for |r| <= 0.02167: Taylor series to degree 14
// (remainder < 2^-122); terms of degree >= 6 are below 2^-42 and are summed
// in binary64, the rest in double-double.
__device__ __forceinline__ dd expm1_dd(dd r) {
  double ph = INV_FACT[EXP_TAYLOR_N].x;
#pragma unroll
  for (int k = EXP_TAYLOR_N - 1; k >= 6; k--) ph = fma(ph, r.hi, INV_FACT[k].x);
  dd p = {ph, 0.0};
#pragma unroll
  for (int k = 5; k >= 1; k--) {
    double2 c = INV_FACT[k];
    p = dd_add(dd_mul(p, r), dd{c.x, c.y});
  }
  return dd_mul(p, r);
}

// e^r - 1 for the accurate path of the binary32 functions, |r| <= 0.0217:
// the Taylor series to degree 9 (remainder below 2^-71.5 |r|) as
// r + r^2/2 + r^3 P(r), with P (degrees 3..9) and r^3 in binary64: their
// rounding errors (< 2^-51 relative) act on a term below 2^-13.6 |r|, so the
// result is within 2^-64.6 |r| of e^r - 1.  r + r^2/2 is double-double.
__device__ __forceinline__ dd expm1_dd_short(dd r) {
  double p = INV_FACT[9].x;
#pragma unroll
  for (int k = 8; k >= 3; k--) p = fma(p, r.hi, INV_FACT[k].x);
  dd r2 = two_prod(r.hi, r.hi);
  r2.lo = fma(2.0 * r.hi, r.lo, r2.lo);
  const double c = (r2.hi * r.hi) * p;      // r^3 P, below |r|/3 of r^2/2
  dd h = fast_two_sum(0.5 * r2.hi, c);
  h.lo += 0.5 * r2.lo;
  return dd_add_ord(r, h);                   // |r| > |h|
}

// Shared set-up of both paths: clamp, k, the table entry and the scale 2^m.
// The clamp keeps k and the scale in range; clamped inputs still over- or
// underflow in the final conversion (|results| reach 2^+-216 at most), and the
// clamp values map to results far from any rounding boundary (2^-200, not the
// exact midpoint 2^-150, for exp2f).
template <int K>
struct ExpSetup {
  double xc, kd, r;
  int m;
  double2 T;
};

template <int K>
__device__ __forceinline__ ExpSetup<K> exp_setup(float xf, const ExpTab& tb) {
  ExpSetup<K> S;
  const double lim = (K == EXPK_10) ? 50.0 : (K == EXPK_2 ? 200.0 : 150.0);
  S.xc = fmin(fmax((double)xf, -lim), lim);
  exp_reduce_fast<K>(S.xc, S.kd, S.r);
  int k = (int)S.kd;
  S.m = k >> 4;
  S.T = tb.t[k & 15];
  return S;
}

// Inputs whose result is fixed without evaluation: NaN (returned quieted),
// exp2f(-150) = 2^-150, the one exact midpoint (ties to even give +0), and
// expm1(+-0) = +-0.
// Branch-free: res is always written (meaningful only when true is returned),
// so the compiler keeps the main computation outside any branch.
template <int K>
__device__ __forceinline__ bool exp_special(float xf, float& res) {
  const bool nan = xf != xf;
  const bool tie = K == EXPK_2 && xf == -150.0f;
  const bool zero = K == EXPK_EM1 && xf == 0.0f;
  float v = zero ? xf : 0.0f;
  res = nan_or(xf, v);
  return nan | tie | zero;
}

// Fast path: binary64 evaluation and the rounding test.  ok = false means the
// returned value is not certified and the accurate path must decide.
template <int K>
__device__ __forceinline__ float exp_fast(float xf, const ExpTab& tb, bool& ok) {
  ExpSetup<K> S = exp_setup<K>(xf, tb);
  double r = S.r;
  double p = EXPM1_P[EXPM1_P_DEG];
#pragma unroll
  for (int i = EXPM1_P_DEG - 1; i >= 0; i--) p = fma(p, r, EXPM1_P[i]);
  double q = fma(r * r, p, r);  // e^r - 1
  double yh;
  if (K == EXPK_EM1) {
    double s = pow2i(S.m);
    double D = fma(s, S.T.x, -1.0);
    yh = fma(s, fma(S.T.x, q, S.T.y), D);
  } else {
    yh = scale_exp(S.T.x + fma(S.T.x, q, S.T.y), S.m);  // |m| <= 217: stays normal
  }
  float res = round_f32_fast<ExpErr<K>::LOG2E>(yh, ok);
  float sp;
  if (exp_special<K>(xf, sp)) {
    res = sp;
    ok = true;
  }
  return res;
}

// Accurate path (double-double), kept out of line: one copy per kernel keeps
// the instruction footprint of the unrolled fast path small, and it only runs
// for the rare elements whose fast result failed the rounding test.
template <int K>
__device__ __noinline__ AccResult exp_accurate(float xf, const ExpTab& tb) {
  float sp;
  if (exp_special<K>(xf, sp)) return {sp, 1};
  ExpSetup<K> S = exp_setup<K>(xf, tb);
  double s = pow2i(S.m);
  dd rr = exp_reduce_acc<K>(S.xc, S.kd);
  dd qq = expm1_dd_short(rr);
  dd Td = {S.T.x, S.T.y};
  dd Tq = dd_mul(Td, qq);
  dd y;
  if (K == EXPK_EM1) {
    dd A = dd_add_d(dd_mul_pow2(Td, s), -1.0);
    y = dd_add(A, dd_mul_pow2(Tq, s));
  } else {
    y = dd_mul_pow2(dd_add(Td, Tq), s);
  }
  // y is within 2^-63.5 of its value relative (e^r - 1 to 2^-64.6 |r|; for
  // expm1 with k != 0 the result can be 0.0214 against terms up to 2), far
  // below the 2^-58.9 that separates the hardest binary32 case from a rounding
  // boundary (exp2f, at 2^-34.9 ulp)
  bool ok;
  float r = round_f32_dd(y.hi, y.lo, 0x1p-63, ok);
  return {r, ok ? 1 : 0};
}

}  // namespace cr
