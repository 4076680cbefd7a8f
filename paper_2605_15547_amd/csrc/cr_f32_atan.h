// cr_f32_atan.h -- correctly rounded atanf, asinf, acosf (device).
//
// atanf, asinf and acosf are among the paper's functions (Sec. II-A); the
// paper's table sizes for cr_atanf (Table I: 0.125 KB, 16 binary64 values)
// suggest a 16-entry atan(c_j) table, used here as follows.  All three are
// atan(Y/X) for Y, X >= 0:
//   atan x = atan(|x| / 1),   asin x = atan(|x| / s),   acos x = atan(s / x)
//   (x >= 0) or pi - atan(s / |x|) (x < 0), with s = sqrt(1 - x^2).
// With z = min(Y, X) / max(Y, X) and c = j/16, j = min(rint(16 z), 15):
//   Y <= X:  atan(Y/X) = atan(c) + atan(t),           t = (Y - c X)/(X + c Y)
//   Y >  X:  atan(Y/X) = (pi/2 - atan(c)) - atan(t),  t = (X - c Y)/(Y + c X)
// |t| <= 1/31, and atan t = t + t^3 P(t^2).  c X and c Y are exact products
// inside the FMAs, so t carries one rounding of each of numerator,
// denominator and quotient.  j = 0 gives c = 0 and t = Y/X exactly rounded,
// so small results (atan/asin of small x, acos near 1) keep full relative
// accuracy.  An error in s moves asin and acos by at most x ds and s ds
// respectively, below 2^-52.4 of the result, so s needs no extra precision
// in the fast path.
#pragma once
#include "cr_consts.h"
#include "cr_round.h"

namespace cr {

enum { ATANK_ATAN = 0, ATANK_ASIN = 1, ATANK_ACOS = 2 };

struct AtanTab {
  double4 t[16];
};

__device__ __forceinline__ void atan_tab_load(AtanTab& t, int tid) {
  if (tid < 16) t.t[tid] = ATAN_T[tid];
}

// atan(Y/X) = hi + lo (not normalised), Y, X >= 0, not both zero
__device__ __forceinline__ void atan_ratio_fast(double Y0, double X0, const AtanTab& tb,
                                                double& hi, double& lo) {
  bool inv = Y0 > X0;
  double Y = inv ? X0 : Y0, X = inv ? Y0 : X0;
  float zf = (float)Y * __builtin_amdgcn_rcpf((float)X);  // index only: an estimate suffices
  int j = (int)rintf(16.0f * zf);
  j = j > 15 ? 15 : (j < 0 ? 0 : j);
  double c = (double)j * 0.0625;
  // the quotient of the rounded num and den within 2^-52 (den >= X > 0)
  double t = div_fast(fma(-c, X, Y), fma(c, Y, X));
  double t2 = t * t;
  double p = ATAN_P[ATAN_P_DEG];
#pragma unroll
  for (int i = ATAN_P_DEG - 1; i >= 0; i--) p = fma(p, t2, ATAN_P[i]);
  double at = fma(t * t2, p, t);
  double4 T = tb.t[j];
  hi = inv ? T.z : T.x;
  lo = (inv ? T.w : T.y) + (inv ? -at : at);
}

// sqrt(w) for w >= 2^-48 (w = 1 - a^2 for a binary32 a in [0, 1), a multiple
// of 2^-48): the hardware reciprocal square root refined by Goldschmidt's
// iteration and two Newton corrections -- the compiler's expansion of sqrt
// without its rescaling of tiny and special operands, which cannot occur here
__device__ __forceinline__ double sqrt_unit(double w) {
  const double y = __builtin_amdgcn_rsq(w);
  double s = w * y, h = 0.5 * y;
  const double r = fma(-h, s, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  s = fma(fma(-s, s, w), h, s);
  return fma(fma(-s, s, w), h, s);
}

// Fast-path error: t has relative error <= 4 2^-53 (num, den, the quotient;
// + P < 2^-66), so atan t is within 2^-56 absolute (|t| <= 1/31); the result
// is >= |t|/2 for j = 0 and >= 0.03 otherwise; with the final addition this is
// below 5 ulps, 10 ulps of yh when yh falls just below a power of two.  The
// bit test of cr_round.h rejects yh within 16 ulps of the midpoint pattern
// (sound below 17 ulps).  It needs results that round to normal binary32
// numbers: the tiny arguments whose results could be subnormal are special
// cases of the fast path (atan_special_fast), and acos is at least 2^-11.5.
constexpr unsigned ATAN_TEST_E = 16;

// Branch-free: res is always written (meaningful only when true is returned).
__device__ __forceinline__ bool atan_special(float xf, int kind, float& res) {
  const bool nan = xf != xf;
  const bool dom = kind != ATANK_ATAN && fabsf(xf) > 1.0f;
  const bool zero = kind != ATANK_ACOS && xf == 0.0f;  // atan(+-0) = asin(+-0) = +-0
  const bool one = kind == ATANK_ACOS && xf == 1.0f;
  float v = zero ? xf : (one ? 0.0f : bits_f32(0x7fc00000u));
  res = nan_or(xf, v);
  return nan | dom | zero | one;
}

// The fast path's special cases: those of atan_special and, for atan and asin,
// the tiny arguments |x| < 2^-13 (zeros and subnormals included), whose
// results round to x itself: atan x lies within x^2/3 < 2^-27.6 of x below x
// (relative), asin x within x^2/6 above it, and half the spacing of the
// binary32 numbers next to x is at least 2^-25 |x| on either side (and the
// deviation is far below half the subnormal quantum for subnormal x).
template <int KIND>
__device__ __forceinline__ bool atan_special_fast(float xf, float& res) {
  bool spc = atan_special(xf, KIND, res);
  if (KIND != ATANK_ACOS) {
    const bool tiny = fabsf(xf) < 0x1p-13f;
    res = tiny ? xf : res;
    spc |= tiny;
  }
  return spc;
}

template <int KIND>
__device__ __forceinline__ float atan_fast(float xf, const AtanTab& tb, bool& ok) {
  // atan(2^100) and atan(inf) both round to RN(pi/2): clamp to keep 0 * inf out
  double x = (double)xf, a = fmin(fabs(x), 0x1p100);
  double hi, lo, yh;
  if (KIND == ATANK_ATAN) {
    atan_ratio_fast(a, 1.0, tb, hi, lo);
    yh = hi + lo;
    if (xf < 0.0f) yh = -yh;
  } else {
    // |x| = 1 gives w = 0, replaced by 2^-100: asin(+-1) and acos(-1) come out
    // within 2^-50 of +-pi/2 and pi and round to them (acos(1) and |x| > 1 are
    // special cases)
    double s = sqrt_unit(fmax(fma(-a, a, 1.0), 0x1p-100));
    if (KIND == ATANK_ASIN) {
      atan_ratio_fast(a, s, tb, hi, lo);
      yh = hi + lo;
      if (xf < 0.0f) yh = -yh;
    } else {
      atan_ratio_fast(s, a, tb, hi, lo);
      // pi - atan(s/|x|) for x < 0, atan(s/x) otherwise, as selects (an
      // if/else compiles to branches that a mixed-sign wave runs both sides of)
      const bool neg = xf < 0.0f;
      dd p = fast_two_sum(neg ? PI_HI : 0.0, neg ? -hi : hi);
      yh = p.hi + (p.lo + ((neg ? PI_LO : 0.0) + (neg ? -lo : lo)));
    }
  }
  float res = round_f32_bits<ATAN_TEST_E>(yh, ok);
  float sp;
  if (atan_special_fast<KIND>(xf, sp)) {
    res = sp;
    ok = true;
  }
  return res;
}

// ------------------------------------------------------------ accurate path
__device__ __forceinline__ dd dd_div_i(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd p = dd_mul_d(b, q1);
  dd r = dd_add(a, dd_neg(p));
  double q2 = r.hi / b.hi;
  return fast_two_sum(q1, q2);
}

// atan(Y/X) in double-double for double-double Y, X >= 0
__device__ __forceinline__ dd atan_ratio_acc(dd Y0, dd X0, const AtanTab& tb) {
  bool inv = Y0.hi > X0.hi;
  dd Y = inv ? X0 : Y0, X = inv ? Y0 : X0;
  float zf = (float)Y.hi * __builtin_amdgcn_rcpf((float)X.hi);
  int j = (int)rintf(16.0f * zf);
  j = j > 15 ? 15 : (j < 0 ? 0 : j);
  double c = (double)j * 0.0625;
  dd num = dd_add(Y, dd_neg(dd_mul_d(X, c)));
  dd den = dd_add(X, dd_mul_d(Y, c));
  dd t = dd_div_i(num, den);
  dd t2 = dd_mul(t, t);
  double ph = ATAN_TAYLOR[ATAN_TAYLOR_N].x;
#pragma unroll
  for (int k = ATAN_TAYLOR_N - 1; k >= 5; k--) ph = fma(ph, t2.hi, ATAN_TAYLOR[k].x);
  dd p = {ph, 0.0};
#pragma unroll
  for (int k = 4; k >= 0; k--) {
    double2 cc = ATAN_TAYLOR[k];
    p = dd_add(dd_mul(p, t2), dd{cc.x, cc.y});
  }
  dd at = dd_mul(p, t);
  double4 T = tb.t[j];
  dd base = inv ? dd{T.z, T.w} : dd{T.x, T.y};
  return dd_add(base, inv ? dd_neg(at) : at);
}

// s = sqrt(1 - a^2) as a double-double (a in [0, 1])
__device__ __forceinline__ dd sqrt_1m_sq(double a) {
  dd p = two_prod(a, a);
  dd w = dd_add_d(dd{-p.hi, -p.lo}, 1.0);
  if (w.hi <= 0.0) return {0.0, 0.0};
  double s0 = sqrt(w.hi);
  dd s2 = two_prod(s0, s0);
  double corr = ((w.hi - s2.hi) - s2.lo + w.lo) / (2.0 * s0);
  return fast_two_sum(s0, corr);
}

template <int KIND>
__device__ __noinline__ AccResult atan_accurate(float xf, const AtanTab& tb) {
  float sp;
  if (atan_special(xf, KIND, sp)) return {sp, 1};
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
  float r = round_f32_dd(y.hi, y.lo, 0x1p-85, ok);
  return {r, ok ? 1 : 0};
}

}  // namespace cr
