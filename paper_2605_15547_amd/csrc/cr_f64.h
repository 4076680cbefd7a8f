// cr_f64.h -- correctly rounded binary64 exp, exp2 and log (device).
//
// Paper, Sec. II-B: a highly accurate SIMD main path, a correct rounding
// test, and a slower path for the lanes that fail it; the paper's cr_exp2
// uses three 16-entry double-double tables and its cr_log one 128-entry
// table.  Every table here has 16 entries:
//
// exp: k = nearest(x 256/ln2), r = x - k ln2/256 (four-part Cody-Waite,
//   |r| <= ln2/512), k = 256 m + 16 i + j, e^x = 2^m T1[i] T2[j] e^r with
//   T1 = 2^(i/16), T2 = 2^(j/256) (double-double in the main path, triple-
//   double in the accurate path).  Subnormal results are rounded at the fixed
//   quantum 2^-1074 by rounding y 2^(m+1074) to an integer; overflow comes
//   from scaling the rounded value.
// log: x = 2^e' m, m in [0.75, 1.5) (subnormal x scaled by 2^64 first), the
//   same 16-entry 9-bit reciprocal table as binary32: t = m c_j - 1 exact as a
//   double-double (TwoProd), log x = e' ln2 - ln c_j + log1p(t) with
//   log1p t = t - t^2/2 + t^3/3 + t^4 S(t) (main path) or 2 atanh(t/(2+t))
//   (accurate path).
// exp2: the paper's own three-table design (Sec. II-B).  x = N/4096 + R with
//   N = nearest(4096 x) and R = x - N/4096 exact (|R| <= 2^-13), N = 4096 m +
//   256 i1 + 16 i2 + i3, 2^x = 2^m T1[i1] T2[i2] T3[i3] 2^R with the 16-entry
//   tables T1 = 2^(i/16), T2 = 2^(i/256), T3 = 2^(i/4096) read as double-
//   doubles by the main path, and 2^R = e^r, r = R ln2 (|r| <= 2^-13.53), by
//   r + r^2 P(r) with P of degree 3.
// The accurate path first tries a double-double middle path, which decides
// all but the inputs within about 2^-42 ulp of a rounding boundary, and only
// those take the triple-double evaluation.
#pragma once
#include "cr_consts.h"
#include "cr_round.h"
#include "cr_td.h"

namespace cr {

struct Exp64Tab {
  double4 t1[16], t2[16];
};
struct Log64Tab {
  double c[16];
  double4 L[16];
};
struct Exp2_64Tab {
  double4 t1[16], t2[16], t3[16];
};

__device__ __forceinline__ void exp64_tab_load(Exp64Tab& t, int tid) {
  if (tid < 16) {
    t.t1[tid] = EXP64_T1[tid];
    t.t2[tid] = EXP64_T2[tid];
  }
}
__device__ __forceinline__ void exp2_64_tab_load(Exp2_64Tab& t, int tid) {
  if (tid < 16) {
    t.t1[tid] = EXP2_64_T1[tid];
    t.t2[tid] = EXP2_64_T2[tid];
    t.t3[tid] = EXP2_64_T3[tid];
  }
}
__device__ __forceinline__ void log64_tab_load(Log64Tab& t, int tid) {
  if (tid < 16) {
    t.c[tid] = LOG_C[tid];
    t.L[tid] = LOG64_L[tid];
  }
}

// ------------------------------------------------------------------- exp
// Branch-free: res is always written (meaningful only when true is returned).
__device__ __forceinline__ bool exp64_special(double x, double& res) {
  const bool nan = x != x;
  res = nan ? __longlong_as_double(__double_as_longlong(x) | 0x0008000000000000ll) : 1.0;
  return nan | (x == 0.0);
}

// main-path error, |r| <= 2^-9.53: q = e^r - 1 carries the roundings of
// r.hi^2 (2^-73.1 after the factor P ~ 1/2), of the fma (2^-73.1), P's
// evaluation error times r^2 (2^-73), the r.lo term left out of r^2 (2^-72)
// and P's approximation error (2^-83.9): below 2^-70.7 in all; the table
// entries (2^-104 each) and T1 (T2 (1 + q)) in double-double (dd_mul_1p and
// dd_mul: 2^-104 and 2^-103.7) add nothing visible.  Relative
// to y >= T (1 - 2^-9.5) that is 2^-70.7; the test uses 2^-69 |y|.
constexpr double EXP64_EPS = 0x1p-69;

// 2^m y rounded to binary64 from the double-double y (in [2^-1/512, 2)) known
// to within e; ok when every value in y +- e rounds the same way.
__device__ __forceinline__ double exp64_round(dd y, int m, double e, bool& ok) {
  if (m >= -1021) {  // normal result: round in the unscaled domain, then scale
    double a = y.hi + (y.lo - e);
    double b = y.hi + (y.lo + e);
    ok = a == b;
    return scale_pow2(b, m);
  }
  // subnormal (or zero) result: round y 2^(m+1074) to an integer
  // (y 2^(m+1074) < 2^53; for m + 1074 < 0 it is below 1 and rounds to 0 or 1)
  double sc = pow2i(m + 1074 > -200 ? m + 1074 : -200);
  double n = round_to_int(y.hi * sc, y.lo * sc, 0.0, e * sc, ok);
  return n * 0x1p-1074;
}

// B (1 + q) as a double-double, for a double-double table entry B (B.lo
// within half an ulp of B.hi) and |q| < 2^-9: B q = B.hi q.hi exactly (TwoProd)
// plus the cross terms B.hi q.lo + B.lo q.hi (each below 2^-62 |B|, rounded
// twice); B.hi + (B q).hi by Fast2Sum; the low parts added once and the sum
// renormalised.  Relative error below 2^-104 -- the product by the
// double-double 1 + q in fewer operations than dd_mul followed by dd_add_ord
// (measured: binary64 exp 3% faster).
__device__ __forceinline__ dd dd_mul_1p(dd B, dd q) {
  const dd p = two_prod(B.hi, q.hi);
  const double pl = fma(B.hi, q.lo, fma(B.lo, q.hi, p.lo));
  const dd s = fast_two_sum(B.hi, p.hi);  // |p.hi| < 2^-9 |B.hi|
  return fast_two_sum(s.hi, s.lo + (B.lo + pl));
}

__device__ __forceinline__ double exp64_fast(double x, const Exp64Tab& tb, bool& ok) {
  double xc = fmin(fmax(x, -746.0), 710.0);  // beyond: 0 or +inf after scaling
  double kd = rint(xc * EXP64_INV);
  int k = (int)kd;
  double r0 = fma(-kd, EXP64_C1, xc);  // exact: |k| < 2^19, C1 has 34 bits
  dd p = two_prod(kd, EXP64_C2);
  dd s = two_sum(r0, -p.hi);
  dd r = fast_two_sum(s.hi, (s.lo - p.lo) - kd * EXP64_C3);
  double pp = EXP64_P[EXP64_P_DEG];
#pragma unroll
  for (int i = EXP64_P_DEG - 1; i >= 0; i--) pp = fma(pp, r.hi, EXP64_P[i]);
  dd q = fast_two_sum(r.hi, fma(r.hi * r.hi, pp, r.lo));  // e^r - 1
  int m = k >> 8;
  double4 A = tb.t1[(k >> 4) & 15], B = tb.t2[k & 15];
  // T e^r = T1 (T2 (1 + q)), in [2^-1/512, 2); |q| < 2^-9
  dd y = dd_mul(dd{A.x, A.y}, dd_mul_1p(dd{B.x, B.y}, q));
  double res = exp64_round(y, m, fabs(y.hi) * EXP64_EPS, ok);
  double sp;
  if (exp64_special(x, sp)) {
    res = sp;
    ok = true;
  }
  return res;
}

struct AccResultD {
  double r;
  int ok;
};

// Middle path (double-double), tried first by the accurate path: the main
// path's reduction (r within 2^-110) and tables (2^-104), with e^r to about
// 2^-104 relative: the Taylor series to degree 9 (remainder below 2^-116), its
// degrees 5..9 in binary64 as r P(r) inside the innermost step (rounding below
// 2^-107 of the result) and degrees 0..4 by double-double Horner steps.
// y = T e^r is within 2^-100 of e^x relative; the test allows 2^-95, so only
// inputs within about 2^-42 ulp of a rounding boundary go on to the
// triple-double path.
__device__ __forceinline__ double exp64_mid(double x, const Exp64Tab& tb, bool& ok) {
  double xc = fmin(fmax(x, -746.0), 710.0);
  double kd = rint(xc * EXP64_INV);
  int k = (int)kd;
  double r0 = fma(-kd, EXP64_C1, xc);
  dd p = two_prod(kd, EXP64_C2);
  dd s = two_sum(r0, -p.hi);
  dd r = fast_two_sum(s.hi, (s.lo - p.lo) - kd * EXP64_C3);
  double P = INV_FACT[9].x;
#pragma unroll
  for (int i = 8; i >= 5; i--) P = fma(P, r.hi, INV_FACT[i].x);
  dd w = dd_add_ord(dd{INV_FACT[4].x, INV_FACT[4].y}, dd{r.hi * P, 0.0});
#pragma unroll
  for (int i = 3; i >= 0; i--) w = dd_add_ord(dd{INV_FACT[i].x, INV_FACT[i].y}, dd_mul(r, w));
  int m = k >> 8;  // w = e^r
  double4 A = tb.t1[(k >> 4) & 15], B = tb.t2[k & 15];
  dd T = dd_mul(dd{A.x, A.y}, dd{B.x, B.y});
  dd y = dd_mul(T, w);
  return exp64_round(y, m, fabs(y.hi) * 0x1p-95, ok);
}

__device__ __noinline__ AccResultD exp64_accurate(double x, const Exp64Tab& tb) {
  double sp;
  if (exp64_special(x, sp)) return {sp, 1};
  bool mid_ok;
  const double rm = exp64_mid(x, tb, mid_ok);
  if (mid_ok) return {rm, 1};
  // triple-double path
  double xc = fmin(fmax(x, -746.0), 710.0);
  double kd = rint(xc * EXP64_INV);
  int k = (int)kd;
  // r = x - k (C1 + C2 + C3 + C4) as a triple-double
  td r = td_from(fma(-kd, EXP64_C1, xc));
  dd p2 = two_prod(kd, EXP64_C2);
  dd p3 = two_prod(kd, EXP64_C3);
  r = td_add(r, td{-p2.hi, -p2.lo, 0.0});
  r = td_add(r, td{-p3.hi, -p3.lo, -kd * EXP64_C4});
  // e^r - 1: Taylor to degree 13 (|r| <= ln2/512: remainder < 2^-150);
  // degrees 6.. in double-double, 1..5 in triple-double
  dd rd = {r.h, r.m};
  dd ph = {INV_FACT[13].x, INV_FACT[13].y};
#pragma unroll
  for (int i = 12; i >= 6; i--) ph = dd_add(dd_mul(ph, rd), dd{INV_FACT[i].x, INV_FACT[i].y});
  td pt = td_from_dd(ph);
#pragma unroll
  for (int i = 5; i >= 1; i--) pt = td_add(td_mul(pt, r), td_ld(INV_FACT_TD[i]));
  td q = td_mul(pt, r);
  int m = k >> 8;
  td T = td_mul(td_ld(tb.t1[(k >> 4) & 15]), td_ld(tb.t2[k & 15]));
  td y = td_add(T, td_mul(T, q));
  double e = fabs(y.h) * 0x1p-135;
  bool ok;
  double res;
  if (m >= -1021) {
    double c = round64_tail(y.h, y.m, y.l, e, ok);
    res = scale_pow2(c, m);
  } else {
    double sc = pow2i(m + 1074 > -200 ? m + 1074 : -200);
    double n = round_to_int(y.h * sc, y.m * sc, y.l * sc, e * sc, ok);
    res = n * 0x1p-1074;
  }
  return {res, ok ? 1 : 0};
}

// ------------------------------------------------------------------ exp2
// Branch-free: res is always written (meaningful only when true is returned).
// 2^x rounds to +0 for x <= -1075 (x = -1075 is the midpoint between +0 and
// the smallest subnormal and ties to +0), overflows for x >= 1024; NaN is
// returned quieted.  Everything else goes through the evaluation, exact
// powers of two included (y = 1 exactly, far from any rounding boundary).
__device__ __forceinline__ bool exp2_64_special(double x, double& res) {
  const bool nan = x != x;
  const bool lo = x <= -1075.0, hi = x >= 1024.0;
  res = nan ? __longlong_as_double(__double_as_longlong(x) | 0x0008000000000000ll)
            : (hi ? INFINITY : 0.0);
  return nan | lo | hi;
}

// The reduction shared by the three paths: N = nearest(4096 x) and the exact
// remainder R = x - N/4096 (|x| <= 1076 after the clamp, so 4096 x and the
// fma are exact and |N| < 2^23).
struct Exp2Red {
  double R;
  int N;
};
__device__ __forceinline__ Exp2Red exp2_64_reduce(double x) {
  double xc = fmin(fmax(x, -1076.0), 1025.0);
  double nd = rint(xc * 4096.0);
  return {fma(nd, -0x1p-12, xc), (int)nd};
}

// T1[i1] T2[i2] T3[i3] as a double-double (each factor to 2^-106, each
// product 5u^2: within 2^-102.5 relative)
__device__ __forceinline__ dd exp2_64_T(const Exp2_64Tab& tb, int N) {
  double4 A = tb.t1[(N >> 8) & 15], B = tb.t2[(N >> 4) & 15], C = tb.t3[N & 15];
  return dd_mul(dd_mul(dd{A.x, A.y}, dd{B.x, B.y}), dd{C.x, C.y});
}

// Main-path error, |r| <= 2^-13.53 (r^2 <= 2^-27.06, P ~ 1/2):
//  * r = R ln2 as r.hi + r.lo: ln2 to 2^-107, the product error-free (fma),
//    R ln2_lo rounded once: below 2^-119 absolute;
//  * q = e^r - 1 = r.hi + (r.hi^2 P(r.hi) + r.lo): the rounding of r.hi^2
//    times P (2^-81.06), P's Horner evaluation (relative 2^-52.4, times r^2/2:
//    2^-80.5), the fma (half an ulp of a value below 2^-28: 2^-82), the term
//    2 r.hi r.lo P left out of r^2 (2^-80.06) and P's approximation error
//    (2^-91.95): below 2^-78.6 in all; the final Fast2Sum is exact;
//  * T1 T2 T3 (1 + q) (|q| < 2^-13.5) as dd_mul(dd_mul(T1, T2),
//    dd_mul_1p(T3, q)): the entries to 2^-106 each, the products and
//    dd_mul_1p within 2^-101.5 relative in all, far below the budget.
// y = T e^r >= 2^-1/8192 carries at most 2^-78.5 relative; the test allows
// 2^-77 |y|.
constexpr double EXP2_64_EPS = 0x1p-77;

__device__ __forceinline__ double exp2_64_fast(double x, const Exp2_64Tab& tb, bool& ok) {
  Exp2Red k = exp2_64_reduce(x);
  double rh = k.R * LN2_TD[0].x;
  double rl = fma(k.R, LN2_TD[0].x, -rh) + k.R * LN2_TD[0].y;
  double pp = EXP2_64_P[EXP2_64_P_DEG];
#pragma unroll
  for (int i = EXP2_64_P_DEG - 1; i >= 0; i--) pp = fma(pp, rh, EXP2_64_P[i]);
  dd q = fast_two_sum(rh, fma(rh * rh, pp, rl));  // e^r - 1
  // T1 T2 (T3 (1 + q)), in [2^-1/8192, 2); |q| < 2^-13.5
  const int N = k.N;
  double4 A = tb.t1[(N >> 8) & 15], B = tb.t2[(N >> 4) & 15], C = tb.t3[N & 15];
  dd y = dd_mul(dd_mul(dd{A.x, A.y}, dd{B.x, B.y}), dd_mul_1p(dd{C.x, C.y}, q));
  double res = exp64_round(y, k.N >> 12, fabs(y.hi) * EXP2_64_EPS, ok);
  double sp;
  if (exp2_64_special(x, sp)) {
    res = sp;
    ok = true;
  }
  return res;
}

// Middle path (double-double): the main path's reduction and tables, e^r by
// its Taylor series to degree 6 (remainder below 2^-106 for |r| <= 2^-13.53),
// degrees 4..6 in binary64 as r^4 P inside the innermost step, 0..3 by
// double-double Horner steps, r = R ln2 to 2^-119 absolute: y within 2^-100
// relative; the test allows 2^-95.
__device__ __forceinline__ double exp2_64_mid(double x, const Exp2_64Tab& tb, bool& ok) {
  Exp2Red k = exp2_64_reduce(x);
  dd r = dd_mul_d(dd{LN2_TD[0].x, LN2_TD[0].y}, k.R);
  double P = fma(fma(INV_FACT[6].x, r.hi, INV_FACT[5].x), r.hi, INV_FACT[4].x);
  dd w = dd_add_ord(dd{INV_FACT[3].x, INV_FACT[3].y}, dd{r.hi * P, 0.0});
#pragma unroll
  for (int i = 2; i >= 0; i--) w = dd_add_ord(dd{INV_FACT[i].x, INV_FACT[i].y}, dd_mul(r, w));
  dd y = dd_mul(exp2_64_T(tb, k.N), w);
  return exp64_round(y, k.N >> 12, fabs(y.hi) * 0x1p-95, ok);
}

__device__ __noinline__ AccResultD exp2_64_accurate(double x, const Exp2_64Tab& tb) {
  double sp;
  if (exp2_64_special(x, sp)) return {sp, 1};
  bool mid_ok;
  const double rm = exp2_64_mid(x, tb, mid_ok);
  if (mid_ok) return {rm, 1};
  // triple-double path: r = R ln2 (R exact, ln2 to 2^-159), e^r - 1 by its
  // Taylor series to degree 10 (remainder below 2^-170), degrees 5.. in
  // double-double, 1..4 in triple-double
  Exp2Red k = exp2_64_reduce(x);
  td r = td_mul_d(td_ld(LN2_TD[0]), k.R);
  dd rd = {r.h, r.m};
  dd ph = {INV_FACT[10].x, INV_FACT[10].y};
#pragma unroll
  for (int i = 9; i >= 5; i--) ph = dd_add(dd_mul(ph, rd), dd{INV_FACT[i].x, INV_FACT[i].y});
  td pt = td_from_dd(ph);
#pragma unroll
  for (int i = 4; i >= 1; i--) pt = td_add(td_mul(pt, r), td_ld(INV_FACT_TD[i]));
  td q = td_mul(pt, r);
  const int N = k.N;
  td T = td_mul(td_mul(td_ld(tb.t1[(N >> 8) & 15]), td_ld(tb.t2[(N >> 4) & 15])),
                td_ld(tb.t3[N & 15]));
  td y = td_add(T, td_mul(T, q));
  double e = fabs(y.h) * 0x1p-135;
  const int m = N >> 12;
  bool ok;
  double res;
  if (m >= -1021) {
    double c = round64_tail(y.h, y.m, y.l, e, ok);
    res = scale_pow2(c, m);
  } else {
    double sc = pow2i(m + 1074 > -200 ? m + 1074 : -200);
    double n = round_to_int(y.h * sc, y.m * sc, y.l * sc, e * sc, ok);
    res = n * 0x1p-1074;
  }
  return {res, ok ? 1 : 0};
}

// ------------------------------------------------------------------- log
// Branch-free: res is always written (meaningful only when true is returned).
__device__ __forceinline__ bool log64_special(double x, double& res) {
  const bool nan = x != x;
  const bool nonpos = x <= 0.0;
  const bool inf = x == INFINITY;
  const bool one = x == 1.0;
  double v = one ? 0.0 : (inf ? INFINITY : __longlong_as_double(0x7ff8000000000000ll));
  v = x == 0.0 ? -INFINITY : v;
  res = nan ? __longlong_as_double(__double_as_longlong(x) | 0x0008000000000000ll) : v;
  return nan | nonpos | inf | one;
}

struct Log64Setup {
  double m, c;
  int e2, j;
};

__device__ __forceinline__ Log64Setup log64_setup(double x) {
  Log64Setup S;
  bool sub = x < 0x1p-1022;
  double xs = sub ? x * 0x1p64 : x;
  int hi = __double2hiint(xs);
  S.j = (hi >> 16) & 15;
  int fold = S.j >> 3;
  S.e2 = ((hi >> 20) & 0x7ff) - 1023 + fold - (sub ? 64 : 0);
  S.m = __hiloint2double((hi & 0x000fffff) | ((1023 - fold) << 20), __double2loint(xs));
  return S;
}

// Main-path error, split by where it arises:
//  * tail = t2.hi^2 sp stands for t^4 S(t): t2.hi carries t^2 within 3u
//    (u = 2^-53; within u when c_j = 1, where t.lo = 0), the square, the
//    Horner evaluation of S at t.hi (at most 1.2u relative: s0 = -1/4
//    dominates, |s1 t / s0| < 0.06) and the product each one more rounding:
//    below 9.2u = 2^-49.8 of |tail| in all.  S's own fit error is at most
//    t^4 sup|g - S| (g the exact quotient; below 2^-57 t^4, checked in the
//    bound tests) = 2^-55 of |tail|, and adding tail to b3.lo one more u of
//    it.  LOG64_TAIL_EPS = 2^-49 covers the sum with a factor 1.6 to spare.
//  * the rest: t, t^2/2 and t^3/3 in double-double (relative 2^-100), the
//    table -ln c_j and e' ln2 to 2^-106, the double-double sums (2^-101):
//    below 2^-99 |y|, where LOG64_EPS = 2^-70 leaves room for the test's own
//    roundings.
// The bound is therefore |tail| 2^-49 + |y| 2^-70.  Where c_j = 1 and e' = 0,
// y = log1p t is small (|t| up to 1/16, |y| down to 2^-4.05) and the tail
// term dominates; elsewhere |y| >= 0.03 and the test is close to 2^-70 |y|.
constexpr double LOG64_TAIL_EPS = 0x1p-49;
constexpr double LOG64_EPS = 0x1p-70;

__device__ __forceinline__ double log64_fast(double x, const Log64Tab& tb, bool& ok) {
  Log64Setup S = log64_setup(x);
  double c = tb.c[S.j];
  double4 L = tb.L[S.j];
  dd p = two_prod(S.m, c);
  dd t = fast_two_sum(p.hi - 1.0, p.lo);  // exact: p.hi - 1 is exact
  // log1p t = t - t^2/2 + t^3/3 + t^4 S(t)
  dd t2 = two_prod(t.hi, t.hi);
  t2.lo = fma(2.0 * t.hi, t.lo, t2.lo);
  // t^3/3 as an unnormalised double-double (dd_add_ord below renormalises):
  // t2.hi t.hi exactly by TwoProd, the cross terms t2.hi t.lo + t2.lo t.hi
  // added by fmas (t2.lo t.lo, below 2^-106 |t|^3, dropped), then the same
  // with 1/3 = THIRD_HI + THIRD_LO: within 10u^2 relative, as two dd_mul
  dd b3;
  {
    const dd p3 = two_prod(t2.hi, t.hi);
    const double p3l = fma(t2.lo, t.hi, fma(t2.hi, t.lo, p3.lo));
    b3 = two_prod(p3.hi, THIRD_HI);
    b3.lo = fma(p3l, THIRD_HI, fma(p3.hi, THIRD_LO, b3.lo));
  }
  double sp = LOG64_S[LOG64_S_DEG];
#pragma unroll
  for (int i = LOG64_S_DEG - 1; i >= 0; i--) sp = fma(sp, t.hi, LOG64_S[i]);
  double tail = t2.hi * t2.hi * sp;
  // |t| <= 1/16: t dominates t^2/2, which dominates t^3/3 + t^4 S(t)
  dd l1 = dd_add_ord(t, dd{-0.5 * t2.hi, -0.5 * t2.lo});
  l1 = dd_add_ord(l1, dd{b3.hi, b3.lo + tail});
  // e' ln2 - ln c_j: |e' ln2| >= ln2 > |ln c_j| unless e' = 0; the total does
  // not cancel (|y| >= 0.03 unless e' = 0 and c_j = 1, where y = l1 exactly)
  double ed = (double)S.e2;
  dd el = dd_mul_d(dd{LN2_TD[0].x, LN2_TD[0].y}, ed);
  dd y = dd_add_nc(dd_add_ord(el, dd{L.x, L.y}), l1);
  double e = fma(fabs(tail), LOG64_TAIL_EPS, fabs(y.hi) * LOG64_EPS);
  double a = y.hi + (y.lo - e);
  double b = y.hi + (y.lo + e);
  ok = a == b;
  double res = b, spv;
  if (log64_special(x, spv)) {
    res = spv;
    ok = true;
  }
  return res;
}

// Middle path (double-double), tried first by the accurate path: t = m c - 1
// exact as in the main path, s = t/(2 + t) in double-double (two divisions,
// |s| < 1/31), log1p t = 2 atanh(s) by its series to s^21 (remainder below
// 2^-105 relative), terms 6..10 in binary64 (rounding below 2^-107) and 0..5
// by double-double Horner steps in s^2; then e' ln2 + (-log c_j) + log1p t in
// double-double (ln2 and the table to 2^-106).  y is within 2^-100 of log x
// relative (|y| >= 0.03 unless e' = 0 and c_j = 1, where y = log1p t); the
// test allows 2^-95.
__device__ __forceinline__ double log64_mid(double x, const Log64Tab& tb, bool& ok) {
  Log64Setup S = log64_setup(x);
  double c = tb.c[S.j];
  double4 L = tb.L[S.j];
  dd p = two_prod(S.m, c);
  dd t = fast_two_sum(p.hi - 1.0, p.lo);
  dd den = dd_add_d(t, 2.0);
  double q1 = t.hi / den.hi;
  dd rr = dd_add(t, dd_neg(dd_mul_d(den, q1)));  // t - q1 (2 + t)
  dd s = fast_two_sum(q1, rr.hi / den.hi);
  dd s2 = dd_mul(s, s);
  double P = INV_ODD_DD[10].x;
#pragma unroll
  for (int k = 9; k >= 6; k--) P = fma(P, s2.hi, INV_ODD_DD[k].x);
  dd w = {P, 0.0};
#pragma unroll
  for (int k = 5; k >= 0; k--) w = dd_add_ord(dd{INV_ODD_DD[k].x, INV_ODD_DD[k].y}, dd_mul(s2, w));
  dd l = dd_mul(s, w);
  l = {2.0 * l.hi, 2.0 * l.lo};
  dd el = dd_mul_d(dd{LN2_TD[0].x, LN2_TD[0].y}, (double)S.e2);
  dd y = dd_add(dd_add(el, dd{L.x, L.y}), l);
  double e = fabs(y.hi) * 0x1p-95;
  double a = y.hi + (y.lo - e);
  double b = y.hi + (y.lo + e);
  ok = a == b;
  return b;
}

__device__ __noinline__ AccResultD log64_accurate(double x, const Log64Tab& tb) {
  double sp;
  if (log64_special(x, sp)) return {sp, 1};
  bool mid_ok;
  const double rm = log64_mid(x, tb, mid_ok);
  if (mid_ok) return {rm, 1};
  // triple-double path
  Log64Setup S = log64_setup(x);
  double c = tb.c[S.j];
  dd p = two_prod(S.m, c);
  dd t = fast_two_sum(p.hi - 1.0, p.lo);
  td tt = td_from_dd(t);
  // log1p t = 2 atanh(s), s = t/(2 + t), |s| < 1/32: series to s^29 (< 2^-145)
  td s = td_div(tt, td_add(tt, td_from(2.0)));
  td s2 = td_mul(s, s);
  dd s2d = {s2.h, s2.m};
  dd ph = {INV_ODD_DD[ATANH64_N].x, INV_ODD_DD[ATANH64_N].y};
#pragma unroll
  for (int k = ATANH64_N - 1; k >= 6; k--)
    ph = dd_add(dd_mul(ph, s2d), dd{INV_ODD_DD[k].x, INV_ODD_DD[k].y});
  td pt = td_from_dd(ph);
#pragma unroll
  for (int k = 5; k >= 0; k--) pt = td_add(td_mul(pt, s2), td_ld(INV_ODD_TD[k]));
  td l = td_scale(td_mul(pt, s), 2.0);
  td y = td_add(td_add(td_mul_d(td_ld(LN2_TD[0]), (double)S.e2), td_ld(tb.L[S.j])), l);
  double e = fabs(y.h) * 0x1p-135;
  bool ok;
  double res = round64_tail(y.h, y.m, y.l, e, ok);
  return {res, ok ? 1 : 0};
}

// ------------------------------------------------- log, 128-entry table
// The paper's cr_log main path (Sec. II-B): a short reciprocal rcp of the
// mantissa m in [0.75, 1.5) and ONE 64-bit table read per element, a scaled
// integer that becomes a double-double.  Here rcp is the hardware binary32
// reciprocal of m rounded to 8 significant bits, so it takes the 128 binary32
// values with encodings (0x3F2B + j) << 16, j = 0..127 (0.66796875 ..
// 1.328125; the one value above, reached from m just above 0.75 only, is
// clamped to j = 127), and |t| = |m rcp - 1| <= 2^-8 (1 + 2^-12).  With
// r = rcp - 1 (exact) the entry holds T = log1p(r)/r - 1 as the integer
// nearest to T 2^65, so -ln rcp = -(r + r T) and
//   ln x = e' ln2 - (r + r Th) - r Tl + log1p(t),
// T = Th + Tl from the integer's two 32-bit halves; r + r Th and r Tl are
// exact (8 x 32-bit products on the 2^-41 and 2^-73 grids).  log1p t =
// t - t^2/2 + t^3/3 + t^4 S(t) with S of low degree (|t| <= 2^-8).
// The accurate path is the 16-entry one above (log64_accurate).
struct Log128Tab {
  long long T[128];
  Log64Tab acc;
};

__device__ __forceinline__ void log128_tab_load(Log128Tab& t, int tid) {
  if (tid < 128) t.T[tid] = LOG128_T[tid];
  log64_tab_load(t.acc, tid);
}

// Main-path error, relative to y (|y| >= 0.28 when e' != 0; when e' = 0,
// |y| >= |r|/2 (1 - 2^-12): m then lies in the rounding interval of rcp, at
// least half a spacing of 8-bit values away from 1/1 = 1, and |y| >= 0.99 |t|
// when r = 0):
//  * the table: T to 2^-66, so -ln rcp within |r| 2^-66 <= 2^-64.97 |y|;
//  * t^3/3 in binary64 (t2.hi t.hi THIRD: about 3.5 units of 2^-53 of
//    |t|^3/3 <= 2^-68.8 |t|) and t^4 S (below 2^-75 |t|), |t| <= 2 |y| when
//    r != 0: within 2^-67.8 |y|;
//  * t^2/2 and the sums in double-double, e' ln2 to 2^-106: below 2^-98 |y|.
// In all below 2^-64.6 |y|; the test allows 2^-64 |y|.
constexpr double LOG128_EPS = 0x1p-64;

__device__ __forceinline__ double log128_fast(double x, const Log128Tab& tb, bool& ok) {
  Log64Setup S = log64_setup(x);
  const float ra = __builtin_amdgcn_rcpf((float)S.m);
  int j = (int)((f32_bits(ra) + 0x8000u) >> 16) - 0x3F2B;
  j = j > 127 ? 127 : (j < 0 ? 0 : j);
  const double rcp = (double)bits_f32((uint32_t)(0x3F2B + j) << 16);
  const long long Ti = tb.T[j];
  const double Th = (double)(int)(Ti >> 32) * 0x1p-33;
  const double Tl = (double)(uint32_t)Ti * 0x1p-65;
  const double r = rcp - 1.0;
  dd A = fast_two_sum(-(r + r * Th), -(r * Tl));  // -ln rcp
  dd p = two_prod(S.m, rcp);
  dd t = fast_two_sum(p.hi - 1.0, p.lo);  // exact: p.hi in [1 - 2^-7, 1 + 2^-7]
  dd t2 = two_prod(t.hi, t.hi);
  t2.lo = fma(2.0 * t.hi, t.lo, t2.lo);
  double sp = LOG128_S[LOG128_S_DEG];
#pragma unroll
  for (int i = LOG128_S_DEG - 1; i >= 0; i--) sp = fma(sp, t.hi, LOG128_S[i]);
  const double b3 = (t2.hi * t.hi) * THIRD_HI + t2.hi * t2.hi * sp;
  dd l = dd_add_ord(t, dd{-0.5 * t2.hi, -0.5 * t2.lo});
  l = fast_two_sum(l.hi, l.lo + b3);
  dd el = dd_mul_d(dd{LN2_TD[0].x, LN2_TD[0].y}, (double)S.e2);
  dd y = dd_add_nc(dd_add_nc(el, A), l);
  double e = fabs(y.hi) * LOG128_EPS;
  double a = y.hi + (y.lo - e);
  double b = y.hi + (y.lo + e);
  ok = a == b;
  double res = b, spv;
  if (log64_special(x, spv)) {
    res = spv;
    ok = true;
  }
  return res;
}

}  // namespace cr
