// cr_f32_log.h -- correctly rounded logf, log2f, log10f, log1pf (device).
//
// Paper, Sec. II-A and Fig. 2 (cr_log2f): the mantissa is brought into
// [0.75, 1.5), a few leading mantissa bits select table entries, and a
// polynomial in the reduced argument plus the exponent term reconstruct the
// result.  Here the table holds a 9-bit reciprocal c_j of each sub-interval
// (16 entries) and -log_b(c_j) as a double-double, so that
//     x = 2^e' m,  m in [0.75, 1.5),  t = m c_j - 1  (exact: 24 + 9 bits),
//     log_b(x) = e' log_b(2) + (-log_b c_j) + K t + t Q(t),
// with K = 1/ln b on 20 bits (K t exact) and Q a minimax polynomial on
// t in [-1/32, 1/16].  c_j = 1 on the two sub-intervals next to 1, so for x
// near 1 the result is K t + t Q(t) with no cancellation.  log1pf reduces
// u = RN(1 + x) the same way.  1 + x is exact for binary32 x unless |x| < 2^-29
// or x >= 2^29.  The fast path returns x itself for |x| < 2^-25 (the correctly
// rounded result there, see log1p_special_fast); for x >= 2^29, log(u) differs
// from log(1 + x) by less than 2^-53 while the result exceeds 20 (ulp 2^-48).
// The accurate path adds the rounding error of u, scaled like m, to t instead.
//
// The binary64 fast path ends with the rounding test of cr_round.h; lanes that
// fail it run the accurate double-double path below (the log1p series to degree
// 17 on the exact double-double t), as in the exponential family.
#pragma once
#include "cr_consts.h"
#include "cr_round.h"

namespace cr {

enum { LOGK_E = 0, LOGK_2 = 1, LOGK_10 = 2, LOGK_1P = 3 };

// One 32-byte row per sub-interval, so that the reads of a lookup share one
// address (j 32) and differ only in their immediate offsets.  -log_b(c_j) =
// L.x + L.y + z with L.x a multiple of 2^-44 (2^-45 for log10): e' log_b(2)
// plus L.x is exact in the fast path; the accurate paths add z back.
struct LogRow {
  double2 L;  // -log_b(c_j): high part, next 53 bits
  double c;   // c_j
  double z;   // the rest of -log_b(c_j)
};
struct LogTab {
  LogRow row[16];
};

template <int K>
__device__ __forceinline__ void log_tab_load(LogTab& t, int tid) {
  if (tid < 16) {
    t.row[tid].L = (K == LOGK_2) ? LOG2_L[tid] : (K == LOGK_10) ? LOG10_L[tid] : LOGE_L[tid];
    t.row[tid].c = LOG_C[tid];
    t.row[tid].z = (K == LOGK_2) ? LOG2_LZ[tid] : (K == LOGK_10) ? LOG10_LZ[tid] : LOGE_LZ[tid];
  }
}

// Fast-path error (t and K t are exact: t is a multiple of 2^-33 below 1/16,
// K has 20 bits).  Q's approximation error (below 2^-57.6) and its Horner
// evaluation error (below 2^-52 |Q|, |Q| < 0.05) enter through t Q, which is
// rounded once inside inner = t Q + lo (< 2^-53 |inner|; lo, the low parts of
// e' log_b(2) and -log_b(c_j), is below 2^-43 and rounded once, the table's
// third part, below 2^-97, is dropped); s = K t + inner is rounded once (half
// an ulp of s, at most 2^-57) and yh = Ah + s once more (half an ulp of y).  Summed per interval of the reduction, for e' = 0 (where |y| can be
// as small as 0.0128 while |s| is not) and e' != 0, over a fine grid of each
// interval and the three bases, the total stays below 0.82 ulp of y.  A y just
// above a power of two may give a yh just below it, whose ulp is half as large:
// the bound is 1.64 ulps of yh.  log1p adds, for x >= 2^29, the rounding of
// 1 + x (below 2^-53 absolute on y > 20: a thirtieth of an ulp): 0.85 ulp of
// y, 1.7 of yh.  Both are below 2, so the bit test rejects yh only when its low
// bits lie within 1 of the boundary pattern (E = 1).  Every binary32 input is
// checked against the accurate path on the GPU.
constexpr unsigned LOG_TEST_E = 1;

template <int K>
__device__ __forceinline__ double log_C_hi() {
  return K == LOGK_2 ? 1.0 : K == LOGK_10 ? LOG10_C_HI : LOGE_C_HI;
}
template <int K>
__device__ __forceinline__ double log_C_lo() {
  return K == LOGK_2 ? 0.0 : K == LOGK_10 ? LOG10_C_LO : LOGE_C_LO;
}
template <int K>
__device__ __forceinline__ double log_K() {
  return K == LOGK_2 ? LOG2_K : K == LOGK_10 ? LOG10_K : 1.0;
}
template <int K>
__device__ __forceinline__ double log_Q(double t) {
  if (K == LOGK_2) {
    double p = LOG2_Q[LOG2_Q_DEG];
#pragma unroll
    for (int i = LOG2_Q_DEG - 1; i >= 0; i--) p = fma(p, t, LOG2_Q[i]);
    return p;
  } else if (K == LOGK_10) {
    double p = LOG10_Q[LOG10_Q_DEG];
#pragma unroll
    for (int i = LOG10_Q_DEG - 1; i >= 0; i--) p = fma(p, t, LOG10_Q[i]);
    return p;
  } else {
    double p = LOGE_Q[LOGE_Q_DEG];
#pragma unroll
    for (int i = LOGE_Q_DEG - 1; i >= 0; i--) p = fma(p, t, LOGE_Q[i]);
    return p;
  }
}

// log1p(t) for the accurate path of the binary32 functions: a double-double
// t with |t| <= 1/16, to within 2^-69.9 |t|.  The series to degree 17
// (remainder below 2^-72.2 |t|) as t (1 + t (-1/2 + t (1/3 + t (-1/4 +
// t R(t))))), with R = sum over n = 5..17 of (-1)^(n+1) t^(n-5) / n in
// binary64 (its rounding, below 2^-54.3, is multiplied by |t|^4 <= 2^-16) and
// the four outer steps in double-double.
__device__ __forceinline__ dd log1p_dd_short(dd t) {
  double R = 1.0 / 17;
#pragma unroll
  for (int n = 16; n >= 5; n--) R = fma(R, t.hi, (n & 1 ? 1.0 : -1.0) / n);
  dd w = two_prod(t.hi, R);
  w.lo = fma(t.lo, R, w.lo);
  w = dd_add_ord(dd{-0.25, 0.0}, w);  // |t R| < 1/64
  w = dd_add_ord(dd{THIRD_HI, THIRD_LO}, dd_mul(t, w));
  w = dd_add_ord(dd{-0.5, 0.0}, dd_mul(t, w));
  w = dd_add_ord(dd{1.0, 0.0}, dd_mul(t, w));
  return dd_mul(t, w);
}

// Shared set-up: u (= x, or 1 + x for log1pf), the decomposition u = 2^e' m
// with m in [0.75, 1.5), the table entries and the reduced argument t.
struct LogSetup {
  double u, m, c, t, z;
  double2 L;
  int e2;
};

// -log_b(c_j) as a double-double for the accurate paths: hi + lo by Fast2Sum
// (exact; |lo| < 2^-44 <= |hi| unless both are 0), then the third part
__device__ __forceinline__ dd log_table_dd(const LogSetup& S) {
  dd l = fast_two_sum(S.L.x, S.L.y);
  l.lo += S.z;
  return l;
}

template <int K>
__device__ __forceinline__ LogSetup log_setup(float xf, const LogTab& tb) {
  LogSetup S;
  double x = (double)xf;
  S.u = (K == LOGK_1P) ? 1.0 + x : x;
  // u = 2^e m, m in [1,2); index j = top 4 fraction bits; fold m >= 1.5 to m/2
  int hi = __double2hiint(S.u);
  int j = (hi >> 16) & 15;
  int fold = j >> 3;
  S.e2 = ((hi >> 20) & 0x7ff) - 1023 + fold;
  S.m = __hiloint2double((hi & 0x000fffff) | ((1023 - fold) << 20), __double2loint(S.u));
  S.c = tb.row[j].c;
  S.L = tb.row[j].L;
  S.z = tb.row[j].z;
  S.t = fma(S.m, S.c, -1.0);
  return S;
}

// NaN (quieted), u <= 0 (-inf at 0, NaN below), u = +inf, log1p(+-0) = +-0,
// decided on the binary32 argument (u = 1 + x is exact for x in [-1, 1], so
// u <= 0 exactly when x <= -1).
// Branch-free: res is always written (meaningful only when true is returned).
template <int K>
__device__ __forceinline__ bool log_special(float xf, float& res) {
  const bool nan = xf != xf;
  const float lim = K == LOGK_1P ? -1.0f : 0.0f;  // log1p(-1) = log(+-0) = -inf
  const bool zero1p = K == LOGK_1P && xf == 0.0f;
  const bool dom = xf <= lim;
  const bool inf = xf == INFINITY;
  float v = inf ? INFINITY : (xf == lim ? -INFINITY : bits_f32(0x7fc00000u));
  v = zero1p ? xf : v;
  res = nan_or(xf, v);
  return nan | zero1p | dom | inf;
}

// The fast path's special cases for logf, log2f and log10f, in fewer
// operations: one class test picks the inputs that are not positive finite
// (NaN, infinities, zeros, negatives), and the hardware base-2 logarithm gives
// their results (measured on gfx950: -inf at +-0, +inf at +inf, a NaN quieted
// with its payload and sign) except for negative inputs, where it returns the
// negative default NaN and the positive one is wanted.  The accurate path keeps
// log_special; the exhaustive test compares both on every encoding.
__device__ __forceinline__ bool log_special_fast(float xf, float& res) {
  const float h = __builtin_amdgcn_logf(xf);
  res = xf < 0.0f ? bits_f32(0x7fc00000u) : h;
  return __builtin_amdgcn_class(xf, 0x27f);  // all classes but +denormal, +normal
}

// The fast path's special cases for log1pf, without a transcendental
// instruction: NaN (returned quieted: canonicalize quiets a signaling NaN and
// keeps the payload and sign), +inf (itself), x = -1 (-inf), x < -1 (the
// default NaN), and the tiny arguments |x| < 2^-25, zeros and subnormals
// included, whose result is x itself: log1p x = x - x^2/2 + ... lies within
// x^2/2 <= 2^-26 |x| of x, below half the spacing of the binary32 numbers on
// either side of x (at least 2^-24 |x|), so it rounds to x.  With these out of
// the way 1 + x is exact in binary64 for every remaining x below 2^29, and the
// result is a normal binary32 number, as the bit test requires.
__device__ __forceinline__ bool log1p_special_fast(float xf, float& res) {
  const uint32_t q = f32_bits(__builtin_canonicalizef(xf));
  // integer selects: as float conditionals the compiler branches around them
  const uint32_t v = f32_bits(xf) == 0xbf800000u ? 0xff800000u : 0x7fc00000u;
  res = bits_f32(xf <= -1.0f ? v : q);
  // NaN and infinities (class mask), tiny arguments, everything at or below -1
  return __builtin_amdgcn_class(xf, 0x207) | (fabsf(xf) < 0x1p-25f) | (xf <= -1.0f);
}

template <int K>
__device__ __forceinline__ float log_fast(float xf, const LogTab& tb, bool& ok) {
  LogSetup S = log_setup<K>(xf, tb);
  double t = S.t;
  double Q = log_Q<K>(t);
  double ed = (double)S.e2;
  // e' log_b(2) + (-log_b c_j), high parts: C_hi has 44 bits and e' at most 8,
  // both terms are multiples of 2^-44 (2^-45 for log10) and their sum is
  // below 2^8 in magnitude, so the fma is exact
  const double Ah = fma(ed, log_C_hi<K>(), S.L.x);
  const double lo = K == LOGK_2 ? S.L.y : fma(ed, log_C_lo<K>(), S.L.y);
  double inner = fma(t, Q, lo);
  double yh = Ah + fma(log_K<K>(), t, inner);
  // logf, log2f and log10f round to normal binary32 numbers (or to +0 at 1),
  // log1pf too except for subnormal x, which are left to the accurate path
  float res = round_f32_bits<LOG_TEST_E>(yh, ok);
  float sp;
  if (K == LOGK_1P ? log1p_special_fast(xf, sp) : log_special_fast(xf, sp)) {
    res = sp;
    ok = true;
  }
  return res;
}

// Accurate path: t rebuilt exactly as a double-double (plus, for log1pf, the
// rounding error of u = 1 + x scaled like m), then
// y = e' log_b 2 + (-log_b c_j) + log1p(t) / ln b in double-double.
template <int K>
__device__ __noinline__ AccResult log_accurate(float xf, const LogTab& tb) {
  LogSetup S = log_setup<K>(xf, tb);
  float sp;
  if (log_special<K>(xf, sp)) return {sp, 1};
  dd p = two_prod(S.m, S.c);
  dd t = fast_two_sum(p.hi - 1.0, p.lo);  // p.hi - 1 is exact (p.hi in [0.96, 1.07])
  if (K == LOGK_1P) {
    // (1 + x) - u exactly (TwoSum), scaled like m
    const double ulo = two_sum(1.0, (double)xf).lo * pow2i(-S.e2);
    t = dd_add_d(t, ulo * S.c);
  }
  dd l = log1p_dd_short(t);
  if (K == LOGK_2) l = dd_mul(l, dd{INV_LN2_HI, INV_LN2_LO});
  if (K == LOGK_10) l = dd_mul(l, dd{INV_LN10_HI, INV_LN10_LO});
  dd C = K == LOGK_2 ? dd{1.0, 0.0}
                     : K == LOGK_10 ? dd{LOG10_2_HI, LOG10_2_LO} : dd{LN2_HI, LN2_LO};
  dd y = dd_add(dd_mul_d(C, (double)S.e2), log_table_dd(S));
  y = dd_add(y, l);
  // log1p(t) is within 2^-69.9 |t|, and |t| <= 4.9 |y| (|y| >= 0.0128 unless
  // e' = 0 and c_j = 1, where y is log1p(t) / ln b): y is within 2^-67.5 of
  // its value relative, below the 2^-66.8 that separates the hardest binary32
  // case from a rounding boundary (log1pf, at 2^-42.8 ulp)
  bool ok;
  float r = round_f32_dd(y.hi, y.lo, 0x1p-67, ok);
  return {r, ok ? 1 : 0};
}

}  // namespace cr
