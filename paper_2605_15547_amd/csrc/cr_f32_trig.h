// cr_f32_trig.h -- correctly rounded sinf, cosf, sincosf, tanf (device).
//
// Paper, Sec. II-A: the trigonometric kernels branch only for large-argument
// reduction.  On the GPU every lane runs the same reduction, branch-free:
// Payne-Hanek (Payne and Hanek, SIGNUM Newsletter 18(1), 1983) in 32-bit
// integer arithmetic for every |x| >= pi/64.
//
//   x = M 2^E (M a 24-bit integer).  N = x 32/pi = M 2^(E+4) sum_i g_i 2^-i
//   with g_i the bits of 2/pi.  Bits with i <= E - 2 only add multiples of 64
//   to N, so a 160-bit window W of 2/pi starting at bit E - 1 suffices:
//   N = M W 2^-154 (mod 64), truncation error < 2^24 2^-154 = 2^-130.
//   The window is read from an 11-word table (two zero words, then 288 bits
//   of 2/pi) with funnel shifts; the binary point of P = M W is always bit
//   154.  The zero words let the window start before the binary point, so the
//   reduction is also right for small arguments (down to 2^-37).
//
//   k = nearest(N), q = k mod 64, f = N - k in [-1/2, 1/2) (64 fraction bits
//   for the fast path, 128 for the accurate path), r = f pi/32, |r| <= pi/64.
//   With theta = q pi/32 = quad pi/2 + j pi/32 (j = q mod 16), a 16-entry table
//   gives sin and cos of j pi/32 (double-double); quadrant symmetries give
//   sin/cos theta, and
//       sin x = sin theta cos r + cos theta sin r,
//       cos x = cos theta cos r - sin theta sin r,   tan x = sin x / cos x.
//   Near the zeros of sin/cos (j = 0) the table terms are exactly 0 and +-1,
//   so the result is +-sin r or +-cos r without cancellation.
#pragma once
#include "cr_consts.h"
#include "cr_round.h"

namespace cr {

enum { TRIGK_SIN = 0, TRIGK_COS = 1, TRIGK_TAN = 2, TRIGK_SINCOS = 3 };

struct TrigTab {
  double4 sc[16];
  unsigned w[11];
};

__device__ __forceinline__ void trig_tab_load(TrigTab& t, int tid) {
  if (tid < 16) t.sc[tid] = SINCOS_T[tid];
  if (tid < 11) t.w[tid] = TWO_OVER_PI_W[tid];
}

struct Reduced {
  int q;                  // k mod 64
  long long fhi;          // f = (fhi + flo 2^-64) 2^-64, signed
  unsigned long long flo;
};

// The 32-bit words of the window W that starts at bit sp of the zero-prefixed
// bit string of 2/pi: word k is bits [sp + 32k, sp + 32k + 32), the funnel
// shift of w[b + k] and w[b + k + 1] right by c, with b = ceil(sp / 32) - 1 and
// c = -sp mod 32 (c = 0 when sp is a multiple of 32: word k is then
// w[b + k + 1] itself), so that the shift count stays in [0, 31].
struct Window {
  int b;
  unsigned c;
};
__device__ __forceinline__ Window window_of(int sp) {
  return {((sp + 31) >> 5) - 1, (unsigned)(-sp) & 31u};
}
// ((hi:lo) >> c) mod 2^32 for c in [0, 31]: one funnel shift
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, unsigned c) {
  return __builtin_amdgcn_alignbit(hi, lo, c);
}
__device__ __forceinline__ uint32_t window_word(uint32_t hi, uint32_t lo, unsigned c) {
  return funnel(hi, lo, c);
}

// Payne-Hanek reduction of |x| (ax = its encoding), 2^-37 <= |x| finite;
// other encodings are clamped to in-range table indices (their result is
// discarded by the caller).
__device__ __forceinline__ Reduced payne_hanek(uint32_t ax, const unsigned* w) {
  int E = (int)(ax >> 23) - 150;
  E = E < -60 ? -60 : (E > 105 ? 105 : E);
  uint32_t M = (ax & 0x007fffffu) | 0x00800000u;
  const Window win = window_of(E - 2 + 64);  // window start: [2, 167]
  const unsigned* t = w + win.b;             // words b .. b + 5 <= 10
  uint32_t W0 = window_word(t[0], t[1], win.c);
  uint32_t W1 = window_word(t[1], t[2], win.c);
  uint32_t W2 = window_word(t[2], t[3], win.c);
  uint32_t W3 = window_word(t[3], t[4], win.c);
  uint32_t W4 = window_word(t[4], t[5], win.c);
  // P = M W, least significant word first (each step is one 32x32+64 multiply-add)
  uint64_t a = (uint64_t)M * W4;
  uint32_t p0 = (uint32_t)a;
  a = (uint64_t)M * W3 + (a >> 32);
  uint32_t p1 = (uint32_t)a;
  a = (uint64_t)M * W2 + (a >> 32);
  uint32_t p2 = (uint32_t)a;
  a = (uint64_t)M * W1 + (a >> 32);
  uint32_t p3 = (uint32_t)a;
  a = (uint64_t)M * W0 + (a >> 32);
  uint32_t p4 = (uint32_t)a;
  // integer bits 154..159 = p4[31:26]; fraction bits 153..26, by 32-bit words
  // the funnel shifts of (p4:p3), (p3:p2), (p2:p1), (p1:p0) right by 26
  Reduced R;
  R.q = (int)((((p4 >> 25) + 1) >> 1) & 63);  // round to nearest: + fraction bit 153
  R.fhi = (long long)(((uint64_t)funnel(p4, p3, 26) << 32) | funnel(p3, p2, 26));  // f - 1 when f >= 1/2
  R.flo = ((uint64_t)funnel(p2, p1, 26) << 32) | funnel(p1, p0, 26);
  return R;
}

// The fast path's form of the same reduction: only the 96 leading bits of the
// window (W0, W1, W2), so P' = M (W >> 64) takes three multiply-adds instead
// of five.  P' is bits 64.. of P less the carry of M (W mod 2^64) < 2^88 out
// of the dropped low part, i.e. less than 2^-66 in units of N; the 64
// fraction bits of f (bits 153..90 of P) come out low by at most one unit of
// 2^-64 (the high word R.fhi only; R.flo is not formed).
__device__ __forceinline__ Reduced payne_hanek_fast(uint32_t ax, const unsigned* w) {
  // the window of payne_hanek from the exponent field directly: with the
  // field clamped below at 90 (E = field - 150 >= -60; the field is at most
  // 255, so the upper clamp never applies), the window starts at
  // sp = field - 88, so b = ((field - 57) >> 5) - 1 and c = (88 - field) mod 32
  const int fe = max((int)(ax >> 23), 90);
  const Window win = {((fe - 57) >> 5) - 1, (unsigned)(88 - fe)};  // c: low 5 bits used
  uint32_t M = (ax & 0x007fffffu) | 0x00800000u;
  const unsigned* t = w + win.b;
  uint32_t W0 = window_word(t[0], t[1], win.c);
  uint32_t W1 = window_word(t[1], t[2], win.c);
  uint32_t W2 = window_word(t[2], t[3], win.c);
  uint64_t a = (uint64_t)M * W2;
  uint32_t p2 = (uint32_t)a;
  a = (uint64_t)M * W1 + (a >> 32);
  uint32_t p3 = (uint32_t)a;
  a = (uint64_t)M * W0 + (a >> 32);
  uint32_t p4 = (uint32_t)a;
  Reduced R;
  // k mod 64 = (bits 159..153 of P, plus 1) >> 1: the same as (p4 + 2^25) >> 26,
  // where a carry out of bit 31 would only add 64
  R.q = (int)((p4 + 0x02000000u) >> 26);
  R.fhi = (long long)(((uint64_t)funnel(p4, p3, 26) << 32) | funnel(p3, p2, 26));
  R.flo = 0;
  return R;
}

// sin/cos of theta = q pi/32 as double-doubles, from the table and the quadrant
struct SinCosTheta {
  double sh, sl, ch, cl;
};

__device__ __forceinline__ SinCosTheta theta_of(int q, const TrigTab& tb) {
  // quad 0: (S, C); 1: (C, -S); 2: (-S, -C); 3: (-C, S).  The swap of odd
  // quadrants picks which half of the 32-byte table row is read for each
  // pair (an address offset instead of selects on four doubles), and the
  // signs are flipped on the sign bits.
  const int quad = q >> 4;
  const int swap = quad & 1;
  const double2* row = reinterpret_cast<const double2*>(&tb.sc[q & 15]);
  const double2 S = row[swap], C = row[swap ^ 1];
  const long long ms = (long long)(quad >= 2) << 63;
  const long long mc = (long long)(quad == 1 || quad == 2) << 63;
  SinCosTheta r;
  r.sh = __longlong_as_double(__double_as_longlong(S.x) ^ ms);
  r.sl = __longlong_as_double(__double_as_longlong(S.y) ^ ms);
  r.ch = __longlong_as_double(__double_as_longlong(C.x) ^ mc);
  r.cl = __longlong_as_double(__double_as_longlong(C.y) ^ mc);
  return r;
}

// Branch-free: res is always written (meaningful only when true is returned).
__device__ __forceinline__ bool trig_special(float xf, float& res, int kind) {
  const bool nan = xf != xf;
  const bool inf = (f32_bits(xf) & 0x7fffffffu) == 0x7f800000u;
  const bool zero = xf == 0.0f;
  float v = zero ? (kind == TRIGK_COS ? 1.0f : xf) : bits_f32(0x7fc00000u);  // sin, tan keep -0
  res = nan_or(xf, v);
  return nan | inf | zero;
}

// The fast path's special cases, with the tiny arguments folded in: for
// |x| < 2^-12 (zeros and subnormals included) sin x = x - x^3/6 + ... and
// tan x = x + x^3/3 + ... lie within x^2/3 < 2^-25.6 |x| of x and cos x =
// 1 - x^2/2 + ... within 2^-25 of 1, less than half the spacing of the
// binary32 numbers next to x (at least 2^-24 |x|) or below 1 (2^-24), so the
// correctly rounded results are x and 1.  NaN is returned quieted
// (canonicalize quiets it and keeps the payload), infinities give the
// default NaN.  One class test and a magnitude compare pick these lanes.
__device__ __forceinline__ bool trig_special_fast(float xf, float& res, int kind) {
  const bool inf = fabsf(xf) == INFINITY;
  const float q = __builtin_canonicalizef(xf);
  const float t = (kind == TRIGK_COS && xf == xf) ? 1.0f : q;
  res = inf ? bits_f32(0x7fc00000u) : t;
  return __builtin_amdgcn_class(xf, 0x207) | (fabsf(xf) < 0x1p-12f);
}

// v with its sign flipped where the mask m has bit 31 set (one operation on
// the high word)
__device__ __forceinline__ double flip(double v, uint32_t m) {
  return __hiloint2double(__double2hiint(v) ^ (int)(m & 0x80000000u), __double2loint(v));
}

// Fast path: binary64 sin and cos of |x| up to the quadrant's signs, with
// absolute error bounds: sin |x| is s with its sign flipped by the mask ss
// (bit 31), cos |x| is c flipped by sc.
struct TrigFast {
  double s, c, es, ec;  // values and error bounds
  uint32_t ss, sc;      // sign masks
};

__device__ __forceinline__ TrigFast trig_fast_core(float xf, const TrigTab& tb) {
  uint32_t ax = f32_bits(xf) & 0x7fffffffu;
  double axd = (double)bits_f32(ax);
  double r;
  int q;
  // The one branch of the method is on the size of the argument (the paper
  // keeps Payne-Hanek for large arguments only): when every lane of the wave
  // has |x| < 2^23, the wave takes a Cody-Waite reduction in binary64
  // instead, k = nearest(|x| 32/pi) (|k| < 2^26.4), r = ((|x| - k C1) - k C2)
  // - k C3 with C1 on 26 bits (k C1 exact, and |x| - k C1 exact: a multiple
  // of 2^-29 below 2^-4) and k C2 as an exact product: r within
  // 2^-53 |r| + 2^-105 of |x| - k pi/32 (the final addition's rounding and
  // the terms below 2^-57), inside the bound below; for |x| < pi/64, k = 0
  // and r = |x| exactly.  The branch is wave-uniform, so it costs no
  // divergence; the result is certified by the same test either way, so it
  // does not depend on which branch runs.  Payne-Hanek is right down to
  // |x| = 2^-37; smaller arguments are special cases (|x| < 2^-12).
  if (__all(ax < 0x4b000000u)) {
    const double kd = rint(axd * INV_PI32);
    const double r1 = fma(-kd, PI32_CW1, axd);
    const dd p = two_prod(kd, PI32_CW2);
    const dd t = two_sum(r1, -p.hi);
    r = t.hi + (fma(-kd, PI32_CW3, t.lo) - p.lo);
    q = (int)kd & 63;
  } else {
    Reduced R = payne_hanek_fast(ax, tb.w);
    // f = fhi 2^-64 (the reduction leaves it low by less than 2^-64; the bits
    // below are not formed), as the exact sum of its signed high and
    // unsigned low 32-bit halves; their weights 2^-32 and 2^-64 are folded
    // into the constants (exact scalings)
    double fh = (double)(int)(R.fhi >> 32);
    double fl = (double)(uint32_t)R.fhi;
    r = fma(fh, PI32_HI * 0x1p-32, fma(fh, PI32_MID * 0x1p-32, fl * (PI32_HI * 0x1p-64)));
    q = R.q;
  }
  double r2 = r * r;
  double ps = fma(fma(SIN_S2[2], r2, SIN_S2[1]), r2, SIN_S2[0]);
  double pc = fma(fma(COS_C2[2], r2, COS_C2[1]), r2, COS_C2[0]);
  double sr = fma(r * r2, ps, r);  // sin r
  double cm1 = r2 * pc;            // cos r - 1
  // theta = q pi/32 = quad pi/2 + j pi/32, with T1, T2 = sin, cos of j pi/32
  // (the high parts of table row j) swapped in odd quadrants: an offset of
  // the two reads, from bit 4 of q.  Then
  //   sin x = +-(T1 + T1 (cos r - 1) + T2 sr'),
  //   cos x = +-(T2 + T2 (cos r - 1) - T1 sr'),
  // with sr' = sin r negated in odd quadrants and the outer signs given by
  // bit 5 of q (sin) and bit 4 xor bit 5 (cos).
  const double* row = reinterpret_cast<const double*>(&tb.sc[q & 15]);
  const int sw = (q >> 3) & 2;
  const double T1 = row[sw], T2 = row[sw ^ 2];
  const uint32_t q32 = (uint32_t)q;
  const double srq = flip(sr, q32 << 27);
  TrigFast o;
  o.s = T1 + fma(T1, cm1, T2 * srq);
  o.c = T2 + fma(T2, cm1, -(T1 * srq));
  o.ss = q32 << 26;
  o.sc = (q32 ^ (q32 << 1)) << 26;
  // Error bounds, absolute: r within 2^-52 |r| + 2^-66.35 (reduction, f to
  // 2^-63 in units of N; exact when the Cody-Waite branch has k = 0); the
  // degree-2 corrections within 2^-50.1 (cos) and 2^-57.6 (sin) -- the bound
  // tests re-derive both; the table entries within 2^-54 each; three
  // roundings of terms below 0.05 and the final one of y.  With |sin x|,
  // |cos x| >= 0.049 unless j = 0 this is below 2^-49.95 absolute, i.e.
  // 2^-45.6 |y|.  For j = 0 the table terms are exactly 0 and 1 and y is
  // +-sin r (within 2^-57.6 + 2^-51.9 |y| + 2^-66.35) or +-cos r (within
  // 2^-50.1, |y| > 0.99).  Bound used: 2^-45 |y| + 2^-57.
  o.es = fma(fabs(o.s), 0x1p-45, 0x1p-57);
  o.ec = fma(fabs(o.c), 0x1p-45, 0x1p-57);
  return o;
}

// bit 31 set when x is negative
__device__ __forceinline__ uint32_t sign_mask(float xf) { return f32_bits(xf); }

// The rounding test of the sin and cos fast paths, read off the bits of yh:
// for |yh| >= 2^-12 the bound above is below 2^-44 |yh| (the absolute term is
// then below 2^-45 |yh|), i.e. below 512 ulps of yh (ulps of 2^-53 |yh| and
// up), so a binary32 midpoint can lie within the error only when the 29 low
// bits of yh come within 512 of the midpoint pattern 2^28 (cr_round.h,
// round_f32_bits).  Results below 2^-12 in magnitude (x within about 2^-12 of
// a zero of sin or cos: about 1.5 10^-4 of random arguments) go to the
// accurate path.
__device__ __forceinline__ float round_trig_fast(double yh, bool& ok) {
  float r = round_f32_bits<512>(yh, ok);
  ok = ok && fabs(yh) >= 0x1p-12;
  return r;
}

// ------------------------------------------------------------ accurate path
__device__ __forceinline__ dd dd_div(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd p = dd_mul_d(b, q1);
  dd r = dd_add(a, dd_neg(p));
  double q2 = r.hi / b.hi;
  return fast_two_sum(q1, q2);
}

// Round h + l to binary32 given an absolute error bound e (accurate path).
__device__ __forceinline__ float round_f32_dd_abs(double h, double l, double e, bool& ok) {
  dd lo = fast_two_sum(h, l - e);
  dd hi = fast_two_sum(h, l + e);
  float a = (float)ro53(lo.hi, lo.lo);
  float b = (float)ro53(hi.hi, hi.lo);
  ok = a == b;
  return b;
}

struct TrigAcc {
  dd s, c;
  double eabs;  // absolute error bound on each of s, c
};

// sin x and cos x in double-double: 128-bit reduction, Taylor series of
// sin r and cos r (|r| <= pi/64; terms of index >= 4 in binary64).
__device__ __forceinline__ TrigAcc trig_acc_core(float xf, const TrigTab& tb) {
  uint32_t ax = f32_bits(xf) & 0x7fffffffu;
  double axd = (double)bits_f32(ax);
  bool small = axd < PI64;
  Reduced R = payne_hanek(ax, tb.w);
  double d1 = (double)(R.fhi >> 11) * 0x1p-53;
  double d2 = (double)(((uint64_t)(R.fhi & 0x7ff) << 42) | (R.flo >> 22)) * 0x1p-117;
  double d3 = (double)(R.flo & 0x3fffff) * 0x1p-128;
  dd f = dd_add_d(fast_two_sum(d1, d2), d3);
  dd r = dd_mul(f, dd{PI32_HI, PI32_MID});
  r = dd_add_d(r, f.hi * PI32_LO);
  int q = R.q;
  if (small) {
    r = {axd, 0.0};
    q = 0;
  }
  dd r2 = dd_mul(r, r);
  double ph = SIN_TAYLOR[TRIG_TAYLOR_N].x;
#pragma unroll
  for (int k = TRIG_TAYLOR_N - 1; k >= 4; k--) ph = fma(ph, r2.hi, SIN_TAYLOR[k].x);
  dd ps = {ph, 0.0};
#pragma unroll
  for (int k = 3; k >= 0; k--) {
    double2 c = SIN_TAYLOR[k];
    ps = dd_add(dd_mul(ps, r2), dd{c.x, c.y});
  }
  dd sr = dd_mul(ps, r);
  ph = COS_TAYLOR[TRIG_TAYLOR_N].x;
#pragma unroll
  for (int k = TRIG_TAYLOR_N - 1; k >= 4; k--) ph = fma(ph, r2.hi, COS_TAYLOR[k].x);
  dd pc = {ph, 0.0};
#pragma unroll
  for (int k = 3; k >= 0; k--) {
    double2 c = COS_TAYLOR[k];
    pc = dd_add(dd_mul(pc, r2), dd{c.x, c.y});
  }
  SinCosTheta th = theta_of(q, tb);
  dd S = {th.sh, th.sl}, C = {th.ch, th.cl};
  TrigAcc o;
  o.s = dd_add(dd_mul(S, pc), dd_mul(C, sr));
  o.c = dd_add(dd_mul(C, pc), dd_neg(dd_mul(S, sr)));
  // reduction: |f| error < 2^-129 (window 2^-130, conversion 2^-130), so r is
  // within 2^-102 |r| + 2^-132; double-double arithmetic adds < 2^-98 |result|
  o.eabs = small ? 0.0 : 0x1p-128;
  return o;
}

template <int KIND>
__device__ __noinline__ AccResult trig_accurate(float xf, const TrigTab& tb) {
  float sp;
  if (trig_special(xf, sp, KIND)) return {sp, 1};
  TrigAcc A = trig_acc_core(xf, tb);
  bool neg = xf < 0.0f;
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
    // relative errors of s and c add; the absolute parts scale with 1/|c|
    double ic = 1.0 / fabs(A.c.hi);
    e = fma(fabs(y.hi), 0x1p-93, A.eabs * ic * (1.0 + fabs(y.hi)) * 2.0);
  }
  bool ok;
  float r = round_f32_dd_abs(y.hi, y.lo, e, ok);
  return {r, ok ? 1 : 0};
}

// sincos accurate path: both results (sin in r, cos in r2)
struct AccResult2 {
  float s, c;
  int ok;
};

__device__ __noinline__ AccResult2 sincos_accurate(float xf, const TrigTab& tb) {
  float ss, cs;
  if (trig_special(xf, ss, TRIGK_SIN)) {
    trig_special(xf, cs, TRIGK_COS);
    return {ss, cs, 1};
  }
  TrigAcc A = trig_acc_core(xf, tb);
  dd s = xf < 0.0f ? dd_neg(A.s) : A.s;
  bool ok1, ok2;
  float rs = round_f32_dd_abs(s.hi, s.lo, fma(fabs(s.hi), 0x1p-95, A.eabs), ok1);
  float rc = round_f32_dd_abs(A.c.hi, A.c.lo, fma(fabs(A.c.hi), 0x1p-95, A.eabs), ok2);
  return {rs, rc, (ok1 && ok2) ? 1 : 0};
}

template <int KIND>
__device__ __forceinline__ float trig_fast(float xf, const TrigTab& tb, bool& ok) {
  TrigFast F = trig_fast_core(xf, tb);
  const uint32_t xs = sign_mask(xf);
  float res;
  if (KIND == TRIGK_COS) {
    res = round_trig_fast(flip(F.c, F.sc), ok);
  } else if (KIND == TRIGK_SIN) {
    res = round_trig_fast(flip(F.s, F.ss ^ xs), ok);
  } else {
    // t = s / c from the hardware reciprocal and two corrections by exact
    // residuals (each squares the relative error of the estimate), within
    // 2^-52 |t|; then the absolute errors of s and c magnified by 1/|c|:
    // |dt| <= |t| 2^-52 + (es + |t| ec) / |c| (bound with margins)
    const double t = div_fast(F.s, F.c);
    const double ic = __builtin_amdgcn_rcp(F.c);
    double e = fma(fabs(t), 0x1p-50, (F.es + fabs(t) * F.ec) * fabs(ic) * 2.0);
    res = round_f32_fast_abs(flip(t, F.ss ^ F.sc ^ xs), e, ok);
  }
  float sp;
  if (trig_special_fast(xf, sp, KIND)) {
    res = sp;
    ok = true;
  }
  return res;
}

// sincos fast path: returns sin in the result, cos in *c
__device__ __forceinline__ float sincos_fast(float xf, const TrigTab& tb, float& c, bool& ok) {
  TrigFast F = trig_fast_core(xf, tb);
  bool ok1, ok2;
  float s = round_trig_fast(flip(F.s, F.ss ^ sign_mask(xf)), ok1);
  c = round_trig_fast(flip(F.c, F.sc), ok2);
  ok = ok1 && ok2;
  float sp;
  if (trig_special_fast(xf, sp, TRIGK_SIN)) {
    s = sp;
    trig_special_fast(xf, c, TRIGK_COS);
    ok = true;
  }
  return s;
}

}  // namespace cr
