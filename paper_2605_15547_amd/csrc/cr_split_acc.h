// cr_split_acc.h -- the accurate step of the binary32-only kernels, in
// triple-float arithmetic: no binary64 operation anywhere on the path.
//
// The paper's binary32 functions test the rounding of a fast evaluation and
// finish the rare failing cases with a slower, more accurate one (Sec. II-A);
// its Sec. IV points to internal arithmetic on 32-bit operations for GPUs on
// which binary64 is slow.  The binary32-only kernels follow both: their fast
// path is float-float (cr_split_*.h) and the lanes whose rounding it cannot
// decide come here.  Each function repeats the reduction of its fast path,
// carried to triple-float (cr_tf.h): tables of 16 triple-float entries, the
// reduced argument to about 2^-70, and a polynomial whose leading terms are
// triple-float products and whose tail is float-float.  The result is rounded
// by comparing its tail with the rounding boundary (round32_tf), given a
// relative error bound:
//   TF_EREL = 2^-62 for every function: the hardest binary32 inputs lie at
//   least 2^-58.9 (exp2f), 2^-57.8 (logf, log1pf), 2^-56 and more (the
//   others) from a rounding boundary, relative to the value, and the
//   triple-float evaluations below stay within a few 2^-66 (each triple-float
//   addition or product contributes below 2^-67 of its larger operand; the
//   float-float tails stay below 2^-66 of the result).
//   log1p of |x| < 2^-12 has the one harder pair, x = +-1.5000004 2^-21 at
//   2^-66.4: there log1p x = x + C with -x^2/2 exact and the rest of C (below
//   2^-25.6 |x|) to 2^-46 of itself, the final sum within 2^-71 |x|, so the
//   result is within about 2^-70.5 of itself and the bound is TF_EREL_TINY =
//   2^-68.
// A lane whose bound still straddles a boundary is counted as an escape (the
// exhaustive scans of all 2^32 inputs find none).
#pragma once
#include "cr_split_atan.h"
#include "cr_split_exp.h"
#include "cr_split_hyp.h"
#include "cr_split_log.h"
#include "cr_split_trig.h"
#include "cr_tf.h"

namespace cr {

#define TF_EREL (0x1p-62f)
#define TF_EREL_TINY (0x1p-68f)

__device__ __forceinline__ tf tf_tab(const float4* t, int i) {
  const float4 v = t[i];
  return {v.x, v.y, v.z};
}

__device__ __forceinline__ tf tf_k(float h, float m, float l) { return {h, m, l}; }

// float-float product of a triple-float (its two leading parts) and a float-float
__device__ __forceinline__ ff ff_mul_tf(tf a, ff b) {
  ff p = ff_two_prod(a.h, b.hi);
  return {p.hi, fmaf(a.h, b.lo, fmaf(a.m, b.hi, p.lo))};
}

// ============================================================ exponentials
// r = x ln b - k ln2/256 as a triple-float (absolute error below 2^-72)
template <int K>
__device__ __forceinline__ tf tfexp_reduce(float x, float& kf) {
  if (K == EXPK_E || K == EXPK_EM1) {
    // ln2/256 = C1 + C2 + C3 + C4: k C1 and x - k C1 are exact (as in the
    // fast path), k C2 and k C3 are exact products
    kf = rintf(x * SEXP_INV_LN2_256);
    const float r1 = fmaf(-kf, SEXP_C1, x);
    const ff p2 = ff_two_prod(kf, SEXP_C2);
    const ff p3 = ff_two_prod(kf, SEXP_C3);
    const ff s = ff_two_sum(r1, -p2.hi);
    const tf a = tf_renorm(s.hi, s.lo, -p2.lo);               // exact
    const tf b = tf_renorm(-p3.hi, -p3.lo, -kf * TFEXP_C4);   // exact but the last product
    return tf_add(a, b);
  } else if (K == EXPK_2) {
    const float t = x * 256.0f;  // exact
    kf = rintf(t);
    const float f = t - kf;      // exact, |f| <= 1/2
    const ff p1 = ff_two_prod(f, TFEXP_LN2_256_H);
    const ff p2 = ff_two_prod(f, TFEXP_LN2_256_M);
    const ff a = ff_two_sum(p1.lo, p2.hi);
    return tf_renorm(p1.hi, a.hi, a.lo + fmaf(f, TFEXP_LN2_256_L, p2.lo));
  } else {
    // f = 256 x log2(10) - k with the constant in four parts, then f ln2/256
    const ff p1 = ff_two_prod(x, SEXP_L10_H);
    kf = rintf(p1.hi);
    const float a = p1.hi - kf;  // exact
    const ff p2 = ff_two_prod(x, SEXP_L10_M);
    const ff p3 = ff_two_prod(x, SEXP_L10_L);
    const tf A = tf_renorm(a, p1.lo, p2.hi);
    const tf B = tf_renorm(p2.lo, p3.hi, fmaf(x, TFEXP_L10_LL, p3.lo));
    const tf f = tf_add(A, B);
    return tf_mul(f, tf_k(TFEXP_LN2_256_H, TFEXP_LN2_256_M, TFEXP_LN2_256_L));
  }
}

// q = e^r - 1 = r + r^2/2 + r^3 (1/6 + r/24 + r^2/120 + r^3/720 + r^4/5040),
// |r| < 2^-9.3 (Taylor; the next term is below 2^-72 |r|).  r^2/2 is a
// triple-float, r^3 (...) a float-float product (2^-46 of itself, itself
// below 2^-10.9 |q|).
__device__ __forceinline__ tf tfexp_q(tf r) {
  const tf z = tf_mul(r, r);
  ff r3 = ff_two_prod(z.h, r.h);
  r3.lo = fmaf(z.h, r.m, fmaf(z.m, r.h, r3.lo));
  const float p5 = fmaf(fmaf(TF_INVFACT7, r.h, TF_INVFACT6), r.h, TF_INV120_H);
  // b = 1/24 + r p5 and c = 1/6 + r b as float-floats
  const ff rp = ff_two_prod(r.h, p5);
  ff b = ff_two_sum(TF_INV24_H, rp.hi);
  b.lo += TF_INV24_L + rp.lo;
  ff rb = ff_mul_tf(r, b);
  ff c = ff_two_sum(TF_SIXTH_H, rb.hi);
  c.lo += TF_SIXTH_M + rb.lo;
  const ff t3 = ff_mul(r3, c);
  const tf s = tf_add_ff(tf_scale(z, 0.5f), t3);
  return tf_add_ord(r, s);  // |s| < 2^-10 |r|
}

template <int K>
__device__ __noinline__ AccResult sexp_acc(float xf) {
  const float lo_lim = (K == EXPK_EM1) ? -20.0f
                       : (K == EXPK_10) ? -50.0f
                       : (K == EXPK_2) ? -200.0f : -150.0f;
  const float hi_lim = (K == EXPK_EM1) ? 90.0f : -lo_lim;
  const float x = (xf == xf) ? fminf(fmaxf(xf, lo_lim), hi_lim) : 0.0f;
  float kf;
  const tf r = tfexp_reduce<K>(x, kf);
  const SExpDigits dg = sexp_digits(kf);
  const int m = dg.m;
  const tf q = tfexp_q(r);
  bool ok;
  float res;
  if (K != EXPK_EM1) {
    // y = T1 T2 (1 + q), in [0.68, 1.42]
    const tf T = tf_mul(tf_tab(TFEXP_T1, dg.i1), tf_tab(TFEXP_T2, dg.i0));
    const tf y = tf_add_ord(T, tf_mul(T, q));  // |T q| < 2^-9 |T|
    if (m > -126) {
      res = ldexpf(round32_tf(y, TF_EREL, ok), m);
    } else {  // below 2^-125: integer multiple of 2^-149 (m >= -217)
      const float sc = pow2f_i(m + 149 < 23 ? m + 149 : 23);
      const tf v = tf_scale(y, sc);
      res = round32_tf_q(v, fmaf(v.h, TF_EREL, 0x1p-60f), ok);
    }
  } else {
    // W = D12 + q (1 + D12), D12 = D1 + D2 + D1 D2 = T1 T2 - 1 (no cancellation
    // beyond a factor 2: |D1| > 2 |D2| and |D12| > 2 |q| unless zero), then
    // e^x - 1 = 2^m ((1 + W) - 2^-m)
    const tf D1 = tf_tab(TFEXP_D1, dg.i1), D2 = tf_tab(TFEXP_D2, dg.i0);
    const tf D12 = tf_add(tf_add(D1, D2), tf_mul(D1, D2));
    const tf W = tf_add(D12, tf_mul(q, tf_add_f(D12, 1.0f)));
    const tf u = (m == 0) ? W : tf_add(W, tf_renorm(1.0f, -pow2f_i(-m), 0.0f));
    res = ldexpf(round32_tf(u, TF_EREL, ok), m);
  }
  float sp;
  if (exp_special<K>(xf, sp)) {
    res = sp;
    ok = true;
  }
  return {res, ok ? 1 : 0};
}

// ============================================================ logarithms
// log1p t = t - t^2/2 + t^3/3 - t^4 (1/4 - t/5 + t^2/6 - t^3/7 + t^4/8 - t^5/9)
// for |t| < 0.0049 (Taylor; next term below 2^-74 |t|): t, t^2/2 and t^3/3
// in triple-float, the t^4 term (below 2^-25 |t|) in float-float.
__device__ __forceinline__ tf tflog1p_poly(tf t) {
  const tf z = tf_mul(t, t);
  const tf c3 = tf_mul(tf_mul(z, t), tf_k(TF_THIRD_H, TF_THIRD_M, TF_THIRD_L));
  const float th = t.h;
  const float in6 = fmaf(fmaf(fmaf(-TF_RECIP9, th, 0.125f), -th, TF_RECIP7), -th, 1.0f / 6.0f);
  // b = 1/5 - t in6, P4 = 1/4 - t b, as float-floats
  const ff tp = ff_two_prod(th, in6);
  ff b = ff_two_sum(TF_FIFTH_H, -tp.hi);
  b.lo += TF_FIFTH_L - tp.lo;
  const ff tb = ff_mul_tf(t, b);
  ff P4 = ff_two_sum(0.25f, -tb.hi);
  P4.lo -= tb.lo;
  ff z2 = ff_two_prod(z.h, z.h);
  z2.lo = fmaf(2.0f * z.h, z.m, z2.lo);
  const ff t4 = ff_mul(z2, P4);
  const tf s = tf_add_ff(c3, ff{-t4.hi, -t4.lo});
  // each sum is ordered: |s| < |t| |t^2/2| and |t^2/2| < |t|/2 (|t| < 2^-7.6)
  return tf_add_ord(t, tf_add_ord(tf_scale(z, -0.5f), s));
}

template <int K>
__device__ __noinline__ AccResult slog_acc(float xf) {
  // the reduction of the fast path (cr_split_log.h), with t kept exact
  float uh, ul = 0.0f;
  if (K == LOGK_1P) {
    const float xs = (xf > -1.0f && xf < INFINITY) ? xf : 0.0f;
    const ff u = ff_two_sum(1.0f, xs);
    uh = u.hi;
    ul = u.lo;
  } else {
    uh = (xf > 0.0f && xf < INFINITY) ? xf : 1.0f;
  }
  int esub = 0;
  if (K != LOGK_1P && uh < 0x1p-126f) {
    uh *= 0x1p24f;
    esub = -24;
  }
  const unsigned bb = __float_as_uint(uh);
  const int j = (bb >> 19) & 15;
  int e = (int)((bb >> 23) & 0xff) - 127 + esub;
  unsigned mb = (bb & 0x007fffffu) | 0x3f800000u;
  const int fold = j >= 8;
  mb -= fold ? 0x00800000u : 0u;
  e += fold;
  const float m = __uint_as_float(mb);
  const float ml = ldexpf(ul, -e);
  const float c1 = SLOG_C1[j];
  const float t1 = fmaf(m, c1, -1.0f);
  int i = (int)rintf(t1 * SLOG_S);
  i = i < -8 ? -8 : (i > 7 ? 7 : i);
  const float C = c1 * SLOG_C2[i + 8];  // exact
  const ff p = ff_two_prod(m, C);
  const float th0 = p.hi - 1.0f;        // exact
  tf t;
  if (K == LOGK_1P) {
    const ff p2 = ff_two_prod(ml, C);
    const ff A = ff_two_sum(p.lo, p2.hi);
    t = tf_add_f(tf_renorm(th0, A.hi, A.lo), p2.lo);
  } else {
    t = tf_renorm(th0, p.lo, 0.0f);
  }
  float erel = TF_EREL;
  tf L;
  if (K == LOGK_1P && fabsf(xf) < 0x1p-12f) {
    // log1p x = x + C, C = -x^2/2 + x^3 (1/3 - x/4 + x^2/5 - x^3/6): -x^2/2
    // exact, the rest in float-float (below 2^-25 |x|); the final sum exact
    const float x = xf;
    const ff x2 = ff_two_prod(x, x);
    const float in = fmaf(fmaf(-1.0f / 6.0f, x, TF_RECIP5), x, -0.25f);
    const ff xi = ff_two_prod(x, in);
    ff c = ff_two_sum(TF_THIRD_H, xi.hi);
    c.lo += TF_THIRD_M + xi.lo;
    ff x3 = ff_two_prod(x2.hi, x);
    x3.lo = fmaf(x2.lo, x, x3.lo);
    const ff k3 = ff_mul(x3, c);
    const tf Cs = tf_add_ff(tf_k(-0.5f * x2.hi, -0.5f * x2.lo, 0.0f), k3);
    L = tf_add_f(Cs, x);
    erel = TF_EREL_TINY;
  } else {
    const tf P = tflog1p_poly(t);
    // Z = -log c1 - log c2 + log1p t
    tf Z = tf_add(tf_add(tf_tab(TFLOG_L1, j), tf_tab(TFLOG_L2, i + 8)), P);
    if (K == LOGK_2) Z = tf_mul(Z, tf_k(TFLOG_INV_LN2_H, TFLOG_INV_LN2_M, TFLOG_INV_LN2_L));
    if (K == LOGK_10) Z = tf_mul(Z, tf_k(TFLOG_INV_LN10_H, TFLOG_INV_LN10_M, TFLOG_INV_LN10_L));
    const float ef = (float)e;
    if (K == LOGK_2) {
      L = tf_add_f(Z, ef);
    } else {
      // e log_b 2 with the constant in four parts, the first 16 bits wide
      const float k1 = K == LOGK_10 ? TFLOG_LG2_H : TFLOG_LN2_H;
      const float k2 = K == LOGK_10 ? TFLOG_LG2_M : TFLOG_LN2_M;
      const float k3 = K == LOGK_10 ? TFLOG_LG2_L : TFLOG_LN2_L;
      const float k4 = K == LOGK_10 ? TFLOG_LG2_LL : TFLOG_LN2_LL;
      const ff e2 = ff_two_prod(ef, k2);
      const ff e3 = ff_two_prod(ef, k3);
      const tf E = tf_add_ord(tf_renorm(ef * k1, e2.hi, e2.lo), tf_renorm(e3.hi, e3.lo, ef * k4));
      // |Z| <= 0.41 < |E| / 1.7 unless e = 0 (then E = 0)
      L = tf_add_ord(E, Z);
    }
  }
  bool ok;
  float res = round32_tf(L, erel, ok);
  float sp;
  if (slog_special<K>(xf, sp)) {
    res = sp;
    ok = true;
  }
  return {res, ok ? 1 : 0};
}

// ============================================================ sin, cos, tan
struct TfTrig {
  tf s, c;     // sin |x| and cos |x|
  bool small;  // |x| < pi/64 (no reduction)
};

// sin and cos of |x| from the integer Payne-Hanek reduction (72 leading bits
// of the normalised fraction), |r| <= pi/64:
//   sin r = r - r^3/6 + r^5 (1/120 - r^2/7! + r^4/9! - r^6/11! + r^8/13!),
//   cos r = 1 - r^2/2 + r^4 (1/24 - r^2/6! + r^4/8! - r^6/10! + r^8/12!)
// (Taylor; next terms below 2^-84), r, r^2/2 and r^3/6 in triple-float, the
// tails (below 2^-17 of the result) in float-float.
__device__ __forceinline__ TfTrig tftrig_core(float xf, const unsigned* w) {
  const uint32_t ax = f32_bits(xf) & 0x7fffffffu;
  const float axf = bits_f32(ax);
  TfTrig o;
  o.small = axf < STRIG_PI64;
  const Reduced R = payne_hanek(ax, w);
  uint64_t hi = (uint64_t)R.fhi, lo = R.flo;
  const bool neg = R.fhi < 0;
  if (neg) {
    lo = ~lo + 1;
    hi = ~hi + (lo == 0 ? 1 : 0);
  }
  int extra = 0;
  if (hi == 0) {
    hi = lo;
    lo = 0;
    extra = 64;
  }
  const int sft = hi ? __clzll((long long)hi) : 0;
  const uint64_t top = sft ? ((hi << sft) | (lo >> (64 - sft))) : hi;
  const uint64_t bot = sft ? (lo << sft) : lo;
  const int S = sft + extra;
  float f0 = ldexpf((float)(uint32_t)(top >> 40), -24 - S);
  float f1 = ldexpf((float)(uint32_t)((top >> 16) & 0xffffffu), -48 - S);
  float f2 = ldexpf((float)(uint32_t)(((top & 0xffffu) << 8) | (bot >> 56)), -72 - S);
  if (neg) {
    f0 = -f0;
    f1 = -f1;
    f2 = -f2;
  }
  tf r = tf_mul(tf_renorm(f0, f1, f2), tf_k(TFTRIG_PI32_H, TFTRIG_PI32_M, TFTRIG_PI32_L));
  int q = R.q;
  if (o.small) {
    r = tf_from(axf);
    q = 0;
  }
  const tf z = tf_mul(r, r);
  const float zh = z.h;
  // sin r
  const tf r3 = tf_mul(z, r);
  const tf r36 = tf_mul(r3, tf_k(TF_SIXTH_H, TF_SIXTH_M, TF_SIXTH_L));
  const float s7 = fmaf(fmaf(fmaf(TFTRIG_S13, zh, TFTRIG_S11), zh, TFTRIG_S9), zh, TFTRIG_S7);
  const ff sp = ff_two_prod(zh, s7);
  ff s5 = ff_two_sum(TF_INV120_H, sp.hi);
  s5.lo += TF_INV120_L + sp.lo;
  ff r5 = ff_two_prod(r3.h, zh);
  r5.lo = fmaf(r3.h, z.m, fmaf(r3.m, zh, r5.lo));
  const ff st = ff_mul(r5, s5);
  const tf sr = tf_add_ord(r, tf_add_ff(tf_neg(r36), st));  // |r^3/6 ...| < 2^-8 |r|
  // cos r - 1
  const float c6 = fmaf(fmaf(fmaf(TFTRIG_C12, zh, TFTRIG_C10), zh, TFTRIG_C8), zh, TFTRIG_C6);
  const ff cp = ff_two_prod(zh, c6);
  ff c4 = ff_two_sum(TF_INV24_H, cp.hi);
  c4.lo += TF_INV24_L + cp.lo;
  ff z2 = ff_two_prod(zh, zh);
  z2.lo = fmaf(2.0f * zh, z.m, z2.lo);
  const ff ct = ff_mul(z2, c4);
  const tf cm = tf_add_ff(tf_scale(z, -0.5f), ct);

  // theta = q pi/32 = quad pi/2 + j pi/32: sin and cos of j pi/32 with the
  // quadrant's swap and signs
  const int quad = q >> 4, jj = q & 15;
  const bool swap = quad & 1;
  tf Sv = tf_tab(swap ? TFTRIG_C : TFTRIG_S, jj);
  tf Cv = tf_tab(swap ? TFTRIG_S : TFTRIG_C, jj);
  if (quad >= 2) Sv = tf_neg(Sv);
  if (quad == 1 || quad == 2) Cv = tf_neg(Cv);
  // sin x = S + (C sin r + S (cos r - 1)), cos x = C + (C (cos r - 1) - S sin r)
  // ordered sums: |S (cos r - 1)| <= |C sin r| / 4 and |C (cos r - 1)| <=
  // |S sin r| / 4 unless the larger term's factor is 0, and the table term
  // (>= 0.098 unless 0) dominates the rest (<= 0.05)
  o.s = tf_add_ord(Sv, tf_add_ord(tf_mul(Cv, sr), tf_mul(Sv, cm)));
  o.c = tf_add_ord(Cv, tf_add_ord(tf_neg(tf_mul(Sv, sr)), tf_mul(Cv, cm)));
  return o;
}

template <int KIND>
__device__ __noinline__ AccResult strig_acc(float xf, const unsigned* w) {
  const TfTrig T = tftrig_core(xf, w);
  const bool neg = xf < 0.0f;
  tf y;
  if (KIND == TRIGK_COS) {
    y = T.c;
  } else if (KIND == TRIGK_SIN) {
    y = neg ? tf_neg(T.s) : T.s;
  } else {
    y = tf_div(T.s, T.c);
    if (neg) y = tf_neg(y);
  }
  bool ok;
  float res = round32_tf(y, TF_EREL, ok);
  float sp;
  if (trig_special(xf, sp, KIND)) {
    res = sp;
    ok = true;
  }
  return {res, ok ? 1 : 0};
}

__device__ __noinline__ AccResult2 ssincos_acc(float xf, const unsigned* w) {
  const TfTrig T = tftrig_core(xf, w);
  const tf s = xf < 0.0f ? tf_neg(T.s) : T.s;
  bool ok1, ok2;
  float rs = round32_tf(s, TF_EREL, ok1);
  float rc = round32_tf(T.c, TF_EREL, ok2);
  float sp;
  if (trig_special(xf, sp, TRIGK_SIN)) {
    rs = sp;
    trig_special(xf, rc, TRIGK_COS);
    ok1 = ok2 = true;
  }
  return {rs, rc, (ok1 && ok2) ? 1 : 0};
}

// ============================================================ atan, asin, acos
// atan(Y/X) for Y, X >= 0 (not both zero) as in the fast path: c = j/16
// nearest to min/max, t = (Y - c X)/(X + c Y) (|t| <= 1/31), and
// atan t = t - t^3/3 + t^5 (1/5 - t^2/7 + t^4/9 - t^6/11 + t^8/13) (Taylor; next
// term below 2^-73 |t|): t and t^3/3 triple-float, the tail float-float.
__device__ __forceinline__ tf tfatan_ratio(tf Y0, tf X0) {
  const bool inv = Y0.h > X0.h;
  const tf Y = inv ? X0 : Y0, X = inv ? Y0 : X0;
  const float zf = Y.h * __builtin_amdgcn_rcpf(X.h);  // index only
  int j = (int)rintf(16.0f * zf);
  j = j > 15 ? 15 : (j < 0 ? 0 : j);
  const float c = (float)j * 0.0625f;
  const tf num = tf_add(Y, tf_neg(tf_mul_f(X, c)));
  const tf den = tf_add(X, tf_mul_f(Y, c));
  const tf t = tf_div(num, den);
  const tf z = tf_mul(t, t);
  const tf c3 = tf_mul(tf_mul(z, t), tf_k(TF_THIRD_H, TF_THIRD_M, TF_THIRD_L));
  const float zh = z.h;
  const float p7 = fmaf(fmaf(fmaf(TFATAN_P13, zh, TFATAN_P11), zh, TFATAN_P9), zh, TFATAN_P7);
  const ff pp = ff_two_prod(zh, p7);
  ff P = ff_two_sum(TF_FIFTH_H, pp.hi);
  P.lo += TF_FIFTH_L + pp.lo;
  ff z2 = ff_two_prod(zh, zh);
  z2.lo = fmaf(2.0f * zh, z.m, z2.lo);
  ff t5 = ff_mul_tf(t, z2);
  const ff tail = ff_mul(t5, P);
  const tf at = tf_add(t, tf_add_ff(tf_neg(c3), tail));
  const tf base = tf_tab(inv ? TFATAN_B : TFATAN_A, j);
  // |atan t| <= atan(1/31) <= base/2, or base = 0 (j = 0, not inverted)
  return tf_add_ord(base, inv ? tf_neg(at) : at);
}

// sqrt(1 - a^2) as a triple-float, a in [0, 1]: two Newton steps from the
// binary32 square root, each with an exact residual
__device__ __forceinline__ tf tfsqrt_1m_sq(float a) {
  const ff p = ff_two_prod(a, a);
  const tf W = tf_renorm(1.0f, -p.hi, -p.lo);  // exact
  if (!(W.h > 0.0f)) return tf_from(0.0f);
  const float s0 = sqrtf(W.h);
  const float ih = 0.5f * __builtin_amdgcn_rcpf(s0);
  const ff s2 = ff_two_prod(s0, s0);
  const tf r0 = tf_add(W, tf_k(-s2.hi, -s2.lo, 0.0f));
  const tf s1 = tf_add_f(tf_mul_f(r0, ih), s0);
  const tf r1 = tf_add(W, tf_neg(tf_mul(s1, s1)));
  return tf_add(s1, tf_mul_f(r1, ih));
}

template <int KIND>
__device__ __noinline__ AccResult satan_acc(float xf) {
  const float a = (xf == xf) ? fminf(fabsf(xf), 0x1p100f) : 0.0f;
  const bool neg = xf < 0.0f;
  tf y;
  if (KIND == ATANK_ATAN) {
    y = tfatan_ratio(tf_from(a), tf_from(1.0f));
    if (neg) y = tf_neg(y);
  } else {
    const float ac = fminf(a, 1.0f);
    const tf s = tfsqrt_1m_sq(ac);
    if (KIND == ATANK_ASIN) {
      y = tfatan_ratio(tf_from(ac), s);
      if (neg) y = tf_neg(y);
    } else {
      y = tfatan_ratio(s, tf_from(ac));
      if (neg) y = tf_add(tf_k(TFATAN_PI_H, TFATAN_PI_M, TFATAN_PI_L), tf_neg(y));
    }
  }
  bool ok;
  float res = round32_tf(y, TF_EREL, ok);
  float sp;
  if (atan_special(xf, KIND, sp)) {
    res = sp;
    ok = true;
  }
  return {res, ok ? 1 : 0};
}

// ============================================================ sinh, cosh, tanh
// The decomposition of the fast path (cr_split_hyp.h) in triple-float:
// e^a = 2^m y with y = T1 T2 (1 + q); for m = 0 the expm1 form E = W avoids
// the cancellation of sinh and tanh near 0.
template <int KIND>
__device__ __noinline__ AccResult shyp_acc(float xf) {
  const float a = (xf == xf) ? fminf(fabsf(xf), KIND == HYPK_TANH ? 20.0f : 100.0f) : 0.0f;
  const float xe = KIND == HYPK_TANH ? 2.0f * a : a;
  float kf;
  const tf r = tfexp_reduce<EXPK_E>(xe, kf);
  const SExpDigits dg = sexp_digits(kf);
  const int m = dg.m;
  const tf q = tfexp_q(r);
  tf v;
  int sc = 0;
  if (KIND != HYPK_COSH && m == 0) {
    const tf D1 = tf_tab(TFEXP_D1, dg.i1), D2 = tf_tab(TFEXP_D2, dg.i0);
    const tf D12 = tf_add(tf_add(D1, D2), tf_mul(D1, D2));
    const tf E = tf_add(D12, tf_mul(q, tf_add_f(D12, 1.0f)));
    if (KIND == HYPK_SINH) {  // (E + E/(E + 1))/2
      v = tf_add_ord(E, tf_div(E, tf_add_f(E, 1.0f)));  // 0 <= E/(E + 1) <= E
      sc = -1;
    } else {                  // E/(E + 2)
      v = tf_div(E, tf_add_f(E, 2.0f));
    }
  } else {
    const tf T = tf_mul(tf_tab(TFEXP_T1, dg.i1), tf_tab(TFEXP_T2, dg.i0));
    const tf Y = tf_add_ord(T, tf_mul(T, q));
    // beyond m = 40 the e^-a terms are below 2^-79 of the result: their scale
    // is frozen at m = 40 (tanh then rounds to 1 either way)
    const int mc = m < 40 ? m : 40;
    if (KIND == HYPK_TANH) {  // (y - 2^-m)/(y + 2^-m)
      const float p = pow2f_i(-mc);
      v = tf_div(tf_add_f(Y, -p), tf_add_f(Y, p));
    } else {                  // 2^(m-1) (y -+ 2^(-2m)/y)
      const float p = pow2f_i(-2 * mc);
      const tf w = tf_scale(tf_div(tf_from(1.0f), Y), p);
      v = tf_add_ord(Y, KIND == HYPK_SINH ? tf_neg(w) : w);  // |w| <= 0.37 Y
      sc = m - 1;
    }
  }
  bool ok;
  float res = ldexpf(round32_tf(v, TF_EREL, ok), sc);
  if (KIND != HYPK_COSH && xf < 0.0f) res = -res;
  float sp;
  if (hyp_special(xf, KIND, sp)) {
    res = sp;
    ok = true;
  }
  return {res, ok ? 1 : 0};
}

}  // namespace cr
