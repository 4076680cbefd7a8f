// cr_split_exp.h -- binary32-only (float-float) expf, exp2f, exp10f, expm1f.
//
// The method of the paper's exponentials (Sec. II-A, Fig. 1: a table of powers
// of two, a short polynomial, a scaling by 2^m) with binary32 arithmetic only.
// k = nearest(256 x log2 b) is split into balanced digits
//     k = 256 m + 16 j1 + j0,   j1, j0 in [-8, 7],
// so that b^x = 2^m 2^(j1/16) 2^(j0/256) e^r, r = x ln b - k ln2/256 and
// |r| <= ln2/512 (plus a hair for the rounded k): two 16-entry tables stand in
// for the 256 entries one lookup would need.  e^r - 1 = r + r^2/2 + r^3/6 +
// r^4/24 (Taylor; remainder below 2^-54 since |r| < 2^-9.4), with only
// r + r^2/2 in float-float.
//
// exp, exp2, exp10: y = T1 T2 (1 + q) in float-float, y in [0.68, 1.41].  The
//   rounding test runs on y (absolute bound 2^-44 -- tables 2^-49 each,
//   products and sums a few 2^-49 -- with margin), then the result is y 2^m,
//   exact for normal results.  For m <= -126 the result is below 2^-125 where
//   the grid is the fixed quantum 2^-149: y 2^(m+149) is rounded to an
//   integer instead.
// expm1: the tables hold 2^(j/16) - 1 and 2^(j/256) - 1, accurate near 0, and
//   W = D12 + q (1 + D12) with D12 = D1 + D2 + D1 D2.  u = (1 + W) - 2^-m is
//   rounded (m = 0: u = W, relative bound 2^-42; otherwise absolute 2^-45) and
//   the result is u 2^m.  For |x| < ln2/512, k = 0 and W = q: no
//   cancellation at all near 0.
// Lanes that fail the test take the triple-float step of cr_split_acc.h.
#pragma once
#include "cr_f32_exp.h"
#include "cr_split.h"
#include "cr_split_consts.h"

namespace cr {

struct SExpTab {
  float2 t1[16], t2[16];
};

template <int K>
__device__ __forceinline__ void sexp_tab_load(SExpTab& t, int tid) {
  if (tid < 16) {
    t.t1[tid] = (K == EXPK_EM1) ? SEXP_D1[tid] : SEXP_T1[tid];
    t.t2[tid] = (K == EXPK_EM1) ? SEXP_D2[tid] : SEXP_T2[tid];
  }
}

// k (as a float) and r = x ln b - k ln2/256 as a normalised float-float
template <int K>
__device__ __forceinline__ ff sexp_reduce(float x, float& kf) {
  if (K == EXPK_E || K == EXPK_EM1) {
    kf = rintf(x * SEXP_INV_LN2_256);
    // k C1 is exact (16 + 8 bits) and so is x - k C1 (C1 is ln2/256 rounded
    // toward zero: x and k C1 are within a factor 2 of each other, or k = 0)
    float r1 = fmaf(-kf, SEXP_C1, x);
    ff p = ff_two_prod(kf, SEXP_C2);
    ff s = ff_two_sum(r1, -p.hi);
    float lo = (s.lo - p.lo) - kf * SEXP_C3;
    return ff_two_sum(s.hi, lo);
  } else if (K == EXPK_2) {
    float t = x * 256.0f;  // exact
    kf = rintf(t);
    float f = t - kf;      // exact, |f| <= 1/2
    ff p = ff_two_prod(f, SEXP_LN2_256_H);
    return ff_fast_two_sum(p.hi, fmaf(f, SEXP_LN2_256_L, p.lo));
  } else {
    // f = 256 x log2(10) - k in float-float (the constant in three parts),
    // then r = f ln2/256
    ff p1 = ff_two_prod(x, SEXP_L10_H);
    kf = rintf(p1.hi);
    float a = p1.hi - kf;  // exact
    ff p2 = ff_two_prod(x, SEXP_L10_M);
    ff A = ff_two_sum(a, p1.lo);
    ff B = ff_two_sum(A.hi, p2.hi);
    float flo = (A.lo + B.lo) + fmaf(x, SEXP_L10_L, p2.lo);
    ff f = ff_two_sum(B.hi, flo);
    ff p = ff_two_prod(f.hi, SEXP_LN2_256_H);
    return ff_fast_two_sum(p.hi, fmaf(f.hi, SEXP_LN2_256_L, fmaf(f.lo, SEXP_LN2_256_H, p.lo)));
  }
}

// k = 256 m + 16 j1 + j0 with balanced digits j1, j0 in [-8, 7]
struct SExpDigits {
  int m, i1, i0;  // i1 = j1 + 8, i0 = j0 + 8: table indices
};

__device__ __forceinline__ SExpDigits sexp_digits(float kf) {
  int k = (int)kf;
  SExpDigits d;
  d.m = (k + 136) >> 8;  // floor: k - 256 m in [-136, 119]
  int rem = k - (d.m << 8);
  int j1 = (rem + 8) >> 4;  // [-8, 7]
  d.i1 = j1 + 8;
  d.i0 = rem - (j1 << 4) + 8;
  return d;
}

// q = e^r - 1 = r + r^2/2 + r^3/6 + r^4/24 for a normalised float-float r
__device__ __forceinline__ ff sexp_q(ff r) {
  ff sq = ff_two_prod(r.hi, r.hi);
  float t3 = sq.hi * r.hi * fmaf(r.hi, SEXP_INV24, SEXP_INV6);
  ff qh = ff_fast_two_sum(r.hi, 0.5f * sq.hi);
  float ql = qh.lo + (r.lo + (fmaf(r.hi, r.lo, 0.5f * sq.lo) + t3));
  return ff_fast_two_sum(qh.hi, ql);
}

// y = T1 T2 (1 + q) (not normalised: |lo| may reach a few ulps of hi)
__device__ __forceinline__ ff sexp_T(float2 A, float2 B, ff q) {
  ff P = ff_two_prod(A.x, B.x);
  float Pl = fmaf(A.x, B.y, fmaf(A.y, B.x, P.lo));
  ff PQ = ff_two_prod(P.hi, q.hi);
  ff Y = ff_fast_two_sum(P.hi, PQ.hi);
  return {Y.hi, Y.lo + (Pl + (PQ.lo + fmaf(P.hi, q.lo, Pl * q.hi)))};
}

// W = D12 + q (1 + D12), D12 = D1 + D2 + D1 D2 = T1 T2 - 1 (tables of 2^j - 1)
__device__ __forceinline__ ff sexp_W(float2 A, float2 B, ff q) {
  // |D1| >= 0.043 > |D2| unless D1 = 0
  ff S = ff_fast_two_sum(A.x, B.x);
  ff P = ff_two_prod(A.x, B.x);
  ff U = ff_fast_two_sum(S.hi, P.hi);
  float ul = U.lo + (S.lo + ((A.y + B.y) + (P.lo + fmaf(A.x, B.y, A.y * B.x))));
  ff D = ff_fast_two_sum(U.hi, ul);
  // |D12| >= 0.0027 > |q| unless D12 = 0
  ff QD = ff_two_prod(q.hi, D.hi);
  ff V = ff_fast_two_sum(D.hi, q.hi);
  ff V2 = ff_fast_two_sum(V.hi, QD.hi);
  return {V2.hi, (V.lo + V2.lo) + ((D.lo + q.lo) + (QD.lo + fmaf(q.hi, D.lo, q.lo * D.hi)))};
}

template <int K>
__device__ __forceinline__ float sexp_fast(float xf, const SExpTab& tb, bool& ok) {
  // clamp: the clamp values over- or underflow by far (expm1: -20 gives -1)
  const float lo_lim = (K == EXPK_EM1) ? -20.0f
                       : (K == EXPK_10) ? -50.0f
                       : (K == EXPK_2) ? -200.0f : -150.0f;
  const float hi_lim = (K == EXPK_EM1) ? 90.0f : -lo_lim;
  float x = fminf(fmaxf(xf, lo_lim), hi_lim);
  float kf;
  ff r = sexp_reduce<K>(x, kf);
  SExpDigits dg = sexp_digits(kf);
  const int m = dg.m;
  float2 A = tb.t1[dg.i1], B = tb.t2[dg.i0];
  ff q = sexp_q(r);

  float res;
  if (K != EXPK_EM1) {
    ff Y = sexp_T(A, B, q);
    bool okn, okq;
    res = ldexpf(round_split(Y.hi, Y.lo, 0x1p-44f, okn), m);
    // results below 2^-125: round y 2^(m+149) to an integer (m >= -217)
    float sc = pow2f_i(m + 149 < 23 ? m + 149 : 23);
    float rq = round_split_q(Y.hi * sc, Y.lo * sc, fmaf(0x1p-44f, sc, 0x1p-22f), okq);
    ok = okn;
    if (m <= -126) {
      res = rq;
      ok = okq;
    }
  } else {
    ff W = sexp_W(A, B, q);
    // u = (1 + W) - 2^-m; m = 0: u = W
    ff O = ff_fast_two_sum(1.0f, W.hi);
    ff Uu = ff_two_sum(O.hi, -pow2f_i(-m));  // m in [-29, 130]
    float uh = Uu.hi, ulo = Uu.lo + (O.lo + W.lo), err = 0x1p-45f;
    if (m == 0) {
      uh = W.hi;
      ulo = W.lo;
      err = fabsf(W.hi) * 0x1p-42f;
    }
    res = ldexpf(round_split(uh, ulo, err, ok), m);
  }
  float sp;
  if (exp_special<K>(xf, sp)) {
    res = sp;
    ok = true;
  }
  return res;
}

}  // namespace cr
