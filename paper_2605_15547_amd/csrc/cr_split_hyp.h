// cr_split_hyp.h -- binary32-only (float-float) sinhf, coshf, tanhf.
//
// From the split exponential core (cr_split_exp.h), a = |x|:
//   e^a = 2^m y (y = T1 T2 (1 + q) in [0.68, 1.42]) gives, for m != 0,
//     sinh a = 2^(m-1) (y - 2^(-2m)/y),   cosh a = 2^(m-1) (y + 2^(-2m)/y),
//     tanh a = (y - 2^-m) / (y + 2^-m)     (with e^(2a) = 2^m y),
//   where the subtraction loses at most about one bit (m >= 1: y >= 0.68 and
//   2^(-2m)/y <= 0.37).
//   For m = 0 (a below about 0.35, or 2a for tanh) the cancellation is avoided
//   through E = e^a - 1 = W (the expm1 form, no cancellation near 0):
//     sinh a = (E + E/(E + 1))/2,   tanh a = E/(E + 2)   (E = e^(2a) - 1);
//   cosh a = 2^-1 (y + 1/y) needs no special form.
// The clamps (|x| <= 100 for sinh and cosh, 20 for tanh) keep m in range while
// the results still overflow or round to 1; beyond m = 30 the e^-a term is
// below 2^-60 of the result and its scale is frozen at 2^-60 (no underflow).
// Rounding test: relative bound 2^-42; failing lanes take the triple-float
// step of cr_split_acc.h.
#pragma once
#include "cr_f32_hyp.h"
#include "cr_split_exp.h"

namespace cr {

struct SHypTab {
  float2 t1[16], t2[16], d1[16], d2[16];
};

__device__ __forceinline__ void shyp_tab_load(SHypTab& t, int tid) {
  if (tid < 16) {
    t.t1[tid] = SEXP_T1[tid];
    t.t2[tid] = SEXP_T2[tid];
    t.d1[tid] = SEXP_D1[tid];
    t.d2[tid] = SEXP_D2[tid];
  }
}

template <int KIND>
__device__ __forceinline__ float shyp_fast(float xf, const SHypTab& tb, bool& ok) {
  float a = fminf(fabsf(xf), KIND == HYPK_TANH ? 20.0f : 100.0f);
  float xe = KIND == HYPK_TANH ? 2.0f * a : a;  // exact
  float kf;
  ff r = sexp_reduce<EXPK_E>(xe, kf);
  SExpDigits dg = sexp_digits(kf);
  const int m = dg.m;
  ff q = sexp_q(r);
  ff v;         // the result before the scaling by 2^sc
  int sc = 0;
  if (KIND != HYPK_COSH && m == 0) {
    ff E = sexp_W(tb.d1[dg.i1], tb.d2[dg.i0], q);
    if (KIND == HYPK_SINH) {
      ff d = ff_fast_two_sum(1.0f, E.hi);  // E > -0.3
      ff Q = ff_div(E, ff{d.hi, d.lo + E.lo});
      ff s = ff_two_sum(E.hi, Q.hi);
      v = {s.hi, s.lo + (E.lo + Q.lo)};
      sc = -1;
    } else {
      ff d = ff_fast_two_sum(2.0f, E.hi);
      v = ff_div(E, ff{d.hi, d.lo + E.lo});
    }
  } else {
    ff y = sexp_T(tb.t1[dg.i1], tb.t2[dg.i0], q);
    y = ff_fast_two_sum(y.hi, y.lo);
    const int mc = m < 30 ? m : 30;
    if (KIND == HYPK_TANH) {
      float p = pow2f_i(-mc);
      ff nu = ff_two_sum(y.hi, -p);
      ff de = ff_two_sum(y.hi, p);
      v = ff_div(ff{nu.hi, nu.lo + y.lo}, ff{de.hi, de.lo + y.lo});
    } else {
      ff iy = ff_div(ff{1.0f, 0.0f}, y);
      float p = pow2f_i(-2 * mc);
      ff w = {iy.hi * p, iy.lo * p};  // exact
      ff s = KIND == HYPK_SINH ? ff_two_sum(y.hi, -w.hi) : ff_two_sum(y.hi, w.hi);
      v = {s.hi, s.lo + (y.lo + (KIND == HYPK_SINH ? -w.lo : w.lo))};
      sc = m - 1;
    }
  }
  float res = ldexpf(round_split(v.hi, v.lo, fabsf(v.hi) * 0x1p-42f, ok), sc);
  if (KIND != HYPK_COSH && xf < 0.0f) res = -res;
  float sp;
  if (hyp_special(xf, KIND, sp)) {
    res = sp;
    ok = true;
  }
  return res;
}

}  // namespace cr
