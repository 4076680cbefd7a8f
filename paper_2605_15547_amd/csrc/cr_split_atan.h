// cr_split_atan.h -- binary32-only (float-float) atanf, asinf, acosf.
//
// The decomposition of cr_f32_atan.h in float-float arithmetic: with Y, X >= 0
//   atan x = atan(|x| / 1),  asin x = atan(|x| / s),  acos x = atan(s / x)
//   (x >= 0) or pi - atan(s / |x|) (x < 0),  s = sqrt(1 - x^2)  (float-float),
// and c = j/16 nearest to min(Y, X)/max(Y, X),
//   t = (Y - c X) / (X + c Y)  (or with Y, X swapped, from pi/2 - atan(c)),
// |t| <= 1/31, atan t = t - t^3/3 + t^5 P(t^2), P of degree 4 (Taylor;
// remainder below 2^-60 |t|).  c X and c Y are exact float-float products, the
// quotient takes one float-float correction step, and t and t^3/3 are
// float-float.  For j = 0 the table term is 0 and atan(Y/X) = atan(t) keeps
// its full relative accuracy (small arguments of atan and asin, acos near 1).
// Rounding test: relative bound 2^-42; failing lanes take the triple-float
// step of cr_split_acc.h.
#pragma once
#include "cr_f32_atan.h"
#include "cr_split.h"
#include "cr_split_consts.h"

namespace cr {

struct SAtanTab {
  float4 t[16];
};

__device__ __forceinline__ void satan_tab_load(SAtanTab& t, int tid) {
  if (tid < 16) t.t[tid] = SATAN_T[tid];
}

// atan(Y/X) as a float-float for float-float Y, X >= 0, not both zero
__device__ __forceinline__ ff satan_ratio(ff Y0, ff X0, const SAtanTab& tb) {
  bool inv = Y0.hi > X0.hi;
  ff Y = inv ? X0 : Y0, X = inv ? Y0 : X0;
  float zf = Y.hi * __builtin_amdgcn_rcpf(X.hi);  // index only
  int j = (int)rintf(16.0f * zf);
  j = j > 15 ? 15 : (j < 0 ? 0 : j);
  float c = (float)j * 0.0625f;
  // num = Y - c X, den = X + c Y
  ff cx = ff_two_prod(c, X.hi);
  ff n1 = ff_two_sum(Y.hi, -cx.hi);
  ff num = ff_two_sum(n1.hi, n1.lo + (Y.lo - fmaf(c, X.lo, cx.lo)));
  ff cy = ff_two_prod(c, Y.hi);
  ff d1 = ff_fast_two_sum(X.hi, cy.hi);  // X >= c Y
  float dlo = d1.lo + (X.lo + fmaf(c, Y.lo, cy.lo));
  // t = num / den: estimate, residual, two corrections
  float ic = __builtin_amdgcn_rcpf(d1.hi);
  float q1 = num.hi * ic;
  ff p = ff_two_prod(q1, d1.hi);
  float rem = ((num.hi - p.hi) - p.lo) + fmaf(-q1, dlo, num.lo);
  float q2 = rem * ic;
  q2 = fmaf(fmaf(-q2, d1.hi, rem), ic, q2);
  ff t = ff_fast_two_sum(q1, q2);
  // atan t = t - t^3/3 + t^5 P(t^2)
  ff sq = ff_two_prod(t.hi, t.hi);
  sq.lo = fmaf(2.0f * t.hi, t.lo, sq.lo);
  ff cu = ff_two_prod(t.hi, sq.hi);
  cu.lo = fmaf(t.hi, sq.lo, fmaf(t.lo, sq.hi, cu.lo));
  ff c3 = ff_two_prod(cu.hi, SATAN_THIRD_H);
  c3.lo = fmaf(cu.hi, SATAN_THIRD_L, fmaf(cu.lo, SATAN_THIRD_H, c3.lo));
  float z = sq.hi;
  float P = fmaf(fmaf(fmaf(fmaf(SATAN_P13, z, SATAN_P11), z, SATAN_P9), z, SATAN_P7), z, SATAN_P5);
  float t5 = (z * z) * t.hi * P;
  ff A = ff_fast_two_sum(t.hi, -c3.hi);
  ff at = {A.hi, A.lo + ((t.lo - c3.lo) + t5)};
  // base +- atan t
  float4 T = tb.t[j];
  float bh = inv ? T.z : T.x, bl = inv ? T.w : T.y;
  float sh = inv ? -at.hi : at.hi, sl = inv ? -at.lo : at.lo;
  ff B = ff_two_sum(bh, sh);
  return {B.hi, B.lo + (bl + sl)};
}

// sqrt(1 - a^2) as a float-float, a in [0, 1]
__device__ __forceinline__ ff ssqrt_1m_sq(float a) {
  ff p = ff_two_prod(a, a);
  ff w = ff_two_sum(1.0f, -p.hi);
  float wl = w.lo - p.lo;
  ff W = ff_fast_two_sum(w.hi, wl);
  if (!(W.hi > 0.0f)) return {0.0f, 0.0f};
  float s0 = sqrtf(W.hi);
  ff s2 = ff_two_prod(s0, s0);
  float r = ((W.hi - s2.hi) - s2.lo) + W.lo;
  return {s0, r * (0.5f * __builtin_amdgcn_rcpf(s0))};
}

template <int KIND>
__device__ __forceinline__ float satan_fast(float xf, const SAtanTab& tb, bool& ok) {
  // atan(2^100) and atan(inf) both round to RN(pi/2): clamp to keep 0 * inf out
  float a = fminf(fabsf(xf), 0x1p100f);
  bool neg = xf < 0.0f;
  ff y;
  if (KIND == ATANK_ATAN) {
    y = satan_ratio(ff{a, 0.0f}, ff{1.0f, 0.0f}, tb);
    if (neg) y = {-y.hi, -y.lo};
  } else {
    float ac = fminf(a, 1.0f);  // |x| > 1 is a special case (NaN)
    ff s = ssqrt_1m_sq(ac);
    if (KIND == ATANK_ASIN) {
      y = satan_ratio(ff{ac, 0.0f}, s, tb);
      if (neg) y = {-y.hi, -y.lo};
    } else {
      y = satan_ratio(s, ff{ac, 0.0f}, tb);
      // pi - atan(s/|x|) for x < 0, as selects (no branch)
      ff d = ff_two_sum(neg ? SATAN_PI_H : 0.0f, neg ? -y.hi : y.hi);
      y = {d.hi, d.lo + ((neg ? SATAN_PI_L : 0.0f) + (neg ? -y.lo : y.lo))};
    }
  }
  float res = round_split(y.hi, y.lo, fabsf(y.hi) * 0x1p-42f, ok);
  float sp;
  if (atan_special(xf, KIND, sp)) {
    res = sp;
    ok = true;
  }
  return res;
}

}  // namespace cr
