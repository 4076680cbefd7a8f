// cr_split_log.h -- binary32-only (float-float) logf, log2f, log10f, log1pf.
//
// The reduction of the paper's logarithm (Sec. II-A, Fig. 2: an exponent, a
// tabulated reciprocal of the mantissa's leading bits, a polynomial in the
// reduced argument) in binary32 arithmetic, with two 16-entry reciprocal
// tables instead of one larger table.  With u = 2^e m, m in [0.75, 1.5):
//   c1 ~ 1/m (9 bits; 1 for the two intervals next to 1) from the mantissa's
//   top 4 bits, c2 ~ 1/(1 + i/112) (12 bits) from i = nearest(112 (m c1 - 1)),
//   so C = c1 c2 has at most 21 bits, m C is an exact float-float and
//   t = m C - 1 is exact (Sterbenz), |t| < 0.0048.
//   log u = e ln2 - log c1 - log c2 + log1p(t),
//   log1p(t) = t - t^2/2 + t^3/3 + t^4 P(t), P of degree 3 (Taylor; remainder
//   below 2^-57 |t|).  t, t^2/2 and t^3/3 are float-float, t^4 P(t) a float.
// log2 and log10 multiply the sum of the last three terms by 1/ln b
// (float-float) and add e log_b 2 (e for log2, exact).
// log1p: u = 1 + x is the exact pair uh + ul; ul enters t through
// (ul 2^-e) C, so t is still exact up to one rounding far below t's ulp.
// For u near 1 (c1 = c2 = 1, e = 0) t = u - 1 exactly and the result keeps its
// full relative accuracy (log1p of tiny x included).
// The rounding test uses a relative bound of 2^-43 (table entries 2^-49 of at
// most 0.29, the float-float sums a few 2^-49, against results >= 2^-9.2 when
// C != 1); failing lanes take the triple-float step of cr_split_acc.h.
#pragma once
#include "cr_f32_log.h"
#include "cr_split.h"
#include "cr_split_consts.h"

namespace cr {

struct SLogTab {
  float c1[16], c2[16];
  float2 L1[16], L2[16];
};

template <int K>
__device__ __forceinline__ void slog_tab_load(SLogTab& t, int tid) {
  if (tid < 16) {
    t.c1[tid] = SLOG_C1[tid];
    t.c2[tid] = SLOG_C2[tid];
    t.L1[tid] = SLOG_L1[tid];
    t.L2[tid] = SLOG_L2[tid];
  }
}

// NaN (quieted), zero and negative arguments, +inf, log1p(+-0) = +-0
// Branch-free: res is always written (meaningful only when true is returned).
template <int K>
__device__ __forceinline__ bool slog_special(float xf, float& res) {
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

template <int K>
__device__ __forceinline__ float slog_fast(float xf, const SLogTab& tb, bool& ok) {
  // u = uh + ul (log1p: 1 + x exactly; otherwise x); out-of-domain inputs are
  // replaced by 1 and fixed by the special-case select at the end
  float uh, ul = 0.0f;
  if (K == LOGK_1P) {
    float xs = (xf > -1.0f && xf < INFINITY) ? xf : 0.0f;
    ff u = ff_two_sum(1.0f, xs);
    uh = u.hi;
    ul = u.lo;
  } else {
    uh = (xf > 0.0f && xf < INFINITY) ? xf : 1.0f;
  }
  // subnormal inputs (log only): scale by 2^24
  int esub = 0;
  if (K != LOGK_1P && uh < 0x1p-126f) {
    uh *= 0x1p24f;
    esub = -24;
  }
  unsigned b = __float_as_uint(uh);
  int j = (b >> 19) & 15;
  int e = (int)((b >> 23) & 0xff) - 127 + esub;
  // m = mantissa in [1, 2), folded to [0.75, 1) when it is >= 1.5
  unsigned mb = (b & 0x007fffffu) | 0x3f800000u;
  int fold = j >= 8;
  mb -= fold ? 0x00800000u : 0u;
  e += fold;
  float m = __uint_as_float(mb);
  float ml = ldexpf(ul, -e);  // exact (log1p only; ul is 0 otherwise)

  float c1 = tb.c1[j];
  float t1 = fmaf(m, c1, -1.0f);  // index only
  int i = (int)rintf(t1 * SLOG_S);
  i = i < -8 ? -8 : (i > 7 ? 7 : i);
  float c2 = tb.c2[i + 8];
  float C = c1 * c2;  // exact: 9 + 12 bits
  ff p = ff_two_prod(m, C);
  float th0 = p.hi - 1.0f;  // exact
  ff t;
  if (K == LOGK_1P) {
    ff p2 = ff_two_prod(ml, C);
    ff S1 = ff_two_sum(p.lo, p2.hi);
    ff S2 = ff_two_sum(th0, S1.hi);
    t = ff_two_sum(S2.hi, S2.lo + (S1.lo + p2.lo));
  } else {
    t = ff_fast_two_sum(th0, p.lo);  // th0 = 0 or exponent(th0) >= exponent(p.lo)
  }

  // P = log1p(t) = t - t^2/2 + t^3/3 + t^4 (-1/4 + t/5 - t^2/6 + t^3/7)
  ff sq = ff_two_prod(t.hi, t.hi);
  sq.lo = fmaf(2.0f * t.hi, t.lo, sq.lo);
  ff cu = ff_two_prod(t.hi, sq.hi);
  cu.lo = fmaf(t.hi, sq.lo, fmaf(t.lo, sq.hi, cu.lo));
  ff c3 = ff_two_prod(cu.hi, SLOG_THIRD_H);
  c3.lo = fmaf(cu.hi, SLOG_THIRD_L, fmaf(cu.lo, SLOG_THIRD_H, c3.lo));
  float pt = fmaf(fmaf(fmaf(SLOG_P7, t.hi, SLOG_P6), t.hi, SLOG_P5), t.hi, SLOG_P4);
  float tail = (sq.hi * sq.hi) * pt;
  ff A = ff_fast_two_sum(t.hi, -0.5f * sq.hi);
  ff B = ff_fast_two_sum(A.hi, c3.hi);
  float plo = (A.lo + B.lo) + ((t.lo - 0.5f * sq.lo) + (c3.lo + tail));

  // Z = -log c1 - log c2 + P
  float2 L1 = tb.L1[j], L2 = tb.L2[i + 8];
  ff Z1 = ff_two_sum(L1.x, L2.x);
  ff Z2 = ff_two_sum(Z1.hi, B.hi);
  ff Z = {Z2.hi, Z2.lo + (Z1.lo + ((L1.y + L2.y) + plo))};
  if (K == LOGK_2 || K == LOGK_10) {
    const float kh = K == LOGK_2 ? SLOG_INV_LN2_H : SLOG_INV_LN10_H;
    const float kl = K == LOGK_2 ? SLOG_INV_LN2_L : SLOG_INV_LN10_L;
    ff P = ff_two_prod(Z.hi, kh);
    Z = {P.hi, fmaf(Z.hi, kl, fmaf(Z.lo, kh, P.lo))};
  }
  // y = e log_b(2) + Z
  float ef = (float)e;
  float yh, yl;
  if (K == LOGK_2) {
    ff S = ff_two_sum(ef, Z.hi);
    yh = S.hi;
    yl = S.lo + Z.lo;
  } else {
    const float k1 = K == LOGK_10 ? SLOG_LG2_H : SLOG_LN2_H;
    const float k2 = K == LOGK_10 ? SLOG_LG2_M : SLOG_LN2_M;
    const float k3 = K == LOGK_10 ? SLOG_LG2_L : SLOG_LN2_L;
    ff E2 = ff_two_prod(ef, k2);
    ff S1 = ff_two_sum(ef * k1, Z.hi);  // e k1 is exact
    ff S2 = ff_two_sum(S1.hi, E2.hi);
    yh = S2.hi;
    yl = (S1.lo + S2.lo) + (Z.lo + fmaf(ef, k3, E2.lo));
  }
  float res = round_split(yh, yl, fabsf(yh) * 0x1p-43f, ok);
  float sp;
  if (slog_special<K>(xf, sp)) {
    res = sp;
    ok = true;
  }
  return res;
}

}  // namespace cr
