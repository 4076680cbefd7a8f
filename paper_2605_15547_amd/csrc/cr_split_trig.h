// cr_split_trig.h -- binary32-only (float-float) sinf, cosf, sincosf, tanf.
//
// The reduction is the integer Payne-Hanek of cr_f32_trig.h (no floating
// point at all): k = nearest(x 32/pi), q = k mod 64 and the 128-bit fraction
// f = x 32/pi - k.  Here f is normalised (leading zeros counted over the 128
// bits) and its 48 leading bits become a float-float, so r = f pi/32 keeps a
// relative error of about 2^-46 however close x lies to a multiple of pi/32.
// With theta = q pi/32 from the 16-entry table (float-float sin and cos of
// j pi/32 and the quadrant symmetries):
//   sin x = S + S (cos r - 1) + C sin r,   cos x = C + C (cos r - 1) - S sin r,
//   sin r = r + r^3 (-1/6 + r^2/120 - r^4/5040 + r^6/9!),
//   cos r - 1 = -r^2/2 + r^4/24 + r^6 (-1/720 + r^2/8!)   (|r| <= pi/64),
// with r, r^2, r^3 (-1/6 + ...) and r^4/24 in float-float, the rest in binary32.
// For j = 0 the table terms are exactly 0 and +-1, so sin/cos of x near a
// multiple of pi/2 is +-sin r or +-(1 + (cos r - 1)) with no cancellation.
// tan x = sin x / cos x by a float-float division.
// Rounding tests: relative bound 2^-43 (2^-42 for tan); for reduced arguments
// an absolute floor of 2^-149 sends a (theoretical) fully cancelled f to the
// accurate path.  Failing lanes take the triple-float
// step of cr_split_acc.h.
#pragma once
#include "cr_f32_trig.h"
#include "cr_split.h"
#include "cr_split_consts.h"

namespace cr {

struct STrigTab {
  float4 sc[16];
  unsigned w[11];  // the words of 2/pi of the Payne-Hanek reduction
};

__device__ __forceinline__ void strig_tab_load(STrigTab& t, int tid) {
  if (tid < 16) t.sc[tid] = STRIG_T[tid];
  if (tid < 11) t.w[tid] = TWO_OVER_PI_W[tid];
}

// float-float product a b (|result| error ~2^-47 relative)
__device__ __forceinline__ ff ff_mul(ff a, ff b) {
  ff p = ff_two_prod(a.hi, b.hi);
  return {p.hi, fmaf(a.hi, b.lo, fmaf(a.lo, b.hi, p.lo))};
}

struct STrigCore {
  ff s, c;     // sin x and cos x for |x|
  bool small;  // |x| < pi/64 (no reduction)
};

__device__ __forceinline__ STrigCore strig_core(float xf, const STrigTab& tb) {
  uint32_t ax = f32_bits(xf) & 0x7fffffffu;
  float axf = bits_f32(ax);
  bool small = axf < STRIG_PI64;
  Reduced R = payne_hanek(ax, tb.w);
  // |f| as a normalised 128-bit integer: f = (fhi 2^64 + flo) 2^-128
  uint64_t hi = (uint64_t)R.fhi, lo = R.flo;
  bool neg = R.fhi < 0;
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
  int sft = hi ? __clzll((long long)hi) : 0;
  uint64_t top = sft ? ((hi << sft) | (lo >> (64 - sft))) : hi;
  int S = sft + extra;
  float fh = ldexpf((float)(uint32_t)(top >> 40), -24 - S);
  float fl = ldexpf((float)(uint32_t)((top >> 16) & 0xffffffu), -48 - S);
  if (neg) {
    fh = -fh;
    fl = -fl;
  }
  // r = f pi/32
  ff p = ff_two_prod(fh, STRIG_PI32_H);
  ff r = ff_fast_two_sum(p.hi, fmaf(fh, STRIG_PI32_L, fmaf(fl, STRIG_PI32_H, p.lo)));
  int q = R.q;
  if (small) {
    r = {axf, 0.0f};
    q = 0;
  }

  ff z = ff_two_prod(r.hi, r.hi);  // r^2
  z.lo = fmaf(2.0f * r.hi, r.lo, z.lo);
  float zh = z.hi;
  // sin r = r + r^3 s3
  float st = zh * fmaf(fmaf(STRIG_S9, zh, STRIG_S7), zh, STRIG_S5);
  ff s3 = ff_fast_two_sum(STRIG_S3_H, st);
  s3.lo += STRIG_S3_L;
  ff r3 = ff_two_prod(r.hi, zh);
  r3.lo = fmaf(r.hi, z.lo, fmaf(r.lo, zh, r3.lo));
  ff t = ff_mul(r3, s3);
  ff sr = ff_fast_two_sum(r.hi, t.hi);
  sr.lo += r.lo + t.lo;
  // cos r - 1 = -r^2/2 + r^4/24 + r^6 (-1/720 + r^2/8!)
  ff z2 = ff_two_prod(zh, zh);
  z2.lo = fmaf(2.0f * zh, z.lo, z2.lo);
  ff c4 = ff_mul(z2, ff{STRIG_C4_H, STRIG_C4_L});
  float c6 = (z2.hi * zh) * fmaf(STRIG_C8, zh, STRIG_C6);
  ff cm = ff_fast_two_sum(-0.5f * zh, c4.hi);
  cm.lo += -0.5f * z.lo + (c4.lo + c6);

  // theta = q pi/32 = quad pi/2 + j pi/32
  // the odd quadrants' swap picks which half of the table row is read
  const int quad = q >> 4;
  const int swap = quad & 1;
  const float2* row = reinterpret_cast<const float2*>(&tb.sc[q & 15]);
  const float2 S2 = row[swap], C2 = row[swap ^ 1];
  const uint32_t ms = (uint32_t)(quad >= 2) << 31;
  const uint32_t mc = (uint32_t)(quad == 1 || quad == 2) << 31;
  ff Sv = {bits_f32(f32_bits(S2.x) ^ ms), bits_f32(f32_bits(S2.y) ^ ms)};
  ff Cv = {bits_f32(f32_bits(C2.x) ^ mc), bits_f32(f32_bits(C2.y) ^ mc)};

  STrigCore o;
  o.small = small;
  {  // sin x = S + C sin r + S (cos r - 1)
    ff P2 = ff_mul(Cv, sr);
    ff P1 = ff_mul(Sv, cm);
    ff A = ff_fast_two_sum(Sv.hi, P2.hi);
    ff B = ff_fast_two_sum(A.hi, P1.hi);
    o.s = {B.hi, (A.lo + B.lo) + (Sv.lo + (P1.lo + P2.lo))};
  }
  {  // cos x = C - S sin r + C (cos r - 1)
    ff P2 = ff_mul(Sv, sr);
    ff P1 = ff_mul(Cv, cm);
    ff A = ff_fast_two_sum(Cv.hi, -P2.hi);
    ff B = ff_fast_two_sum(A.hi, P1.hi);
    o.c = {B.hi, (A.lo + B.lo) + (Cv.lo + (P1.lo - P2.lo))};
  }
  return o;
}

template <int KIND>
__device__ __forceinline__ float strig_fast(float xf, const STrigTab& tb, bool& ok) {
  STrigCore T = strig_core(xf, tb);
  const float floor_err = T.small ? 0.0f : 0x1p-149f;
  bool neg = xf < 0.0f;
  float res;
  if (KIND == TRIGK_COS) {
    res = round_split(T.c.hi, T.c.lo, fmaf(fabsf(T.c.hi), 0x1p-43f, floor_err), ok);
  } else if (KIND == TRIGK_SIN) {
    float h = neg ? -T.s.hi : T.s.hi, l = neg ? -T.s.lo : T.s.lo;
    res = round_split(h, l, fmaf(fabsf(h), 0x1p-43f, floor_err), ok);
  } else {
    // t = s / c: q1 = s/c, then one correction from the float-float residual
    float ic = __builtin_amdgcn_rcpf(T.c.hi);
    float q1 = T.s.hi * ic;
    ff pc = ff_two_prod(q1, T.c.hi);
    float rem = ((T.s.hi - pc.hi) - pc.lo) + fmaf(-q1, T.c.lo, T.s.lo);
    float q2 = rem * ic;
    float t2 = fmaf(rem - q2 * T.c.hi, ic, q2);  // second correction of the tail
    float h = neg ? -q1 : q1, l = neg ? -t2 : t2;
    res = round_split(h, l, fmaf(fabsf(h), 0x1p-42f, floor_err), ok);
  }
  float sp;
  if (trig_special(xf, sp, KIND)) {
    res = sp;
    ok = true;
  }
  return res;
}

__device__ __forceinline__ float ssincos_fast(float xf, const STrigTab& tb, float& c, bool& ok) {
  STrigCore T = strig_core(xf, tb);
  const float floor_err = T.small ? 0.0f : 0x1p-149f;
  bool neg = xf < 0.0f;
  float h = neg ? -T.s.hi : T.s.hi, l = neg ? -T.s.lo : T.s.lo;
  bool ok1, ok2;
  float s = round_split(h, l, fmaf(fabsf(h), 0x1p-43f, floor_err), ok1);
  c = round_split(T.c.hi, T.c.lo, fmaf(fabsf(T.c.hi), 0x1p-43f, floor_err), ok2);
  ok = ok1 && ok2;
  float sp;
  if (trig_special(xf, sp, TRIGK_SIN)) {
    s = sp;
    trig_special(xf, c, TRIGK_COS);
    ok = true;
  }
  return s;
}

}  // namespace cr
