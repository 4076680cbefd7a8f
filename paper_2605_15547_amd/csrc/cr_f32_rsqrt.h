// cr_f32_rsqrt.h -- correctly rounded rsqrtf (device).
//
// rsqrtf is one of the paper's functions (Sec. II-A).  Its correct rounding
// can be decided exactly, so it needs no accurate path:
//  * y ~ 1/sqrt(x) from the hardware reciprocal square root (binary64) and
//    one Newton step, relative error far below one binary32 ulp, so
//    z = RN_f32(y) is the correct result or one of its neighbours;
//  * for a midpoint m next to z, 1/sqrt(x) > m  <=>  m^2 x < 1.  m has 25
//    significant bits, so m^2 is exact in binary64, and fma(m^2, x, -1) is the
//    exact m^2 x - 1 rounded once, whose sign is exact.  1/sqrt(x) is never a
//    midpoint itself (x = 2^(2e) / M^2 has no binary32 solution with M odd
//    > 1), so the comparisons are strict.
#pragma once
#include "cr_round.h"

namespace cr {

struct NoTab {
  int unused;
};

// Branch-free: res is always written (meaningful only when true is returned).
__device__ __forceinline__ bool rsqrt_special(float xf, float& res) {
  const bool nan = xf != xf;
  const bool zero = xf == 0.0f;  // rsqrt(+-0) = +-inf
  const bool neg = xf < 0.0f;
  const bool inf = xf == INFINITY;
  float v = inf ? 0.0f : bits_f32(0x7fc00000u);
  v = zero ? bits_f32((f32_bits(xf) & 0x80000000u) | 0x7f800000u) : v;
  res = nan ? bits_f32(f32_bits(xf) | 0x00400000u) : v;
  return nan | zero | neg | inf;
}

__device__ __forceinline__ float rsqrt_eval(float xf) {
  double x = (double)xf;
  double y = __builtin_amdgcn_rsq(x);
  // Newton step for 1/sqrt: y += y (1 - x y^2) / 2
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  float z = (float)y;
  // neighbouring midpoints of z (z is a positive normal binary32 here)
  uint32_t zb = f32_bits(z);
  double zd = (double)z;
  double half = __hiloint2double((int)(((zb >> 23) + (1023 - 127 - 24)) << 20), 0);  // ulp/2
  double mhi = zd + half;
  double mlo = (zb & 0x007fffffu) ? zd - half : zd - 0.5 * half;  // binade edge below
  if (fma(mhi * mhi, x, -1.0) < 0.0) zb += 1;       // 1/sqrt(x) above the upper midpoint
  else if (fma(mlo * mlo, x, -1.0) > 0.0) zb -= 1;  // below the lower midpoint
  return bits_f32(zb);
}

__device__ __forceinline__ float rsqrt_fast(float xf, bool& ok) {
  ok = true;
  float sp;
  const bool s = rsqrt_special(xf, sp);
  const float r = rsqrt_eval(s ? 1.0f : xf);  // special inputs: any valid operand
  return s ? sp : r;
}

}  // namespace cr
