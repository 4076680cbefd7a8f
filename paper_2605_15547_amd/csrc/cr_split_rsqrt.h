// cr_split_rsqrt.h -- correctly rounded rsqrtf without binary64 (device).
//
// As in cr_f32_rsqrt.h the rounding is decided exactly, here with the binary32
// hardware reciprocal square root and integer arithmetic only.  With
// x = Mx 2^ex and a positive normal float y1 = M1 2^e1, the midpoint between
// y1 and its successor is m = (2 M1 + 1) 2^(e1 - 1), and
//     1/sqrt(x) > m  <=>  m^2 x < 1  <=>  (2 M1 + 1)^2 Mx < 2^K,
//     K = -(2 e1 - 2 + ex),
// an integer comparison of a 74-bit product with a power of two (never equal:
// the product has the odd factor (2 M1 + 1)^2 > 1).  Starting from the
// hardware estimate (about 1 ulp), two correction rounds move the candidate to
// the float whose rounding interval holds 1/sqrt(x).
#pragma once
#include "cr_f32_rsqrt.h"

namespace cr {

__device__ __forceinline__ bool srsqrt_above(uint32_t yb, uint32_t Mx, int ex) {
  uint64_t M1 = (yb & 0x007fffffu) | 0x00800000u;
  int e1 = (int)(yb >> 23) - 150;
  uint64_t o = 2 * M1 + 1;
  uint64_t A = o * o;                           // < 2^50
  uint64_t lo = (A & 0xffffffffull) * Mx;       // < 2^56, odd low word: lo != 0
  uint64_t H = (A >> 32) * Mx + (lo >> 32);     // P = H 2^32 + (lo mod 2^32), H < 2^43
  int bl = H ? 96 - __clzll((long long)H) : 64 - __clzll((long long)lo);  // bit length of P
  int K = -(2 * e1 - 2 + ex);
  return bl <= K;
}

// rsqrt of a positive finite nonzero binary32 x
__device__ __forceinline__ float srsqrt_eval(float xf) {
  bool sub = f32_bits(xf) < 0x00800000u;
  float xs = sub ? xf * 0x1p24f : xf;  // exact
  uint32_t sb = f32_bits(xs);
  uint32_t Mx = (sb & 0x007fffffu) | 0x00800000u;
  int ex = (int)(sb >> 23) - 150;
  uint32_t yb = f32_bits(__builtin_amdgcn_rsqf(xs));
#pragma unroll
  for (int it = 0; it < 2; it++) {
    if (srsqrt_above(yb, Mx, ex)) yb += 1;             // above the upper midpoint
    else if (!srsqrt_above(yb - 1, Mx, ex)) yb -= 1;   // below the lower midpoint
  }
  float r = bits_f32(yb);
  return sub ? r * 0x1p12f : r;  // rsqrt(x) = rsqrt(x 2^24) 2^12, exact
}

__device__ __forceinline__ float srsqrt_fast(float xf, bool& ok) {
  ok = true;
  float sp;
  const bool s = rsqrt_special(xf, sp);
  const float r = srsqrt_eval(s ? 1.0f : xf);  // special inputs: any valid operand
  return s ? sp : r;
}

}  // namespace cr
