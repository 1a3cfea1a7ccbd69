// canon_math.h -- canonical binary32 exp and log for values that feed integer decisions.
//
// The preprocess derives the opacity, scales, shape modification and alpha-floor threshold with
// these two functions so that a decision (screen radius, tile rectangle, q <= q_max) never depends
// on which exp/log implementation a machine ships.  Method (Cody and Waite argument reduction with
// Taylor / atanh series):
//   exp(x): k = rint(x log2 e); r = (x - k ln2_hi) - k ln2_lo with ln2_hi = ln 2 truncated to 15
//           significant bits (k ln2_hi exact) and ln2_lo the binary32 rounding of the remainder;
//           exp(r) by the degree-7 Taylor polynomial in Horner form; times 2^k built in the
//           exponent field.  x > 88.72283935546875 -> +inf; x < -87.33654022216797 -> 0.
//   log(x): x = m 2^e with m in [sqrt(1/2), sqrt(2)]; s = (m-1)/(m+1);
//           log m = 2 (s + s^3/3 + s^5/5 + s^7/7 + s^9/9); log x = e ln2_hi + (e ln2_lo + log m).
// Every constant is the binary32 value nearest to its definition (1/k!, 1/k, log2 e, sqrt 2).
// All operations are single binary32 operations in the order written; files including this header
// are compiled with -ffp-contract=off so none of them fuse.
#pragma once
#include <hip/hip_runtime.h>

namespace ges {

__device__ __forceinline__ float canon_exp(float x) {
  if (x != x) return x;
  if (x > 88.72283935546875f) return __builtin_huge_valf();
  if (x < -87.33654022216797f) return 0.0f;
  const float kLog2e = 0x1.715476p+0f;
  const float kLn2Hi = 0x1.62e4p-1f;          // 0.693145751953125
  const float kLn2Lo = 0x1.7f7d1cp-20f;
  float k = __builtin_rintf(x * kLog2e);
  float r = x - k * kLn2Hi;
  r = r - k * kLn2Lo;
  float p = 0x1.a01a02p-13f;                   // 1/5040
  p = p * r; p = p + 0x1.6c16c2p-10f;         // 1/720
  p = p * r; p = p + 0x1.111112p-7f;          // 1/120
  p = p * r; p = p + 0x1.555556p-5f;          // 1/24
  p = p * r; p = p + 0x1.555556p-3f;          // 1/6
  p = p * r; p = p + 0.5f;
  p = p * r; p = p + 1.0f;
  p = p * r; p = p + 1.0f;
  int ki = (int)k;
  if (ki > 127) {
    p = p * __uint_as_float((uint32_t)(127 + 127) << 23);
    return p * 2.0f;
  }
  return p * __uint_as_float((uint32_t)(ki + 127) << 23);
}

__device__ __forceinline__ float canon_log(float x) {
  if (x != x) return x;
  if (x < 0.0f) return __builtin_nanf("");
  if (x == 0.0f) return -__builtin_huge_valf();
  if (x == __builtin_huge_valf()) return x;
  int e = 0;
  uint32_t b = __float_as_uint(x);
  if (b < 0x00800000u) {
    x = x * 8388608.0f;
    b = __float_as_uint(x);
    e = -23;
  }
  e += (int)((b >> 23) & 0xffu) - 127;
  float m = __uint_as_float((b & 0x007fffffu) | 0x3f800000u);
  if (m > 0x1.6a09e6p+0f) { m = m * 0.5f; e += 1; }
  float f = m - 1.0f;
  float den = m + 1.0f;
  float s = f / den;
  float s2 = s * s;
  float poly = 0x1.c71c72p-4f;                 // 1/9
  poly = poly * s2; poly = poly + 0x1.24924ap-3f;   // 1/7
  poly = poly * s2; poly = poly + 0x1.99999ap-3f;   // 1/5
  poly = poly * s2; poly = poly + 0x1.555556p-2f;   // 1/3
  poly = poly * s2;
  float lm = s * poly;
  lm = s + lm;
  lm = lm + lm;
  float ef = (float)e;
  float lo = ef * 0x1.7f7d1cp-20f;
  lo = lo + lm;
  float hi = ef * 0x1.62e4p-1f;
  return hi + lo;
}

// Canonical binary32 ln Gamma(x) for x > 0, for the exact shape modification 2 Gamma(3/b) / Gamma(1/b):
//   while x < 8: prod = prod * x; x = x + 1   (Gamma(x) = Gamma(x + k) / (x (x+1) ... (x+k-1)));
//   Stirling: (x - 1/2) ln x - x + ln(2 pi)/2 + (1/x) (1/12 - (1/x^2)(1/360 - (1/x^2)/1260));
//   minus ln prod.  Binary32 operations in the order written; constants the nearest binary32 values.
__device__ __forceinline__ float canon_lgamma(float x) {
  float prod = 1.0f;
  while (x < 8.0f) {
    prod = prod * x;
    x = x + 1.0f;
  }
  const float lz = canon_log(x);
  float t = x - 0.5f;
  t = t * lz;
  t = t - x;
  t = t + 0x1.d67f1cp-1f;                       // ln(2 pi) / 2
  const float iz = 1.0f / x;
  const float iz2 = iz * iz;
  float c = iz2 * 0x1.a01a02p-11f;              // 1/1260
  c = 0x1.6c16c2p-9f - c;                       // 1/360
  c = c * iz2;
  c = 0x1.555556p-4f - c;                       // 1/12
  c = c * iz;
  t = t + c;
  return t - canon_log(prod);
}

}  // namespace ges
