// OCP e4m3 ("e4m3fn") encoding and power-of-two scale selection on the device.
//
// e4m3: 1 sign, 4 exponent (bias 7), 3 mantissa bits, no infinities, NaN =
// 0x7F / 0xFF, largest finite 448, subnormals m * 2^-9.  Encoding rounds to
// the nearest value with ties to the even code, saturates magnitudes >= 448
// to 448, keeps the sign of values that round to zero and maps NaN to 0x7F.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mtk {

__device__ __forceinline__ uint32_t e4m3_encode_dev(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t sign = (u >> 24) & 0x80u;
  const uint32_t a = u & 0x7fffffffu;
  if (a > 0x7f800000u) return 0x7fu;                 // NaN
  if (a >= 0x43e00000u) return sign | 0x7eu;         // |x| >= 448 (and inf): saturate
  if (a >= 0x3c800000u) {                            // |x| >= 2^-6: normal e4m3
    // Round the binary32 mantissa to 3 bits, ties to even (carry may bump
    // the exponent, which is the correct next code).
    const uint32_t r = a + 0x7ffffu + ((a >> 20) & 1u);
    const uint32_t e = (r >> 23) - 120u;             // rebias 127 -> 7
    return sign | (e << 3) | ((r >> 20) & 7u);
  }
  // Subnormal e4m3: code = nearest integer (ties to even) of |x| * 2^9, in 0..8
  // (8 is the smallest normal, code 0x08).  Scaling by 2^9 is exact.
  const float m = __builtin_rintf(__uint_as_float(a) * 512.0f);
  return sign | static_cast<uint32_t>(m);
}

// Smallest e in [-126, 119] with amax <= 448 * 2^e; 0 for amax == 0 or not
// finite.  448 * 2^e is exact in binary32 over that range, so every
// comparison is exact.
__device__ __forceinline__ int scale_exponent_dev(float amax) {
  if (!(amax > 0.f) || !(amax <= 3.402823466e38f)) return 0;
  int e = ilogbf(amax) - 8;
  if (e < -126) e = -126;
  if (e > 119) e = 119;
  while (e < 119 && amax > ldexpf(448.f, e)) ++e;
  while (e > -126 && amax <= ldexpf(448.f, e - 1)) --e;
  return e;
}

}  // namespace mtk
