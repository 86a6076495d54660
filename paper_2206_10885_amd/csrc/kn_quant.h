// Host-side rounding of weights to the low-precision march formats.
//   bfloat16: round to nearest even of the upper 16 bits of a float32.
//   OCP fp8 e4m3fn: 1 sign, 4 exponent (bias 7), 3 mantissa bits; normal
//     values 2^-6 .. 448, subnormals k * 2^-9; no infinities; 0x7F / 0xFF
//     are NaN.  Values are clamped to [-448, 448] (saturation), then
//     rounded to nearest, ties to even.
// Scales of the fp8 layers are powers of two, so scaling is exact.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>

namespace kn {

inline uint16_t bf16_bits(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  const uint32_t r = ((u >> 16) & 1u) + 0x7fffu;
  return (uint16_t)((u + r) >> 16);
}

inline float bf16_value(float x) {
  uint32_t u = (uint32_t)bf16_bits(x) << 16;
  float y;
  memcpy(&y, &u, 4);
  return y;
}

constexpr float kE4m3Max = 448.0f;

inline uint8_t e4m3_bits(float x) {
  const uint8_t sign = std::signbit(x) ? 0x80 : 0x00;
  double a = std::fabs((double)x);
  if (!(a <= kE4m3Max)) a = kE4m3Max;  // saturate (also catches +-inf)
  if (a < std::ldexp(1.0, -6)) {
    // subnormal: multiples of 2^-9 (8 of them reach the smallest normal)
    const double n = std::nearbyint(std::ldexp(a, 9));  // ties to even
    if (n >= 8.0) return sign | 0x08;                     // 2^-6
    return sign | (uint8_t)n;
  }
  int e;
  (void)std::frexp(a, &e);   // a = m * 2^e, m in [0.5, 1)
  int E = e - 1;             // a in [2^E, 2^(E+1))
  double n = std::nearbyint(std::ldexp(a, 3 - E));  // 8 .. 16
  if (n >= 16.0) {
    n = 8.0;
    ++E;
  }
  return sign | (uint8_t)((E + 7) << 3) | (uint8_t)((int)n - 8);
}

inline float e4m3_value(uint8_t b) {
  const int s = b >> 7, E = (b >> 3) & 15, m = b & 7;
  const double v = E == 0 ? std::ldexp((double)m, -9) : std::ldexp(1.0 + m / 8.0, E - 7);
  return (float)(s ? -v : v);
}

// smallest power of two s with bound / s <= 448 (bound > 0), else 1
inline float pow2_scale(double bound) {
  if (!(bound > 0.0) || !std::isfinite(bound)) return 1.0f;
  int e;
  (void)std::frexp(bound / kE4m3Max, &e);   // bound/448 in [2^(e-1), 2^e)
  double s = std::ldexp(1.0, e);
  if (bound / std::ldexp(1.0, e - 1) <= kE4m3Max) s = std::ldexp(1.0, e - 1);
  return (float)s;
}

}  // namespace kn
