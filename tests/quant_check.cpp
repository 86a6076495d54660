// Test helper: exposes the host-side rounding of the scene packer
// (paper_2206_10885_amd/csrc/kn_quant.h) to ctypes.
#include <cstdint>

#include "../paper_2206_10885_amd/csrc/kn_quant.h"

extern "C" {
void e4m3_many(const float* x, uint8_t* out, int n) {
  for (int i = 0; i < n; ++i) out[i] = kn::e4m3_bits(x[i]);
}
void e4m3_decode(const uint8_t* b, float* out, int n) {
  for (int i = 0; i < n; ++i) out[i] = kn::e4m3_value(b[i]);
}
void bf16_many(const float* x, uint16_t* out, int n) {
  for (int i = 0; i < n; ++i) out[i] = kn::bf16_bits(x[i]);
}
float pow2_scale_of(double b) { return kn::pow2_scale(b); }
}
