// Device helpers for the CDNA4 (gfx950) kernels: MFMA wrappers, the per-lane
// Fourier encoding, softplus/sigmoid on the hardware exp2/log2 units, and
// wave-level utilities.  Wave size is 64; a 16-point MFMA tile maps point p
// to lanes p, p+16, p+32, p+48 (lane group g = lane / 16).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kn_internal.h"

namespace kn {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// sin(2 pi r), cos(2 pi r) on the hardware units (input in revolutions).
__device__ __forceinline__ float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }
__device__ __forceinline__ float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }

// softplus_beta(u) = max(u, 0) + log1p(exp(-beta |u|)) / beta, evaluated as
// max(u,0) + log2(1 + 2^(-beta log2e |u|)) * ln2 / beta.
// max(u, 0) is written as (u + |u|) / 2, which is exact and avoids the NaN
// canonicalisation the compiler adds in front of v_max_f32.
__device__ __forceinline__ float softplus(float u, SoftplusK k) {
  float e = __builtin_amdgcn_exp2f(k.nbl2e * fabsf(u));
  return fmaf(__builtin_amdgcn_logf(1.0f + e), k.ln2b, 0.5f * (u + fabsf(u)));
}
// softplus and its derivative sigmoid(beta u) from one exponential
__device__ __forceinline__ float softplus_d(float u, SoftplusK k, float* dsp) {
  float e = __builtin_amdgcn_exp2f(k.nbl2e * fabsf(u));
  float inv = __builtin_amdgcn_rcpf(1.0f + e);
  *dsp = u >= 0.0f ? inv : e * inv;
  return fmaxf(u, 0.0f) + __builtin_amdgcn_logf(1.0f + e) * k.ln2b;
}
__device__ __forceinline__ float sigmoid(float x) {
  float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * x);
  return __builtin_amdgcn_rcpf(1.0f + e);
}

__device__ __forceinline__ float bf16_round(float x) { return (float)(__bf16)x; }

// Per-lane description of the encoding slots this lane computes.
struct PeLane {
  uint32_t axes;     // 2 bits per slot: axis of the component (3 = padding)
  float scale[kPeSlots];   // 2^(k-1): revolutions per unit of x (sin/cos slots)
  float dscale[kPeSlots];  // pi 2^k: derivative factor of sin/cos slots
  int g;
};

__device__ __forceinline__ PeLane make_pe_lane(int g) {
  PeLane L;
  L.g = g;
  L.axes = 0;
#pragma unroll
  for (int j = 0; j < kPeSlots; ++j) {
    int idx = pe_index(j, g);
    int ax = idx < 0 ? 3 : (idx < 3 ? idx : (idx - 3) / 12);
    int k = idx < 3 ? 0 : ((idx - 3) % 12) / 2;
    L.axes |= (uint32_t)ax << (2 * j);
    L.scale[j] = ldexpf(1.0f, k - 1);
    L.dscale[j] = 3.14159265358979f * ldexpf(1.0f, k);
  }
  return L;
}

__device__ __forceinline__ float pick(uint32_t ax, float x, float y, float z) {
  return ax == 0 ? x : (ax == 1 ? y : z);
}

// Encoding values of this lane's slots at local position (x, y, z):
// slot 0 is raw (g < 3) or a sine (g == 3); slots 1..4 sines; 5..8 cosines;
// slot 9 sine (g == 0), cosine (g == 1, 2) or padding (g == 3).
__device__ __forceinline__ void pe_values(const PeLane& L, float x, float y, float z,
                                          float (&v)[kPeSlots]) {
  {
    float xa = pick(L.axes & 3u, x, y, z);
    float s = sin_rev(xa * L.scale[0]);
    v[0] = L.g == 3 ? s : xa;
  }
#pragma unroll
  for (int j = 1; j <= 4; ++j) v[j] = sin_rev(pick((L.axes >> (2 * j)) & 3u, x, y, z) * L.scale[j]);
#pragma unroll
  for (int j = 5; j <= 8; ++j) v[j] = cos_rev(pick((L.axes >> (2 * j)) & 3u, x, y, z) * L.scale[j]);
  {
    float r = pick((L.axes >> 18) & 3u, x, y, z) * L.scale[9];
    float s = sin_rev(r), c = cos_rev(r);
    v[9] = L.g == 0 ? s : (L.g == 3 ? 0.0f : c);
  }
}

// Encoding values of a value column (s == 0) or of the derivative along
// world axis s-1 (s = 1..3; inv_half = 1/h of that axis) of this lane's
// slots, for forward-mode differentiation in the shading kernel.
__device__ __forceinline__ void pe_values_tangent(const PeLane& L, int s, float inv_half, float x,
                                                  float y, float z, float (&v)[kPeSlots]) {
#pragma unroll
  for (int j = 0; j < kPeSlots; ++j) {
    uint32_t ax = (L.axes >> (2 * j)) & 3u;
    float xa = pick(ax, x, y, z);
    float r = xa * L.scale[j];
    float sn = sin_rev(r), cs = cos_rev(r);
    // kind of the slot for this lane group
    bool raw = (j == 0 && L.g < 3);
    bool pad = (j == 9 && L.g == 3);
    bool is_sin = (j == 0 && L.g == 3) || (j >= 1 && j <= 4) || (j == 9 && L.g == 0);
    float val;
    if (s == 0) {
      val = raw ? xa : (pad ? 0.0f : (is_sin ? sn : cs));
    } else {
      bool on = (int)ax == s - 1;
      float dv = raw ? 1.0f : (pad ? 0.0f : (is_sin ? cs * L.dscale[j] : -sn * L.dscale[j]));
      val = on ? dv * inv_half : 0.0f;
    }
    v[j] = val;
  }
}

// LDS visibility between lanes of one wave (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// value of lane (lane & ~3) + src within each quad
template <int SRC>
__device__ __forceinline__ float quad_bcast(float v) {
  constexpr int ctrl = SRC | (SRC << 2) | (SRC << 4) | (SRC << 6);
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), ctrl, 0xF,
                                                            0xF, false));
}

}  // namespace kn
