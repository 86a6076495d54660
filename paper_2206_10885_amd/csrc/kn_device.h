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

// OCP fp8 e4m3 (gfx950): 16x16x32 product with the same lane layout as the
// bfloat16 one (8 elements of K per lane).
__device__ __forceinline__ f32x4 mfma_fp8(long a, long b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

constexpr float kE4m3MaxF = 448.0f;

// eight float32 values (|x| <= 448) rounded to fp8 e4m3, nearest even
__device__ __forceinline__ long fp8x8(float a, float b, float c, float d, float e, float f, float g, float h) {
  int lo = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  lo = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, lo, true);
  int hi = __builtin_amdgcn_cvt_pk_fp8_f32(e, f, 0, false);
  hi = __builtin_amdgcn_cvt_pk_fp8_f32(g, h, hi, true);
  return (long)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// sin(2 pi r), cos(2 pi r) on the hardware units (input in revolutions).
__device__ __forceinline__ float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }
__device__ __forceinline__ float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }

// softplus_beta(u) = max(u, 0) + log1p(exp(-beta |u|)) / beta, evaluated as
// max(u,0) + log2(1 + 2^(-beta log2e |u|)) * ln2 / beta.
// max(u, 0) is written as (u + |u|) / 2, which is exact and avoids the NaN
// canonicalisation the compiler adds in front of v_max_f32.
// 2 softplus(u) = (u + |u|) + 2 ln(1 + e^(-beta |u|)) / beta
// (bit for bit twice softplus(): the factor 2 is exact in every step)
__device__ __forceinline__ float softplus_x2(float u, SoftplusK k) {
  float e = __builtin_amdgcn_exp2f(k.nbl2e * fabsf(u));
  return fmaf(__builtin_amdgcn_logf(1.0f + e), 2.0f * k.ln2b, u + fabsf(u));
}

// 2k softplus(u) from u' = k u with k = beta log2(e):
// u' + |u'| + 2 log2(1 + 2^(-|u'|)); the negated absolute value is a source
// modifier of the exponential, so the scale costs no instruction
__device__ __forceinline__ float softplus_x2k(float up) {
  float e = __builtin_amdgcn_exp2f(-fabsf(up));
  return fmaf(__builtin_amdgcn_logf(1.0f + e), 2.0f, up + fabsf(up));
}

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

// Per-lane description of the encoding slots this lane computes (the slot
// layout of pe_index: slots 3a, 3a + 1 and 3a + 2 read axis a in every lane
// group, slot 9 holds the raw coordinate or padding).
struct PeLane {
  float s0, s2;    // revolutions per unit of x: 2^(k-1) of slots 3a, 3a+1 (k = g) and 3a+2 (k = 4 + g%2)
  float d0, d2;    // derivative factors pi 2^k of the same slots
  float ph2;       // phase of slot 3a+2 in revolutions: 1/4 (a cosine) for g >= 2
  int g;
};

__host__ __device__ constexpr bool pe_layout_as_read() {
  for (int g = 0; g < 4; ++g) {
    if (pe_index(9, g) != (g < 3 ? g : -1)) return false;
    for (int a = 0; a < 3; ++a) {
      const int k2 = 4 + (g & 1);
      if (pe_index(3 * a, g) != 3 + 12 * a + 2 * g) return false;
      if (pe_index(3 * a + 1, g) != 3 + 12 * a + 2 * g + 1) return false;
      if (pe_index(3 * a + 2, g) != 3 + 12 * a + 2 * k2 + (g >= 2 ? 1 : 0)) return false;
    }
  }
  return true;
}
static_assert(pe_layout_as_read(), "the encoding evaluators read the slot layout of pe_index");

__device__ __forceinline__ PeLane make_pe_lane(int g) {
  PeLane L;
  L.g = g;
  L.s0 = ldexpf(1.0f, g - 1);
  L.s2 = ldexpf(1.0f, 3 + (g & 1));
  L.d0 = 3.14159265358979f * ldexpf(1.0f, g);
  L.d2 = 3.14159265358979f * ldexpf(1.0f, 4 + (g & 1));
  L.ph2 = g >= 2 ? 0.25f : 0.0f;
  return L;
}

// the raw coordinate of slot 9 (lane groups 0..2) or its padding (group 3)
__device__ __forceinline__ float pe_raw(int g, float x, float y, float z) {
  return g == 0 ? x : (g == 1 ? y : (g == 2 ? z : 0.0f));
}

// Encoding values of this lane's slots at local position (x, y, z).
// PHASE: slot 3a + 2 takes its cosines as sines a quarter revolution on
// (one transcendental instead of two and a select; the argument is rounded
// once more, by at most 2^-21 revolutions at the highest frequency, which
// the low-precision march evaluators round away with the layer input).
template <bool PHASE>
__device__ __forceinline__ void pe_values(const PeLane& L, float x, float y, float z,
                                          float (&v)[kPeSlots]) {
  const float xs[3] = {x, y, z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float r = xs[a] * L.s0;
    v[3 * a] = sin_rev(r);
    v[3 * a + 1] = cos_rev(r);
    if constexpr (PHASE) {
      v[3 * a + 2] = sin_rev(fmaf(xs[a], L.s2, L.ph2));
    } else {
      const float r2 = xs[a] * L.s2;
      v[3 * a + 2] = L.g < 2 ? sin_rev(r2) : cos_rev(r2);
    }
  }
  v[9] = pe_raw(L.g, x, y, z);
}

// Encoding values of a value column (s == 0) or of the derivative along
// world axis s-1 (s = 1..3; inv_half = 1/h of that axis) of this lane's
// slots, for forward-mode differentiation in the shading kernel.
__device__ __forceinline__ void pe_values_tangent(const PeLane& L, int s, float inv_half, float x,
                                                  float y, float z, float (&v)[kPeSlots]) {
  const float xs[3] = {x, y, z};
  const bool sin2 = L.g < 2;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float r = xs[a] * L.s0, r2 = xs[a] * L.s2;
    const float sn = sin_rev(r), cs = cos_rev(r), sn2 = sin_rev(r2), cs2 = cos_rev(r2);
    if (s == 0) {
      v[3 * a] = sn;
      v[3 * a + 1] = cs;
      v[3 * a + 2] = sin2 ? sn2 : cs2;
    } else {
      const bool on = a == s - 1;
      v[3 * a] = on ? cs * L.d0 * inv_half : 0.0f;
      v[3 * a + 1] = on ? -sn * L.d0 * inv_half : 0.0f;
      v[3 * a + 2] = on ? (sin2 ? cs2 : -sn2) * L.d2 * inv_half : 0.0f;
    }
  }
  v[9] = s == 0 ? pe_raw(L.g, x, y, z) : (L.g == s - 1 ? inv_half : 0.0f);
}

// Encoding values of a value column (value == true) or of the derivative
// along a direction whose local-coordinate rates are (tx, ty, tz) per axis.
__device__ __forceinline__ void pe_values_dir(const PeLane& L, bool value, float tx, float ty, float tz,
                                              float x, float y, float z, float (&v)[kPeSlots]) {
  const float xs[3] = {x, y, z}, ts[3] = {tx, ty, tz};
  const bool sin2 = L.g < 2;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float r = xs[a] * L.s0, r2 = xs[a] * L.s2;
    const float sn = sin_rev(r), cs = cos_rev(r), sn2 = sin_rev(r2), cs2 = cos_rev(r2);
    if (value) {
      v[3 * a] = sn;
      v[3 * a + 1] = cs;
      v[3 * a + 2] = sin2 ? sn2 : cs2;
    } else {
      v[3 * a] = cs * L.d0 * ts[a];
      v[3 * a + 1] = -sn * L.d0 * ts[a];
      v[3 * a + 2] = (sin2 ? cs2 : -sn2) * L.d2 * ts[a];
    }
  }
  v[9] = value ? pe_raw(L.g, x, y, z) : pe_raw(L.g, tx, ty, tz);
}

// LDS visibility between lanes of one wave (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// set bits of m (a mask over the wave) below this lane
__device__ __forceinline__ uint32_t lane_rank(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// value of lane (lane & ~3) + src within each quad
template <int SRC>
__device__ __forceinline__ float quad_bcast(float v) {
  constexpr int ctrl = SRC | (SRC << 2) | (SRC << 4) | (SRC << 6);
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), ctrl, 0xF,
                                                            0xF, false));
}

// value of the even lane of each lane pair
__device__ __forceinline__ float pair_bcast(float v) {
  constexpr int ctrl = 0 | (0 << 2) | (2 << 4) | (2 << 6);
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), ctrl, 0xF,
                                                            0xF, false));
}

// forward-mode groups: C columns per point, the value column first
template <int C>
__device__ __forceinline__ float group_bcast(float v) {
  if constexpr (C == 4) return quad_bcast<0>(v);
  else return pair_bcast(v);
}

// value of lane SRC of each lane pair (SRC = 0, 1)
template <int SRC>
__device__ __forceinline__ float pair_from(float v) {
  constexpr int ctrl = SRC | (SRC << 2) | ((2 + SRC) << 4) | ((2 + SRC) << 6);
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), ctrl, 0xF,
                                                            0xF, false));
}

// Forward-mode activation of one MFMA output block: z holds the lane's four
// units of its column, s = lane % C its column within the point (0: value).
// The value column takes softplus(z); a tangent column takes
// sigma(beta z_value) * dz.  Only the value column's four units need the
// softplus, so they are spread over the point's C adjacent lanes (C = 4: one
// unit each, C = 2: two each) and the results broadcast back: the same
// arithmetic as every lane evaluating its own, a quarter (a half) of it.
template <int C>
__device__ __forceinline__ void act_forward(const f32x4& z, int s, bool value_col, SoftplusK k, float (&a)[4]) {
  if constexpr (C == 4) {
    const float z0 = quad_bcast<0>(z[0]), z1 = quad_bcast<0>(z[1]);
    const float z2 = quad_bcast<0>(z[2]), z3 = quad_bcast<0>(z[3]);
    const float zs = s == 0 ? z0 : s == 1 ? z1 : s == 2 ? z2 : z3;
    float ds;
    const float sp = softplus_d(zs, k, &ds);
    const float sp_r[4] = {quad_bcast<0>(sp), quad_bcast<1>(sp), quad_bcast<2>(sp), quad_bcast<3>(sp)};
    const float ds_r[4] = {quad_bcast<0>(ds), quad_bcast<1>(ds), quad_bcast<2>(ds), quad_bcast<3>(ds)};
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = value_col ? sp_r[r] : ds_r[r] * z[r];
  } else {
    static_assert(C == 2, "two or four columns per point");
    const float z0 = pair_bcast(z[0]), z1 = pair_bcast(z[1]), z2 = pair_bcast(z[2]), z3 = pair_bcast(z[3]);
    const float za = s == 0 ? z0 : z1, zb = s == 0 ? z2 : z3;   // units s and s + 2
    float da, db;
    const float pa = softplus_d(za, k, &da), pb = softplus_d(zb, k, &db);
    const float sp_r[4] = {pair_from<0>(pa), pair_from<1>(pa), pair_from<0>(pb), pair_from<1>(pb)};
    const float ds_r[4] = {pair_from<0>(da), pair_from<1>(da), pair_from<0>(db), pair_from<1>(db)};
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = value_col ? sp_r[r] : ds_r[r] * z[r];
  }
}

// ---------------------------------------------------------------------------
// Path tracing helpers
// ---------------------------------------------------------------------------
// Philox-4x32-10 counter-based generator (Salmon et al., SC 2011): ten
// rounds of two 32x32 -> 64-bit products on counter words 0 and 2, the high
// halves xored into the other words with the key, the key stepped by the two
// Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

// uniform in [0, 1) from the top 24 bits
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

// the two uniforms of path (pixel, sample) at event k (0: pixel jitter,
// k >= 1: the k-th scatter)
__device__ __forceinline__ void path_uniforms(uint32_t seed_lo, uint32_t seed_hi, uint32_t pixel, uint32_t sample,
                                              uint32_t k, float* a, float* b) {
  const uint4 x = philox4x32_10(make_uint4(pixel, sample, k, 0u), make_uint2(seed_lo, seed_hi));
  *a = u01(x.x);
  *b = u01(x.y);
}

// cosine-weighted direction about the unit normal n, in the orthonormal
// basis of Duff et al. (JCGT 2017)
__device__ __forceinline__ void cosine_dir(const float n[3], float u1, float u2, float out[3]) {
  const float sign = n[2] >= 0.0f ? 1.0f : -1.0f;
  const float a = -1.0f / (sign + n[2]);
  const float b = n[0] * n[1] * a;
  const float b1[3] = {1.0f + sign * n[0] * n[0] * a, sign * b, -sign * n[0]};
  const float b2[3] = {b, sign + n[1] * n[1] * a, -n[1]};
  const float r = sqrtf(u1), phi = 6.283185307179586f * u2;
  float sp, cp;
  sincosf(phi, &sp, &cp);
  const float lx = r * cp, ly = r * sp, lz = sqrtf(fmaxf(1.0f - u1, 0.0f));
#pragma unroll
  for (int k = 0; k < 3; ++k) out[k] = lx * b1[k] + ly * b2[k] + lz * n[k];
}

// The same address as a pointer into global memory.  Pointers read from
// tables in memory are generic to the compiler; its flat accesses through them
// also count against the LDS wait counter, so that LDS waits after a flat
// store wait for the store.  Accesses through the cast are global.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// equirectangular environment [h][w][3]: u = 1/2 + atan2(d_x, -d_z) / 2 pi,
// v = acos(d_y) / pi; bilinear between texel centres, wrap in u, clamp in v
__device__ __forceinline__ void env_lookup(const float* env, uint32_t w, uint32_t h, const float d[3],
                                           float rgb[3]) {
  if (!env) {
    rgb[0] = rgb[1] = rgb[2] = 0.0f;
    return;
  }
  const float u = 0.5f + atan2f(d[0], -d[2]) * 0.15915494309189535f;
  const float v = acosf(fminf(fmaxf(d[1], -1.0f), 1.0f)) * 0.3183098861837907f;
  const float x = u * (float)w - 0.5f, y = v * (float)h - 0.5f;
  const float fx0 = floorf(x), fy0 = floorf(y);
  const float fx = x - fx0, fy = y - fy0;
  int x0 = (int)fx0 % (int)w;
  if (x0 < 0) x0 += (int)w;
  const int x1 = (x0 + 1) % (int)w;
  const int y0 = min(max((int)fy0, 0), (int)h - 1), y1 = min(max((int)fy0 + 1, 0), (int)h - 1);
  const auto r0 = gmem(env + (size_t)y0 * w * 3);
  const auto r1 = gmem(env + (size_t)y1 * w * 3);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float t0 = (1.0f - fx) * r0[3 * x0 + c] + fx * r0[3 * x1 + c];
    const float t1 = (1.0f - fx) * r1[3 * x0 + c] + fx * r1[3 * x1 + c];
    rgb[c] = (1.0f - fy) * t0 + fy * t1;
  }
}

}  // namespace kn
