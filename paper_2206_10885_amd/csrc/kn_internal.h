// Internal definitions shared by the HIP kernels and the host runtime.
//
// Data layout in HBM (per render):
//   RayStatic[rid]   32 B  origin, box exit t_far, direction, output pixel
//   RayRec  lists    16 B  march state (t, t_entry, cell|steps, rid)
//     U  : rays for the next round; ray generation writes one per pixel,
//          the march writes each chunk's leavers into that chunk's range
//     S  : U counting-sorted by global cell (one bin per cell)
//     HL : hits, indexed by ray id (key 0xFFFFFFFF = no hit)
//   counts[2][cells] : per-cell arrivals for the current / next round
//   cursor[cells]    : scatter positions (bin starts)
//   chunks[2][]      : (cell | count << 22, start) work items of a round
//   chunk_out[2][]   : per chunk, rays leaving through each of the 6 faces
//   hit_count[cells] : hits binned by cell for shading
// Packed per-cell weights (built on the host, see runtime):
//   march block  : MFMA A-operand fragments of W1, W2 in per-lane order
//                  (float32, or bfloat16 bits), then float32 vectors
//                  b1[H], b2[H], w3row[H] (SDF output row), b3_0
//   shade block  : float32 fragments of W1, W2, W3 (all 16 rows), Wc1, Wc2
//                  plus b1, b2, b3[16], bc1[32], bc2[4]
#pragma once
#include <stdint.h>

namespace kn {

constexpr int kWave = 64;
constexpr int kSdfIn = 39;          // gamma_6 of a 3-vector (Sec. 3.1)
constexpr int kFeat = 15;           // feature z
constexpr int kColIn = 48;          // [x_l, gamma_4(v), n, z]
constexpr int kColHid = 32;
constexpr int kPeSlots = 10;        // encoding values computed per lane (4 lane groups x 10 = 40 K slots)
constexpr int kCellBits = 22;
constexpr uint32_t kCellMask = (1u << kCellBits) - 1u;
constexpr int kMaxSteps = 1023;     // steps live in the upper 10 bits of RayRec::key

// march status codes (also kn_trace_record::status)
enum : int32_t { kBoxMiss = 0, kHit = 1, kExitMiss = 2, kBudgetMiss = 3 };

struct RayRec {
  float t;
  float t_entry;
  uint32_t key;   // global cell | steps << 22
  uint32_t rid;
};

struct RayStatic {
  float ox, oy, oz, t_far;
  float dx, dy, dz;
  uint32_t pix;
};

struct TraceRec {   // mirrors kn_trace_record
  float t_march, t_entry;
  int32_t cell, status;
};

// Device-side counters of one render (zeroed per frame).
constexpr int kGroups = 8;          // work ranges, one per XCD-like group of workgroups
constexpr int kGroupStride = 32;    // words between range cursors (one 128-byte line each)

struct Ctrl {
  uint32_t n_chunks[3];    // chunks of the round with parity 0 / 1; of the hit binning
  uint32_t pad0;
  unsigned long long evals;  // SDF evaluations by the march
  unsigned long long tiles;  // 16-ray tiles evaluated by the march
  unsigned long long chunks; // march work items
  uint32_t n_hits;           // hits shaded
  uint32_t pad[3];
  uint32_t grab[kGroups * kGroupStride];  // work cursors of the current kernel, per range
  uint32_t grab0[kGroups * kGroupStride]; // their initial values
};

constexpr uint32_t kChunk = 256;    // rays per march work item (one per thread)

// Encoding slot assignment: lane group g (lane / 16) computes the values of
// slots j = 0..9; slot (j, g) holds gamma_6 component pe_index(j, g), or
// zero padding (-1).  Slots 1..4 hold only sines and 5..8 only cosines so a
// wave issues one transcendental per slot there.  Components: 0..2 raw
// x, y, z; 3 + 12a + 2k = sin(2^k pi x_a); 3 + 12a + 2k + 1 = cos(...).
__host__ __device__ constexpr int pe_sin(int m) { return 3 + 12 * (m / 6) + 2 * (m % 6); }
__host__ __device__ constexpr int pe_index(int j, int g) {
  return j == 0 ? (g < 3 ? g : pe_sin(0))
       : j <= 4 ? pe_sin(1 + 4 * (j - 1) + g)
       : j <= 8 ? pe_sin(4 * (j - 5) + g) + 1
       : (g == 0 ? pe_sin(17) : g == 1 ? pe_sin(16) + 1 : g == 2 ? pe_sin(17) + 1 : -1);
}

// Hidden-unit order of MFMA K positions for a layer whose input is the
// previous layer's MFMA output.  The previous output gives lane group g the
// units 16b + 4g + r (output block b, register r).
//   fp32 16x16x4 : K position 4q + g      <-> unit 16(q/4) + 4g + q%4
//   bf16 16x16x32: K position 32c + 8g + i <-> unit 16(2c + i/4) + 4g + i%4
__host__ __device__ constexpr int unit_f32(int q, int g) { return 16 * (q / 4) + 4 * g + (q % 4); }
__host__ __device__ constexpr int unit_bf16(int c, int g, int i) {
  return 16 * (2 * c + i / 4) + 4 * g + (i % 4);
}

// Constants of softplus_beta: nbl2e = -beta * log2(e), ln2b = ln(2) / beta.
struct SoftplusK {
  float nbl2e;
  float ln2b;
};

// Scene geometry as seen by the kernels.
struct SceneGeom {
  int32_t N;
  int32_t H;
  uint32_t cell_base;      // global cell id of this scene's cell 0
  float beta;
  float bmin[3];
  float bmax[3];
  float side[3];
  float inv_side[3];
  float half[3];
  float inv_half[3];
};

// Sizes (in 32-bit words) of the packed per-cell blocks.
__host__ __device__ constexpr int march_frag_words_f32(int H) {
  return 64 * ((H / 16) * kPeSlots + (H / 16) * (H / 4));
}
__host__ __device__ constexpr int march_frag_words_bf16(int H) {
  // (H/16) blocks x 2 K-chunks (layer 1, K padded to 64) + (H/16) x (H/32) (layer 2), 4 words/lane each
  return 64 * 4 * ((H / 16) * 2 + (H / 16) * (H / 32));
}
__host__ __device__ constexpr int march_vec_words(int H) { return 3 * H + 4; }
__host__ __device__ constexpr int march_block_words(int H, int bf16) {
  return (bf16 ? march_frag_words_bf16(H) : march_frag_words_f32(H)) + march_vec_words(H);
}
// shade block: W1 (NB*10), W2 (NB*H/4), W3 (H/4), Wc1 (2*12), Wc2 (8) fragments
// (one float per lane each), then b1[H], b2[H], b3[16], bc1[32], bc2[4]
__host__ __device__ constexpr int shade_frag_slots(int H) {
  return (H / 16) * kPeSlots + (H / 16) * (H / 4) + H / 4 + 2 * 12 + 8;
}
__host__ __device__ constexpr int shade_block_words(int H) {
  return 64 * shade_frag_slots(H) + 2 * H + 16 + kColHid + 4;
}

}  // namespace kn
