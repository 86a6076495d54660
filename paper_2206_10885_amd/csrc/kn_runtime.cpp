// Host runtime of the C ABI (include/kn.h): contexts, scene packing, the
// per-frame round driver, the point query, and the serving loop.
#include <hip/hip_runtime.h>
#include <link.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/kn.h"
#include "kn_launch.h"
#include "kn_quant.h"

using namespace kn;

namespace {

thread_local std::string g_err;

kn_status fail(kn_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

// Paths of the HIP runtimes (libamdhip64.so*) mapped into this process.  A
// process that loads this library before another program's own copy of the
// runtime (torch wheels ship one, with a different file name) ends up with
// two: each keeps its own devices, streams and allocations, and a pointer or
// stream of one passed to the other crashes the process.
std::vector<std::string> hip_runtimes_loaded() {
  std::vector<std::string> found;
  dl_iterate_phdr(
      [](struct dl_phdr_info* info, size_t, void* data) -> int {
        auto* v = static_cast<std::vector<std::string>*>(data);
        const char* path = info->dlpi_name ? info->dlpi_name : "";
        const char* base = std::strrchr(path, '/');
        base = base ? base + 1 : path;
        if (std::strncmp(base, "libamdhip64.so", 14) == 0 &&
            std::find(v->begin(), v->end(), std::string(path)) == v->end())
          v->push_back(path);
        return 0;
      },
      &found);
  return found;
}

constexpr uint32_t kShadeChunk = 64;    // hits per shading work item
constexpr uint32_t kQueryChunk = 256;   // points per query work item
constexpr uint32_t kGridMaxR = 4096;    // lattice points per axis of kn_grid_sample
constexpr uint64_t kEikMaxPoints = (1ull << 28) / 6u;   // stencil points fit one point query

}  // namespace

// ---------------------------------------------------------------------------
// scene packing (host): per-cell MFMA fragment blocks, see kn_internal.h
// ---------------------------------------------------------------------------
namespace kn {

struct SdfView {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
};

static SdfView sdf_view(const float* blk, int H) {
  SdfView v;
  v.W1 = blk;
  v.b1 = v.W1 + kSdfIn * H;
  v.W2 = v.b1 + H;
  v.b2 = v.W2 + H * H;
  v.W3 = v.b2 + H;
  v.b3 = v.W3 + 16 * H;
  return v;
}

static void pack_march_f32(const float* blk, int H, float* out) {
  const SdfView w = sdf_view(blk, H);
  const int NB = H / 16, S1 = NB * kPeSlots, SF = S1 + NB * (H / 4);
  for (int s = 0; s < SF; ++s) {
    for (int lane = 0; lane < 64; ++lane) {
      const int m = lane % 16, g = lane / 16;
      float val;
      if (s < S1) {
        const int b = s / kPeSlots, q = s % kPeSlots, idx = pe_index(q, g);
        val = idx < 0 ? 0.0f : w.W1[(16 * b + m) * kSdfIn + idx];
      } else {
        const int s2 = s - S1, b = s2 / (H / 4), q = s2 % (H / 4);
        val = 0.5f * w.W2[(16 * b + m) * H + unit_f32(q, g)];   // layer 1 hands on 2 softplus
      }
      out[(s / 4) * 256 + lane * 4 + (s % 4)] = val;
    }
  }
  float* vec = out + 64 * SF;
  for (int j = 0; j < H; ++j) {
    vec[j] = w.b1[j];
    vec[H + j] = w.b2[j];
    vec[2 * H + j] = 0.5f * w.W3[j];
  }
  vec[3 * H] = w.b3[0];
  vec[3 * H + 1] = vec[3 * H + 2] = vec[3 * H + 3] = 0.0f;
}

// SDF output row as bfloat16 MFMA A fragments, K order of the layer-2
// outputs: row 0 = hi = bf16(w), row 1 = lo = bf16(w - hi) for the row
// w = `scale` x W3[0] rounded to float32 (the two product rows add up to the
// row at about 2^-16 relative); rows 2..15 zero
static void pack_w3_bf16(const SdfView& w, int H, double scale, uint16_t* out) {
  for (int c = 0; c < H / 32; ++c)
    for (int lane = 0; lane < 64; ++lane) {
      const int m = lane % 16, g = lane / 16;
      for (int i = 0; i < 8; ++i) {
        const float x = (float)(scale * w.W3[unit_bf16(c, g, i)]);
        const float hi = bf16_value(x);
        out[((size_t)c * 64 + lane) * 8 + i] = bf16_bits(m == 0 ? hi : m == 1 ? x - hi : 0.0f);
      }
    }
}

// bfloat16 march block.  The two hidden layers work on u' = k u with
// k = beta log2(e): W1, b1 and b2 are stored times k, so the activation
// 2k softplus(u) = u' + |u'| + 2 log2(1 + 2^(-|u'|)) needs no scaling
// multiply; W2 keeps the factor 1/2 of the other blocks and the output row
// takes 1/(2k).
static void pack_march_bf16(const float* blk, int H, float beta, float* out_words) {
  const SdfView w = sdf_view(blk, H);
  const double k = (double)beta / std::log(2.0);
  const int NB = H / 16, F1 = NB * 2, NF = F1 + NB * (H / 32);
  uint16_t* out = reinterpret_cast<uint16_t*>(out_words);
  for (int f = 0; f < NF; ++f) {
    for (int lane = 0; lane < 64; ++lane) {
      const int m = lane % 16, g = lane / 16;
      for (int i = 0; i < 8; ++i) {
        float val;
        if (f < F1) {
          const int b = f / 2, c = f % 2, j = 8 * c + i;
          const int idx = j < kPeSlots ? pe_index(j, g) : -1;
          val = idx < 0 ? 0.0f : (float)(k * w.W1[(16 * b + m) * kSdfIn + idx]);
        } else {
          const int f2 = f - F1, b = f2 / (H / 32), c = f2 % (H / 32);
          val = 0.5f * w.W2[(16 * b + m) * H + unit_bf16(c, g, i)];   // layer 1 hands on 2k softplus
        }
        out[((size_t)f * 64 + lane) * 8 + i] = bf16_bits(val);
      }
    }
  }
  pack_w3_bf16(w, H, 0.5 / k, out + (size_t)NF * 64 * 8);
  const int NFW = NF + H / 32;
  float* vec = out_words + 64 * 4 * NFW;
  for (int j = 0; j < H; ++j) {
    vec[j] = (float)(k * w.b1[j]);
    vec[H + j] = (float)(k * w.b2[j]);
    vec[2 * H + j] = bf16_value(w.W3[j]);
  }
  vec[3 * H] = w.b3[0];
  vec[3 * H + 1] = vec[3 * H + 2] = vec[3 * H + 3] = 0.0f;
}

static double softplus_host(double u, double beta) {
  return std::max(u, 0.0) + std::log1p(std::exp(-beta * std::fabs(u))) / beta;
}

// fp8 e4m3 march block: W1 and W2 scaled by power-of-two per-layer scales
// (absmax / 448 rounded up); the layer-2 input scale from a bound on the
// layer-1 activations over inputs with |e_k| <= 1:
//   a1_j <= softplus(sum_k |W1[j][k]| + b1[j]).
// As in the bfloat16 block the first hidden layer works on u' = k u
// (k = beta log2(e)), here through its dequantisation scale and bias: the
// e4m3 layer-2 inputs are the same numbers; layer 2 keeps the plain scale.
static void pack_march_fp8(const float* blk, int H, float beta, float* out_words) {
  const SdfView w = sdf_view(blk, H);
  const double k = (double)beta / std::log(2.0);
  const int NB = H / 16, F1 = NB * 2, NF = F1 + NB * (H / 32);
  double m1 = 0.0, m2 = 0.0, abound = 0.0;
  for (int j = 0; j < H; ++j) {
    double row = 0.0;
    for (int k = 0; k < kSdfIn; ++k) {
      m1 = std::max(m1, (double)std::fabs(w.W1[j * kSdfIn + k]));
      row += std::fabs((double)w.W1[j * kSdfIn + k]);
    }
    abound = std::max(abound, softplus_host(row + w.b1[j], beta));
    for (int k = 0; k < H; ++k) m2 = std::max(m2, (double)std::fabs(w.W2[j * H + k]));
  }
  const float s1 = pow2_scale(m1), s2 = pow2_scale(m2), sa = pow2_scale(abound * 1.01);
  uint8_t* out = reinterpret_cast<uint8_t*>(out_words);
  for (int f = 0; f < NF; ++f) {
    for (int lane = 0; lane < 64; ++lane) {
      const int m = lane % 16, g = lane / 16;
      for (int i = 0; i < 8; ++i) {
        float val;
        if (f < F1) {
          const int b = f / 2, c = f % 2, j = 8 * c + i;
          const int idx = j < kPeSlots ? pe_index(j, g) : -1;
          val = idx < 0 ? 0.0f : w.W1[(16 * b + m) * kSdfIn + idx] / s1;
        } else {
          const int f2 = f - F1, b = f2 / (H / 32), c = f2 % (H / 32);
          val = w.W2[(16 * b + m) * H + unit_bf16(c, g, i)] / s2;
        }
        out[((size_t)f * 64 + lane) * 8 + i] = e4m3_bits(val);
      }
    }
  }
  pack_w3_bf16(w, H, 0.5, reinterpret_cast<uint16_t*>(out_words + 2 * 64 * NF));
  float* vec = out_words + 2 * 64 * NF + 4 * 64 * (H / 32);
  for (int j = 0; j < H; ++j) {
    vec[j] = (float)(k * w.b1[j]);
    vec[H + j] = w.b2[j];
    vec[2 * H + j] = bf16_value(w.W3[j]);
  }
  vec[3 * H] = w.b3[0];
  vec[3 * H + 1] = (float)(k * s1);
  vec[3 * H + 2] = s2 * sa;
  vec[3 * H + 3] = (float)(0.5 / (sa * k));   // layer 1 hands on 2k softplus
}

static void pack_shade(const float* blk, const float* cblk, int H, float* out) {
  const SdfView w = sdf_view(blk, H);
  const float* Wc1 = cblk;
  const float* bc1 = Wc1 + kColIn * kColHid;
  const float* Wc2 = bc1 + kColHid;
  const float* bc2 = Wc2 + 3 * kColHid;
  const int NB = H / 16, S1 = NB * kPeSlots, S2 = S1 + NB * (H / 4), S3 = S2 + H / 4, S4 = S3 + 24;
  const int ST = shade_frag_slots(H);
  for (int s = 0; s < ST; ++s) {
    for (int lane = 0; lane < 64; ++lane) {
      const int m = lane % 16, g = lane / 16;
      float val;
      if (s < S1) {
        const int b = s / kPeSlots, q = s % kPeSlots, idx = pe_index(q, g);
        val = idx < 0 ? 0.0f : w.W1[(16 * b + m) * kSdfIn + idx];
      } else if (s < S2) {
        const int s2 = s - S1, b = s2 / (H / 4), q = s2 % (H / 4);
        val = w.W2[(16 * b + m) * H + unit_f32(q, g)];
      } else if (s < S3) {
        val = w.W3[m * H + unit_f32(s - S2, g)];
      } else if (s < S4) {
        const int t = s - S3, b = t / 12, q = t % 12;
        val = Wc1[(16 * b + m) * kColIn + 4 * q + g];
      } else {
        const int q = s - S4;
        val = m < 3 ? Wc2[m * kColHid + unit_f32(q, g)] : 0.0f;
      }
      out[s * 64 + lane] = val;
    }
  }
  float* vec = out + 64 * ST;
  for (int j = 0; j < H; ++j) {
    vec[j] = w.b1[j];
    vec[H + j] = w.b2[j];
  }
  for (int o = 0; o < 16; ++o) vec[2 * H + o] = w.b3[o];
  for (int j = 0; j < kColHid; ++j) vec[2 * H + 16 + j] = bc1[j];
  for (int c = 0; c < 3; ++c) vec[2 * H + 16 + kColHid + c] = bc2[c];
  vec[2 * H + 16 + kColHid + 3] = 0.0f;
}

// Split-bfloat16 shading block: every weight w of the SDF MLP as hi =
// bf16(w) and lo = bf16(w - hi), in the bf16 march's fragment layout (W1, W2
// and W3 unhalved, all 16 rows of W3); the colour fragments and the biases
// are the float32 block's.
static void pack_shade3(const float* blk, const float* cblk, int H, float* out_words) {
  const SdfView w = sdf_view(blk, H);
  const int NB = H / 16, F1 = NB * 2, F2 = F1 + NB * (H / 32), NF = shade3_frags(H);
  uint16_t* hi = reinterpret_cast<uint16_t*>(out_words);
  uint16_t* lo = hi + (size_t)NF * 64 * 8;
  for (int f = 0; f < NF; ++f)
    for (int lane = 0; lane < 64; ++lane) {
      const int m = lane % 16, g = lane / 16;
      for (int i = 0; i < 8; ++i) {
        float val;
        if (f < F1) {
          const int b = f / 2, c = f % 2, j = 8 * c + i;
          const int idx = j < kPeSlots ? pe_index(j, g) : -1;
          val = idx < 0 ? 0.0f : w.W1[(16 * b + m) * kSdfIn + idx];
        } else if (f < F2) {
          const int f2 = f - F1, b = f2 / (H / 32), c = f2 % (H / 32);
          val = w.W2[(16 * b + m) * H + unit_bf16(c, g, i)];
        } else {
          val = w.W3[m * H + unit_bf16(f - F2, g, i)];
        }
        const size_t at = ((size_t)f * 64 + lane) * 8 + i;
        hi[at] = bf16_bits(val);
        lo[at] = bf16_bits(val - bf16_value(val));
      }
    }
  // colour fragments and biases, copied from the float32 block
  std::vector<float> f32((size_t)shade_block_words(H));
  pack_shade(blk, cblk, H, f32.data());
  const int S3 = NB * kPeSlots + NB * (H / 4) + H / 4, ST = shade_frag_slots(H);
  float* rest = out_words + 2 * 256 * NF;
  std::copy(f32.begin() + 64 * S3, f32.end(), rest);
  static_assert(2 * 12 + 8 == 32, "colour fragments");
  (void)ST;
}

}  // namespace kn

// ---------------------------------------------------------------------------
// context and scenes
// ---------------------------------------------------------------------------
struct KnScene {
  kn_scene_id id = 0;
  SceneGeom geom{};
  int N = 0, H = 0;
  float* march_f32 = nullptr;
  float* march_bf16 = nullptr;
  float* march_fp8 = nullptr;
  float* shade = nullptr;    // float32 shading blocks (float32 pools, point queries)
  float* shade3 = nullptr;   // split-bfloat16 shading blocks (bf16 and fp8 pools)
  uint32_t march_f32_words = 0, march_bf16_words = 0, march_fp8_words = 0, shade_words = 0, shade3_words = 0;

  const float* march(int prec) const {
    return prec == KN_BF16 ? march_bf16 : prec == KN_FP8_E4M3 ? march_fp8 : march_f32;
  }
  uint32_t march_words(int prec) const {
    return prec == KN_BF16 ? march_bf16_words : prec == KN_FP8_E4M3 ? march_fp8_words : march_f32_words;
  }
  const float* shading(int prec) const { return prec == KN_FP32 ? shade : shade3; }
  uint32_t shading_words(int prec) const { return prec == KN_FP32 ? shade_words : shade3_words; }
  size_t bytes = 0;
  std::atomic<int> refs{0};
  int world_refs = 0;      // worlds that place this scene (under kn_ctx::mu)
};

// A world (shared scenes): instances of resident scenes and primitives on
// the device.
struct KnWorld {
  kn_world_id id = 0;
  std::vector<kn_instance> inst;
  std::vector<KnScene*> scenes;    // per instance
  PrimDev* prims = nullptr;        // [n_prims] on the device
  uint32_t n_prims = 0;
  uint32_t cells = 0;              // global cells of the instances
  size_t bytes = 0;
  std::atomic<int> refs{0};
};

// Device buffers of a ray pool: up to `cap` rays (ids 0..cap-1) over
// `cells` global cells (record layouts in kn_internal.h).
struct Pool {
  size_t cap = 0, cells = 0, chunks = 0;
  RayStatic* rs = nullptr;
  RayRec* U = nullptr;             // next-round records, in the ranges of the round's chunks
  RayRec* S = nullptr;             // a round's records sorted by cell
  RayRec* Uin = nullptr;           // records of newly generated rays
  RayRec* HL = nullptr;            // hit list since the last shading pass
  PathRec* path = nullptr;         // path tracing state (allocated on first use)
  RayRec* J = nullptr;             // [2][cap]: rays of unclamped steps that jumped cells, per
                                   // round parity (allocated on first use)
  WorldRec* W = nullptr;           // [2][cap]: world renders, rays waiting for their next object
  WState* WS = nullptr;            // [cap]: world renders, each ray's segment origin
  // primary frames whose hits are shaded in two passes, the first one on a
  // second stream while the last rounds run (allocated on first use): the
  // later rounds' per-cell hit counts, and the first pass's cursors and
  // control block (its bins are Uin, which a primary frame uses only to
  // bring its camera rays into round 0)
  uint32_t* hit_count2 = nullptr;  // [cells * cs]
  uint32_t* cursor2 = nullptr;     // [cells * cs]
  Ctrl* ctrl2 = nullptr;
  // per-cell counters, cell c at word c * cs: on grids of up to
  // kPadCells cells each counter has a 128-byte line of its own
  uint32_t cs = 1;
  uint32_t* counts = nullptr;      // [2][cells * cs]: new records arriving for a round
  uint32_t* runs = nullptr;        // [2][cells * cs]: rays handed on by the previous round's chunks
  uint32_t* hit_count = nullptr;   // [cells * cs]
  uint32_t* cursor = nullptr;      // [cells * cs]
  uint32_t* base = nullptr;        // [cells]: bin starts of the current round
  uint2* chunk = nullptr;          // [4][chunks]: rounds of parity 0 / 1, shading, early shading
  uint4* chunk_out = nullptr;      // [2][chunks][4]
  Ctrl* ctrl = nullptr;
  SceneEnt* scenes = nullptr;      // [kMaxScenes]
  ReqEnt* reqs = nullptr;          // [kMaxSlots]
  size_t bytes = 0;
};

namespace kn {
class ServeLoop;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free point query (kn_query_noalloc): one array
// per GPU, in the library's code object, holding the query's records,
// per-cell counters, work items and control block for up to
// kNoAllocMaxPoints points over up to kNoAllocMaxCells cells.  Host code
// never uses the array's name as an address: each context looks up its
// device's address once (hipGetSymbolAddress, in kn_ctx_create) and passes
// that pointer to the kernels.
// ---------------------------------------------------------------------------
constexpr uint32_t kNoAllocMaxPoints = 1u << 18;
constexpr uint32_t kNoAllocMaxCells = 1u << 18;   // every grid_n <= 64

namespace {
constexpr size_t align256(size_t x) { return (x + 255u) & ~(size_t)255u; }

struct NoAllocLayout {
  size_t ctrl, counts, cursor, chunks, U, S, bytes;
};

constexpr NoAllocLayout noalloc_layout() {
  NoAllocLayout L{};
  L.ctrl = 0;
  L.counts = align256(sizeof(Ctrl));
  L.cursor = L.counts + align256((size_t)kNoAllocMaxCells * 4u);
  L.chunks = L.cursor + align256((size_t)kNoAllocMaxCells * 4u);
  L.U = L.chunks + align256(((size_t)kNoAllocMaxPoints / kQueryChunk + kNoAllocMaxCells + 2u) * 8u);
  L.S = L.U + align256((size_t)kNoAllocMaxPoints * sizeof(RayRec));
  L.bytes = L.S + align256((size_t)kNoAllocMaxPoints * sizeof(RayRec));
  return L;
}

constexpr size_t kScratchBytes = noalloc_layout().bytes;   // about 12.2 MB
static_assert(kScratchBytes < ((size_t)16 << 20), "scratch stays modest");

std::mutex& scratch_mutex(int device) {
  static std::mutex mus[64];
  return mus[(unsigned)device % 64u];
}
}  // namespace

static __device__ __align__(256) uint8_t kn_scratch[kScratchBytes];

struct kn_ctx {
  int device = 0;
  uint8_t* scratch = nullptr;  // this device's address of kn_scratch
  hipError_t scratch_err = hipSuccess;
  int num_cu = 256;
  hipStream_t stream = nullptr;
  hipStream_t stream2 = nullptr;   // early shading of primary frames
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  uint64_t budget = 0;
  std::atomic<uint64_t> used{0};
  std::mutex mu;              // scenes map, scene reference counts
  std::mutex render_mu;       // one render / query at a time on the workspace
  std::mutex serve_mu;        // serving loop start / stop
  std::map<kn_scene_id, KnScene*> scenes;
  kn_scene_id next_id = 1;
  std::map<kn_world_id, KnWorld*> worlds;   // under mu
  kn_world_id next_world = 1;
  std::atomic<bool> poisoned{false};
  Pool ws;                     // the workspace of kn_render and kn_query
  void* aux = nullptr;         // grow-only work buffer of kn_eikonal_fd
  size_t aux_bytes = 0;
  uint32_t* pinned = nullptr;  // round counters read back by the host
  // host-mapped ring of primary rounds' chunk counts, written by the scan
  // (tag << 32 | count at slot tag % kRoundRing); tags are frame_seq << 11 | round
  unsigned long long* ring = nullptr;
  unsigned long long* ring_dev = nullptr;
  uint32_t frame_seq = 0;
  SceneEnt* h_scene = nullptr; // pinned staging of kn_render's tables ([kMaxScenes])
  ReqEnt* h_req = nullptr;
  hipEvent_t ev_start = nullptr, ev_end = nullptr;
  hipEvent_t ev_round[4] = {nullptr, nullptr, nullptr, nullptr};
  // in-cell passes of a march work item per round (the rest go on in the
  // next round, in the same cell, with the same arithmetic); 1080p C3 BF16
  // frames: caps 2 / 3 / 4 gave 370.6 / 370.3 / 368.4 M rays/s
  int max_passes = 2;
  std::vector<hipEvent_t> ev_kernel;  // pairs around timed kernel launches
  std::shared_ptr<kn::ServeLoop> serve;
};

namespace {

#define KN_HIP(ctx, call)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      (ctx)->poisoned = true;                                                             \
      return fail(KN_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));            \
    }                                                                                     \
  } while (0)

kn_status check_ctx(kn_ctx* ctx) {
  if (!ctx) return fail(KN_E_INVALID, "ctx is NULL");
  if (ctx->poisoned) return fail(KN_E_DEVICE, "context poisoned by an earlier device error");
  return KN_OK;
}

// The cell scan's look-back wait is bounded; running out of it leaves a tile
// with a zero prefix (overlapping bins), so every path that ran a scan reads
// the flag back and treats it as a device error.
kn_status check_scan(kn_ctx* ctx, uint32_t scan_err) {
  if (!scan_err) return KN_OK;
  ctx->poisoned = true;
  return fail(KN_E_DEVICE, "cell scan: a look-back wait ran out; results of this call are invalid");
}

// words of kn_ctx::pinned that receive Ctrl::scan_err at the end of a call
// (render and query; the allocation-free query)
constexpr int kPinnedScanErr = 16;
constexpr int kPinnedScanErrNoAlloc = 17;
constexpr int kPinnedScanErr2 = 18;

// Early shading of primary frames: once a round's work items fall below
// this fraction of the largest round's, the hits so far are shaded on a
// second stream beside the remaining rounds (frames of at least
// kEarlyShadeMinRays rays whose rounds reached kEarlyShadeMinChunks items).
// KN_EARLY_SHADE overrides the fraction (0 turns it off).
constexpr size_t kEarlyShadeMinRays = (size_t)1 << 18;
constexpr uint32_t kEarlyShadeMinChunks = 512;
double early_shade_fraction() {
  if (const char* e = std::getenv("KN_EARLY_SHADE")) return std::atof(e);
  // 1080p C3 BF16 frames, two in-cell passes per round: 0.3 / 0.35 / 0.4 /
  // 0.45 gave 375.6 / 373.9 / 367.8 / 362.5 M rays/s (5.47 / 5.50 / 5.64 /
  // 5.68 ms p50)
  return 0.3;
}

void free_pool(Pool& w) {
  void* ptrs[] = {w.rs, w.U, w.S, w.Uin, w.HL, w.path, w.J, w.W, w.WS, w.hit_count2, w.cursor2, w.ctrl2,
                  w.counts, w.runs, w.hit_count, w.cursor, w.base, w.chunk, w.chunk_out, w.ctrl, w.scenes,
                  w.reqs};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  w = Pool{};
}

constexpr size_t kRayBytes = sizeof(RayStatic) + 4 * sizeof(RayRec);

size_t uin_entries(size_t R) { return R + R / 8 + kListSlack; }

// Per-cell counters are targets of atomics from many workgroups at once
// (arrivals, bin cursors, runs, hits).  Counters of neighbouring cells share
// a cache line when packed, and on a view that enters the grid through a
// face of consecutive cells their atomics queue at the same line; one line
// per counter removes that.  Large pools stay packed: the scan reads every
// counter each round.
// The environment variable KN_COUNTER_STRIDE (1 or 32) overrides the choice
// for pools created afterwards; tests use it to compare the two layouts.
constexpr size_t kPadCells = 65536;
uint32_t counter_stride(size_t C) {
  if (const char* e = std::getenv("KN_COUNTER_STRIDE")) {
    if (std::strcmp(e, "1") == 0) return 1u;
    if (std::strcmp(e, "32") == 0) return 32u;
  }
  return C <= kPadCells ? 32u : 1u;
}

size_t pool_bytes(size_t R, size_t C, size_t K) {
  return R * kRayBytes + (uin_entries(R) - R) * sizeof(RayRec) + C * 4 * (6 * (size_t)counter_stride(C) + 1) +
         K * (4 * 8 + 2 * 64) +
         sizeof(Ctrl) + kMaxScenes * sizeof(SceneEnt) + kMaxSlots * sizeof(ReqEnt);
}

// grow-only pool for `rays` records over `cells` cells (with path state if
// `paths`)
kn_status ensure_pool(kn_ctx* ctx, Pool& w, size_t rays, size_t cells, bool paths = false,
                      bool jumps = false, bool world = false, bool early = false) {
  const size_t chunks = rays / kShadeChunk + cells + 2;
  if (w.ctrl && w.cap >= rays && w.cells >= cells && w.chunks >= chunks && (!paths || w.path) &&
      (!jumps || w.J) && (!world || w.W) && (!early || w.ctrl2))
    return KN_OK;
  const size_t R = std::max(w.cap, rays), C = std::max(w.cells, cells), K = std::max(w.chunks, chunks);
  const bool P = paths || w.path || world, J = jumps || w.J, Wd = world || w.W, E = early || w.ctrl2;
  const size_t cs = counter_stride(C);
  const size_t bytes = pool_bytes(R, C, K) + (P ? R * sizeof(PathRec) : 0) + (J ? 2 * R * sizeof(RayRec) : 0) +
                       (Wd ? R * (2 * sizeof(WorldRec) + sizeof(WState)) : 0) +
                       (E ? 2 * C * cs * 4 + sizeof(Ctrl) : 0);
  const uint64_t other = ctx->used.load() - w.bytes;
  if (other + bytes > ctx->budget)
    return fail(KN_E_NOMEM, "ray workspace of %zu bytes exceeds the HBM budget", bytes);
  if (w.ctrl) KN_HIP(ctx, hipDeviceSynchronize());
  ctx->used -= w.bytes;
  free_pool(w);
  Pool n;
  n.cap = R;
  n.cells = C;
  n.chunks = K;
  n.bytes = bytes;
  n.cs = counter_stride(C);
  KN_HIP(ctx, hipMalloc(&n.rs, R * sizeof(RayStatic)));
  KN_HIP(ctx, hipMalloc(&n.U, R * sizeof(RayRec)));
  KN_HIP(ctx, hipMalloc(&n.S, R * sizeof(RayRec)));
  // Uin also takes path-tracing spawns in per-wave blocks: a block is
  // re-reserved only when a half-tile's <= 4 spawns do not fit (<= 3 of 64
  // entries lost), plus one partial block per wave at the end of a pass
  KN_HIP(ctx, hipMalloc(&n.Uin, uin_entries(R) * sizeof(RayRec)));
  KN_HIP(ctx, hipMalloc(&n.HL, R * sizeof(RayRec)));
  if (P) KN_HIP(ctx, hipMalloc(&n.path, R * sizeof(PathRec)));
  if (J) KN_HIP(ctx, hipMalloc(&n.J, 2 * R * sizeof(RayRec)));
  if (Wd) {
    KN_HIP(ctx, hipMalloc(&n.W, 2 * R * sizeof(WorldRec)));
    KN_HIP(ctx, hipMalloc(&n.WS, R * sizeof(WState)));
  }
  if (E) {
    KN_HIP(ctx, hipMalloc(&n.hit_count2, C * n.cs * 4));
    KN_HIP(ctx, hipMalloc(&n.cursor2, C * n.cs * 4));
    KN_HIP(ctx, hipMalloc(&n.ctrl2, sizeof(Ctrl)));
  }
  KN_HIP(ctx, hipMalloc(&n.counts, 2 * C * n.cs * 4));
  KN_HIP(ctx, hipMalloc(&n.runs, 2 * C * n.cs * 4));
  KN_HIP(ctx, hipMalloc(&n.hit_count, C * n.cs * 4));
  KN_HIP(ctx, hipMalloc(&n.cursor, C * n.cs * 4));
  KN_HIP(ctx, hipMalloc(&n.base, C * 4));
  KN_HIP(ctx, hipMalloc(&n.chunk, 4 * K * 8));
  KN_HIP(ctx, hipMalloc(&n.chunk_out, 2 * K * 64));
  KN_HIP(ctx, hipMalloc(&n.ctrl, sizeof(Ctrl)));
  KN_HIP(ctx, hipMemset(n.HL, 0xFF, R * sizeof(RayRec)));   // no hits
  KN_HIP(ctx, hipMalloc(&n.scenes, kMaxScenes * sizeof(SceneEnt)));
  KN_HIP(ctx, hipMalloc(&n.reqs, kMaxSlots * sizeof(ReqEnt)));
  w = n;
  ctx->used += bytes;
  return KN_OK;
}

// grow-only device buffer of at least `bytes` (kn_eikonal_fd's stencil)
kn_status ensure_aux(kn_ctx* ctx, size_t bytes) {
  if (ctx->aux_bytes >= bytes) return KN_OK;
  const uint64_t other = ctx->used.load() - ctx->aux_bytes;
  if (other + bytes > ctx->budget)
    return fail(KN_E_NOMEM, "work buffer of %zu bytes exceeds the HBM budget", bytes);
  if (ctx->aux) {
    KN_HIP(ctx, hipDeviceSynchronize());
    (void)hipFree(ctx->aux);
    ctx->used -= ctx->aux_bytes;
    ctx->aux = nullptr;
    ctx->aux_bytes = 0;
  }
  KN_HIP(ctx, hipMalloc(&ctx->aux, bytes));
  ctx->aux_bytes = bytes;
  ctx->used += bytes;
  return KN_OK;
}

SoftplusK softplus_consts(float beta) {
  return SoftplusK{(float)(-(double)beta / std::log(2.0)), (float)(std::log(2.0) / (double)beta)};
}

// at most 4096 workgroups: the spawn list holds kListSlack entries for
// partly used blocks (kSpawnBlock per wave of a shading pass)
uint32_t persistent_grid(kn_ctx* ctx, uint32_t per_cu) {
  static_assert((size_t)4096 * 4 * kSpawnBlock <= kListSlack, "list slack too small for the largest grid");
  return std::min<uint32_t>((uint32_t)ctx->num_cu * per_cu, 4096u);
}

PoolTabs pool_tabs(const Pool& w, uint32_t n_scenes) {
  return PoolTabs{w.scenes, w.reqs, n_scenes, &w.ctrl->miss_done[0], &w.ctrl->hit_done[0], w.path};
}

// prec: the march precision; split: refinement and shading of a bf16 or fp8
// march on the split-bfloat16 block (else the float32 block)
SceneEnt scene_entry(const KnScene* s, int prec, uint32_t cell_base, bool split) {
  const int shade_prec = split ? prec : KN_FP32;
  SceneEnt e{};
  e.sg = s->geom;
  e.sg.cell_base = cell_base;
  e.cell_end = cell_base + (uint32_t)(s->N * s->N * s->N);
  e.march = s->march(prec);
  e.march_words = s->march_words(prec);
  e.shade = s->shading(shade_prec);
  e.shade_words = s->shading_words(shade_prec);
  e.spk = softplus_consts(s->geom.beta);
  e.wt[0] = e.wt[1] = e.wt[2] = 0.0f;
  e.ws = 1.0f;
  return e;
}

OutPtrs out_ptrs(const kn_frame* fr) {
  return OutPtrs{fr->rgb, fr->depth, fr->normal, fr->hit, fr->steps,
                 reinterpret_cast<TraceRec*>(fr->trace), reinterpret_cast<SegRec*>(fr->segments),
                 {0.0f, 0.0f, 0.0f}};
}

// What the kernels of one pool round need to know about its tables.
struct RoundCfg {
  int hmode;              // 32 or 64 when every scene has that width, else 0
  int prec;               // march precision (kn_precision)
  uint32_t n_scenes;
  uint32_t march_words;   // largest march block of the scenes
  uint32_t shade_words;   // largest shading block
  bool split;             // bf16 / fp8 pools: split-bfloat16 shading (else float32)
  bool jumps;             // unclamped steps: rays that jump cells go through Pool::J
  uint32_t cells;         // global cells in use
  int max_passes;
  int wpar = -1;          // world renders: the world list (parity) that rays leaving a box
                          // go to this round; -1 otherwise
  bool wzero = false;     // ... and this round's scan clears that list's count first
  unsigned long long* ring = nullptr;   // device address of kn_ctx::ring, or null
  uint32_t tag0 = 0;      // round r's count goes to the ring with tag tag0 + r
  uint32_t* hit_count = nullptr;    // per-cell hit counts the march adds to (null: Pool::hit_count)
};

// Round r: bins the records arriving for it (the previous round's leavers,
// still in U, and n_new new records in Uin, or *n_new_dev of them) by cell,
// then marches them.  Hits go to HL[ray id].
kn_status enqueue_round(kn_ctx* ctx, Pool& w, const RoundCfg& c, int r, uint32_t n_new, hipStream_t st,
                        hipEvent_t e0, hipEvent_t e1, const uint32_t* n_new_dev = nullptr) {
  const int par = r & 1;
  const PoolTabs tabs = pool_tabs(w, c.n_scenes);
  ScanArgs sa{};
  sa.counts = w.counts + par * w.cells * w.cs;
  sa.runs = w.runs + par * w.cells * w.cs;
  sa.cs = w.cs;
  sa.base = w.base;
  sa.C = c.cells;
  sa.T = kChunk;
  sa.zero_counts = 1;
  sa.cursor = w.cursor;
  sa.chunks = w.chunk + (size_t)par * w.chunks;
  sa.n_chunks = &w.ctrl->n_chunks[par];
  sa.grab = w.ctrl->grab;
  sa.grab0 = w.ctrl->grab0;
  sa.ticket = &w.ctrl->scan_ticket;
  sa.flags = w.ctrl->scan_flags;
  sa.err = &w.ctrl->scan_err;
  // the march of this round appends the rays that jump cells to J[par ^ 1]
  sa.zero_word = c.jumps ? &w.ctrl->n_jump[par ^ 1] : nullptr;
  sa.zero_word2 = c.wpar >= 0 && c.wzero ? &w.ctrl->n_w[c.wpar] : nullptr;
  sa.total = nullptr;
  sa.host_ring = c.ring;
  sa.ring_tag = c.tag0 + (uint32_t)r;
  KN_HIP(ctx, launch_scan(sa, st));
  if (r > 0) {
    ScatterChunksArgs sc{tabs,
                         w.chunk + (size_t)(par ^ 1) * w.chunks,
                         w.chunk_out + (size_t)(par ^ 1) * w.chunks * 4,
                         &w.ctrl->n_chunks[par ^ 1],
                         w.U,
                         w.S,
                         w.base};
    KN_HIP(ctx, launch_scatter_chunks(sc, persistent_grid(ctx, 16), st));
  }
  if (n_new) {
    ScatterArgs sc{w.Uin, w.S, n_new, nullptr, w.cursor, 0, w.cs};
    KN_HIP(ctx, launch_scatter(sc, std::min<uint32_t>((n_new + 255u) / 256u, 65536u), st));
  }
  if (n_new_dev) {
    ScatterArgs sc{w.Uin, w.S, 0u, n_new_dev, w.cursor, 0, w.cs};
    KN_HIP(ctx, launch_scatter(sc, persistent_grid(ctx, 4), st));
  }
  if (c.jumps && r > 0) {
    ScatterArgs sc{w.J + (size_t)par * w.cap, w.S, 0u, &w.ctrl->n_jump[par], w.cursor, 0, w.cs};
    KN_HIP(ctx, launch_scatter(sc, persistent_grid(ctx, 4), st));
  }
  MarchArgs ma{};
  ma.tabs = tabs;
  ma.S = w.S;
  ma.rs = w.rs;
  ma.chunks = w.chunk + (size_t)par * w.chunks;
  ma.n_chunks = &w.ctrl->n_chunks[par];
  ma.grab = w.ctrl->grab;
  ma.chunk_out = w.chunk_out + (size_t)par * w.chunks * 4;
  ma.U = w.U;
  ma.runs_next = w.runs + (par ^ 1) * w.cells * w.cs;
  ma.hits = w.HL;
  ma.hit_count = c.hit_count ? c.hit_count : w.hit_count;
  ma.cs = w.cs;
  ma.evals = &w.ctrl->tally[0][0];
  ma.max_passes = c.max_passes;
  if (c.jumps) {
    ma.jump = w.J + (size_t)(par ^ 1) * w.cap;
    ma.n_jump = &w.ctrl->n_jump[par ^ 1];
    ma.counts_next = w.counts + (par ^ 1) * w.cells * w.cs;
  }
  if (c.wpar >= 0) {
    ma.wlist = w.W + (size_t)c.wpar * w.cap;
    ma.n_w = &w.ctrl->n_w[c.wpar];
    ma.ws = w.WS;
  }
  if (e0) KN_HIP(ctx, hipEventRecord(e0, st));
  // the grid is what the CUs hold at once: bf16 and fp8 march kernels 3
  // workgroups per CU (3 waves per SIMD, about 33 KB of LDS each), the
  // float32 one 2 (about 220 VGPRs).  A larger grid only adds workgroups
  // that start as others exit, find the work taken and exit (bf16 march
  // 3.44 -> 3.38 ms, fp32 9.02 -> 8.97 ms per 1080p frame).
  const uint32_t march_per_cu = c.prec == KN_FP32 ? 2u : 3u;
  KN_HIP(ctx, launch_march(ma, c.hmode, c.prec, c.march_words, persistent_grid(ctx, march_per_cu), st));
  if (e1) KN_HIP(ctx, hipEventRecord(e1, st));
  return KN_OK;
}

// Shading pass over the hits of ray ids [0, n_ids): binned by cell (the
// scatter clears each hit it takes), refined, shaded.  With path tracing,
// hits that scatter append their next segment to Uin (count in ctrl->n_in,
// cleared first) for round `next_round`.
// The buffers one shading pass works in: the hit list and per-cell hit
// counts it takes, and its own bins, cursors, work items and control block.
struct ShadeSet {
  RayRec* hits;
  uint32_t* hit_count;
  RayRec* S;
  uint32_t* cursor;
  uint2* chunks;
  Ctrl* ctrl;
};

ShadeSet main_shade_set(const Pool& w) {
  return ShadeSet{w.HL, w.hit_count, w.S, w.cursor, w.chunk + 2 * w.chunks, w.ctrl};
}

// With kst, the binning (scan and scatter, which takes the hits out of the
// list) stays on st and the shading kernel runs on kst after it (ev_fork),
// with per_cu workgroups per CU; ev_join marks its end on kst.
kn_status enqueue_shade(kn_ctx* ctx, Pool& w, const RoundCfg& c, uint32_t n_ids, hipStream_t st, hipEvent_t e0,
                        hipEvent_t e1, bool pt = false, int next_round = 0, const ShadeSet* set = nullptr,
                        hipStream_t kst = nullptr, uint32_t per_cu = 3) {
  const ShadeSet ss = set ? *set : main_shade_set(w);
  uint2* chunks = ss.chunks;
  ScanArgs sa{};
  sa.counts = ss.hit_count;
  sa.cs = w.cs;
  sa.C = c.cells;
  sa.T = kShadeChunk;
  sa.zero_counts = 1;
  sa.cursor = ss.cursor;
  sa.chunks = chunks;
  sa.n_chunks = &ss.ctrl->n_chunks[2];
  sa.grab = ss.ctrl->grab;
  sa.grab0 = ss.ctrl->grab0;
  sa.ticket = &ss.ctrl->scan_ticket;
  sa.flags = ss.ctrl->scan_flags;
  sa.err = &ss.ctrl->scan_err;
  sa.zero_word = pt ? &w.ctrl->n_in : nullptr;
  sa.total = &ss.ctrl->n_hits;
  KN_HIP(ctx, launch_scan(sa, st));
  ScatterArgs sc{ss.hits, ss.S, n_ids, nullptr, ss.cursor, 1, w.cs};
  KN_HIP(ctx, launch_scatter(sc, std::min<uint32_t>((n_ids + 255u) / 256u, 65536u), st));
  ShadeArgs sh{};
  sh.tabs = pool_tabs(w, c.n_scenes);
  sh.S = ss.S;
  sh.rs = w.rs;
  sh.chunks = chunks;
  sh.n_chunks = &ss.ctrl->n_chunks[2];
  sh.grab = ss.ctrl->grab;
  sh.spawn = w.Uin;
  sh.n_spawn = &w.ctrl->n_in;
  sh.counts_next = w.counts + (next_round & 1) * w.cells * w.cs;
  sh.cs = w.cs;
  if (c.wpar >= 0) {
    sh.wlist = w.W + (size_t)c.wpar * w.cap;
    sh.n_w = &w.ctrl->n_w[c.wpar];
  }
  if (kst) {
    KN_HIP(ctx, hipEventRecord(ctx->ev_fork, st));
    KN_HIP(ctx, hipStreamWaitEvent(kst, ctx->ev_fork, 0));
  }
  hipStream_t ks = kst ? kst : st;
  if (e0) KN_HIP(ctx, hipEventRecord(e0, ks));
  KN_HIP(ctx, launch_shade(sh, c.hmode, c.split ? c.prec : (int)KN_FP32, pt, c.shade_words,
                           persistent_grid(ctx, per_cu), ks));
  if (e1) KN_HIP(ctx, hipEventRecord(e1, ks));
  if (kst) KN_HIP(ctx, hipEventRecord(ctx->ev_join, kst));
  return KN_OK;
}

}  // namespace

extern "C" {

const char* kn_last_error(void) { return g_err.c_str(); }

kn_status kn_ctx_create(int hip_device, uint64_t hbm_budget_bytes, kn_ctx** out) {
  if (!out) return fail(KN_E_INVALID, "out is NULL");
  *out = nullptr;
  const std::vector<std::string> rts = hip_runtimes_loaded();
  if (rts.size() > 1)
    return fail(KN_E_DEVICE,
                "%zu HIP runtimes are loaded in this process (%s and %s): device pointers and streams of "
                "one are invalid in the other; load the runtime that allocates the frame buffers (for "
                "example import torch) before this library",
                rts.size(), rts[0].c_str(), rts[1].c_str());
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(KN_E_DEVICE, "no HIP device");
  if (hip_device < 0 || hip_device >= n) return fail(KN_E_INVALID, "device %d out of range", hip_device);
  std::unique_ptr<kn_ctx> ctx(new kn_ctx());
  ctx->device = hip_device;
  KN_HIP(ctx, hipSetDevice(hip_device));
  // this device's copy of the allocation-free query's scratch array (the
  // array's name is a host-side stand-in, not a device address).  Without
  // it only kn_query_noalloc fails, with the code kept here.
  ctx->scratch_err = hipGetSymbolAddress(reinterpret_cast<void**>(&ctx->scratch), HIP_SYMBOL(kn_scratch));
  if (ctx->scratch_err != hipSuccess) {
    ctx->scratch = nullptr;
    (void)hipGetLastError();
  }
  hipDeviceProp_t prop;
  KN_HIP(ctx, hipGetDeviceProperties(&prop, hip_device));
  ctx->num_cu = prop.multiProcessorCount;
  size_t freeb = 0, total = 0;
  KN_HIP(ctx, hipMemGetInfo(&freeb, &total));
  ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)freeb);
  KN_HIP(ctx, hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
  KN_HIP(ctx, hipStreamCreateWithFlags(&ctx->stream2, hipStreamNonBlocking));
  KN_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
  KN_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
  KN_HIP(ctx, hipHostMalloc((void**)&ctx->pinned, 64 * sizeof(uint32_t), hipHostMallocDefault));
  KN_HIP(ctx, hipHostMalloc((void**)&ctx->ring, kRoundRing * sizeof(unsigned long long),
                            hipHostMallocCoherent | hipHostMallocMapped));
  for (uint32_t i = 0; i < kRoundRing; ++i) ctx->ring[i] = ~0ull;
  KN_HIP(ctx, hipHostGetDevicePointer((void**)&ctx->ring_dev, ctx->ring, 0));
  KN_HIP(ctx, hipHostMalloc((void**)&ctx->h_scene, kMaxScenes * sizeof(SceneEnt), hipHostMallocDefault));
  KN_HIP(ctx, hipHostMalloc((void**)&ctx->h_req, sizeof(ReqEnt), hipHostMallocDefault));
  KN_HIP(ctx, hipEventCreate(&ctx->ev_start));
  KN_HIP(ctx, hipEventCreate(&ctx->ev_end));
  for (auto& e : ctx->ev_round) KN_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  *out = ctx.release();
  return KN_OK;
}

kn_status kn_ctx_destroy(kn_ctx* ctx) {
  if (!ctx) return fail(KN_E_INVALID, "ctx is NULL");
  if (ctx->serve) kn_serve_stop(ctx);
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->worlds) {
    if (kv.second->prims) (void)hipFree(kv.second->prims);
    delete kv.second;
  }
  for (auto& kv : ctx->scenes) {
    KnScene* s = kv.second;
    if (s->march_f32) (void)hipFree(s->march_f32);
    if (s->march_bf16) (void)hipFree(s->march_bf16);
    if (s->march_fp8) (void)hipFree(s->march_fp8);
    if (s->shade) (void)hipFree(s->shade);
    if (s->shade3) (void)hipFree(s->shade3);
    delete s;
  }
  free_pool(ctx->ws);
  if (ctx->aux) (void)hipFree(ctx->aux);
  ctx->used -= ctx->aux_bytes;
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->ring) (void)hipHostFree(ctx->ring);
  if (ctx->h_scene) (void)hipHostFree(ctx->h_scene);
  if (ctx->h_req) (void)hipHostFree(ctx->h_req);
  if (ctx->ev_start) (void)hipEventDestroy(ctx->ev_start);
  if (ctx->ev_end) (void)hipEventDestroy(ctx->ev_end);
  for (auto& e : ctx->ev_round)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->ev_kernel) (void)hipEventDestroy(e);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->stream2) {
    (void)hipStreamSynchronize(ctx->stream2);
    (void)hipStreamDestroy(ctx->stream2);
  }
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return KN_OK;
}

kn_status kn_scene_create(kn_ctx* ctx, const kn_scene_desc* d, kn_scene_id* out) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  if (!d || !out) return fail(KN_E_INVALID, "desc or out is NULL");
  if (d->abi_version != KN_ABI_VERSION)
    return fail(KN_E_INVALID, "abi_version %u, library is %u", d->abi_version, KN_ABI_VERSION);
  if (!d->sdf_params || !d->col_params) return fail(KN_E_INVALID, "parameter arrays are NULL");
  if (d->grid_n < 1 || d->grid_n > 64) return fail(KN_E_UNSUPPORTED, "grid_n %u not in 1..64", d->grid_n);
  for (int k = 0; k < 3; ++k)
    if (!(d->bbox_max[k] > d->bbox_min[k]) || !std::isfinite(d->bbox_min[k]) || !std::isfinite(d->bbox_max[k]))
      return fail(KN_E_INVALID, "empty or non-finite bounding box on axis %d", k);
  if (d->pos_freqs != 6 || d->dir_freqs != 4)
    return fail(KN_E_UNSUPPORTED, "encoding frequencies (%u, %u), only (6, 4)", d->pos_freqs, d->dir_freqs);
  if (d->sdf_hidden != 32 && d->sdf_hidden != 64)
    return fail(KN_E_UNSUPPORTED, "sdf_hidden %u, only 32 or 64", d->sdf_hidden);
  if (d->sdf_layers != 2 || d->feat_dim != 15 || d->col_hidden != 32 || d->col_layers != 1 ||
      d->col_in_has_x != 1)
    return fail(KN_E_UNSUPPORTED, "MLP shape not supported (2 SDF layers, 15 features, 1x32 color)");
  if (!(d->softplus_beta > 0.0f) || !std::isfinite(d->softplus_beta))
    return fail(KN_E_INVALID, "softplus_beta must be positive and finite");
  if (d->precisions & ~((1u << KN_BF16) | (1u << KN_FP8_E4M3)))
    return fail(KN_E_INVALID, "unknown precision bits 0x%x", d->precisions);

  const int N = (int)d->grid_n, H = (int)d->sdf_hidden;
  const size_t cells = (size_t)N * N * N;
  const size_t psdf = (size_t)kSdfIn * H + H + H * H + H + 16 * H + 16;
  const size_t pcol = (size_t)kColIn * kColHid + kColHid + 3 * kColHid + 3;
  for (size_t i = 0; i < cells * psdf; ++i)
    if (!std::isfinite(d->sdf_params[i])) return fail(KN_E_INVALID, "non-finite SDF parameter at %zu", i);
  for (size_t i = 0; i < cells * pcol; ++i)
    if (!std::isfinite(d->col_params[i])) return fail(KN_E_INVALID, "non-finite color parameter at %zu", i);

  std::unique_ptr<KnScene> s(new KnScene());
  s->N = N;
  s->H = H;
  SceneGeom& g = s->geom;
  g.N = N;
  g.H = H;
  g.cell_base = 0;
  g.beta = d->softplus_beta;
  for (int k = 0; k < 3; ++k) {
    g.bmin[k] = d->bbox_min[k];
    g.bmax[k] = d->bbox_max[k];
    const double side = ((double)d->bbox_max[k] - (double)d->bbox_min[k]) / N;
    g.side[k] = (float)side;
    g.inv_side[k] = (float)(1.0 / side);
    g.half[k] = (float)(0.5 * side);
    g.inv_half[k] = (float)(2.0 / side);
  }
  s->march_f32_words = (uint32_t)march_block_words(H, kPrecF32);
  s->march_bf16_words = (uint32_t)march_block_words(H, kPrecBf16);
  s->march_fp8_words = (uint32_t)march_block_words(H, kPrecFp8);
  s->shade_words = (uint32_t)shade_block_words(H);
  s->shade3_words = (uint32_t)shade3_block_words(H);
  const bool want_bf16 = (d->precisions >> KN_BF16) & 1u;
  const bool want_fp8 = (d->precisions >> KN_FP8_E4M3) & 1u;
  const size_t bytes = cells * 4 * ((size_t)s->march_f32_words + s->shade_words +
                                    (want_bf16 ? s->march_bf16_words : 0) +
                                    (want_fp8 ? s->march_fp8_words : 0) +
                                    (want_bf16 || want_fp8 ? s->shade3_words : 0));
  if (ctx->used.load() + bytes > ctx->budget)
    return fail(KN_E_NOMEM, "scene needs %zu bytes; budget %llu, in use %llu", bytes,
                (unsigned long long)ctx->budget, (unsigned long long)ctx->used.load());

  std::vector<float> host;
  auto upload = [&](float** dst, uint32_t words, auto packer) -> kn_status {
    host.assign(cells * (size_t)words, 0.0f);
    for (size_t c = 0; c < cells; ++c) packer(c, host.data() + c * words);
    KN_HIP(ctx, hipMalloc(dst, host.size() * 4));
    KN_HIP(ctx, hipMemcpy(*dst, host.data(), host.size() * 4, hipMemcpyHostToDevice));
    return KN_OK;
  };
  KN_HIP(ctx, hipSetDevice(ctx->device));
  st = upload(&s->march_f32, s->march_f32_words,
              [&](size_t c, float* o) { pack_march_f32(d->sdf_params + c * psdf, H, o); });
  if (st != KN_OK) return st;
  if (want_bf16) {
    const float beta = d->softplus_beta;
    st = upload(&s->march_bf16, s->march_bf16_words,
                [&](size_t c, float* o) { pack_march_bf16(d->sdf_params + c * psdf, H, beta, o); });
    if (st != KN_OK) return st;
  }
  if (want_fp8) {
    const float beta = d->softplus_beta;
    st = upload(&s->march_fp8, s->march_fp8_words,
                [&](size_t c, float* o) { pack_march_fp8(d->sdf_params + c * psdf, H, beta, o); });
    if (st != KN_OK) return st;
  }
  st = upload(&s->shade, s->shade_words, [&](size_t c, float* o) {
    pack_shade(d->sdf_params + c * psdf, d->col_params + c * pcol, H, o);
  });
  if (st != KN_OK) return st;
  if (want_bf16 || want_fp8) {
    st = upload(&s->shade3, s->shade3_words, [&](size_t c, float* o) {
      pack_shade3(d->sdf_params + c * psdf, d->col_params + c * pcol, H, o);
    });
    if (st != KN_OK) return st;
  }
  s->bytes = bytes;
  ctx->used += bytes;
  std::lock_guard<std::mutex> lk(ctx->mu);
  KnScene* sp = s.release();
  sp->id = ctx->next_id++;
  ctx->scenes[sp->id] = sp;
  *out = sp->id;
  return KN_OK;
}

kn_status kn_scene_destroy(kn_ctx* ctx, kn_scene_id id) {
  if (!ctx) return fail(KN_E_INVALID, "ctx is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->scenes.find(id);
  if (it == ctx->scenes.end()) return fail(KN_E_NOT_FOUND, "scene %u not found", id);
  KnScene* s = it->second;
  if (s->refs.load() > 0) return fail(KN_E_BUSY, "scene %u has requests in flight", id);
  if (s->world_refs > 0) return fail(KN_E_BUSY, "scene %u is placed in %d world(s)", id, s->world_refs);
  std::lock_guard<std::mutex> rk(ctx->render_mu);
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (s->march_f32) (void)hipFree(s->march_f32);
  if (s->march_bf16) (void)hipFree(s->march_bf16);
  if (s->march_fp8) (void)hipFree(s->march_fp8);
  if (s->shade) (void)hipFree(s->shade);
  if (s->shade3) (void)hipFree(s->shade3);
  ctx->used -= s->bytes;
  delete s;
  ctx->scenes.erase(it);
  return KN_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// rendering
// ---------------------------------------------------------------------------
namespace {

KnScene* find_scene(kn_ctx* ctx, kn_scene_id id) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->scenes.find(id);
  return it == ctx->scenes.end() ? nullptr : it->second;
}

constexpr int kMaxBounces = 16;
constexpr int kMaxSpp = 64;

kn_status validate_camera(const kn_camera* c, const KnScene* s) {
  if (!c) return fail(KN_E_INVALID, "camera is NULL");
  if (c->width == 0 || c->height == 0) return fail(KN_E_INVALID, "empty image %ux%u", c->width, c->height);
  if ((uint64_t)c->width * c->height > (uint64_t)kPixMask + 1u)
    return fail(KN_E_INVALID, "image %ux%u has more than 2^24 pixels", c->width, c->height);
  if (c->max_steps < 1 || c->max_steps > (uint32_t)kMaxSteps)
    return fail(KN_E_INVALID, "max_steps %u not in 1..%d", c->max_steps, kMaxSteps);
  if (!(c->eps > 0.0f) || !std::isfinite(c->eps)) return fail(KN_E_INVALID, "eps must be positive");
  if (c->bounces > kMaxBounces) return fail(KN_E_INVALID, "bounces %u above %d", c->bounces, kMaxBounces);
  if (c->spp < 1 || c->spp > kMaxSpp) return fail(KN_E_INVALID, "spp %u not in 1..%d", c->spp, kMaxSpp);
  if (c->bounces == 0 && (c->spp != 1 || c->env_rgb))
    return fail(KN_E_UNSUPPORTED, "spp > 1 and environment maps need path tracing (bounces >= 1)");
  if ((uint64_t)c->width * c->height * c->spp > ((uint64_t)1 << 30))
    return fail(KN_E_INVALID, "%ux%u x %u spp paths exceed 2^30", c->width, c->height, c->spp);
  if (c->env_rgb && (c->env_w == 0 || c->env_h == 0))
    return fail(KN_E_INVALID, "environment map of size %ux%u", c->env_w, c->env_h);
  if (c->precision != KN_FP32 && c->precision != KN_BF16 && c->precision != KN_FP8_E4M3)
    return fail(KN_E_INVALID, "unknown precision %d", (int)c->precision);
  if (c->flags & ~(uint32_t)(KN_CAMERA_SPLIT_BF16_SHADING | KN_CAMERA_UNCLAMPED_STEPS))
    return fail(KN_E_INVALID, "unknown camera flags 0x%x", c->flags);
  if (c->sample_offset && c->bounces == 0)
    return fail(KN_E_INVALID, "sample_offset needs path tracing (bounces >= 1)");
  if (c->sample_offset > (1u << 30)) return fail(KN_E_INVALID, "sample_offset %u above 2^30", c->sample_offset);
  if (s && !s->march(c->precision))
    return fail(KN_E_INVALID, "scene has no copy in precision %d (set its bit in precisions)",
                (int)c->precision);
  if (c->tan_half_diag < 0.0f || !std::isfinite(c->tan_half_diag))
    return fail(KN_E_INVALID, "tan_half_diag must be >= 0");
  double f[3], dist2 = 0;
  for (int k = 0; k < 3; ++k) {
    f[k] = (double)c->look_at[k] - c->eye[k];
    dist2 += f[k] * f[k];
  }
  if (!(dist2 > 0)) return fail(KN_E_INVALID, "eye equals look_at");
  if (c->tan_half_diag == 0.0f && !(dist2 > 1.0))
    return fail(KN_E_INVALID, "default field of view needs |eye - look_at| > 1");
  const double cr[3] = {f[1] * c->up[2] - f[2] * c->up[1], f[2] * c->up[0] - f[0] * c->up[2],
                        f[0] * c->up[1] - f[1] * c->up[0]};
  if (!(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2] > 1e-12 * dist2))
    return fail(KN_E_INVALID, "up is parallel to the view direction");
  return KN_OK;
}

kn_status validate_frame(const kn_frame* fr, const kn_camera* c) {
  if (!fr || !fr->rgb) return fail(KN_E_INVALID, "frame or frame->rgb is NULL");
  if (fr->accum && c->bounces == 0)
    return fail(KN_E_UNSUPPORTED, "progressive accumulation needs path tracing (bounces >= 1)");
  return KN_OK;
}

// camera basis in double precision, rounded to float for the kernels
void camera_basis(const kn_camera* c, RaygenArgs& a) {
  double f[3], up[3] = {c->up[0], c->up[1], c->up[2]}, dist2 = 0;
  for (int k = 0; k < 3; ++k) {
    f[k] = (double)c->look_at[k] - c->eye[k];
    dist2 += f[k] * f[k];
  }
  const double fl = std::sqrt(dist2);
  for (double& v : f) v /= fl;
  double r[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
  const double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  for (double& v : r) v /= rl;
  const double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
  const double T = c->tan_half_diag > 0.0f ? (double)c->tan_half_diag : 1.0 / std::sqrt(dist2 - 1.0);
  const double W = c->width, Hh = c->height, diag = std::sqrt(W * W + Hh * Hh);
  a.tx = (float)(T * W / diag);
  a.ty = (float)(T * Hh / diag);
  for (int k = 0; k < 3; ++k) {
    a.eye[k] = c->eye[k];
    a.fwd[k] = (float)f[k];
    a.right[k] = (float)r[k];
    a.up[k] = (float)u[k];
  }
}

kn_status validate_query(const KnScene* s, kn_precision precision, const float* points, uint64_t n) {
  if (!points) return fail(KN_E_INVALID, "points is NULL");
  if (n > (1ull << 28)) return fail(KN_E_INVALID, "too many points (%llu)", (unsigned long long)n);
  if (precision != KN_FP32 && precision != KN_BF16 && precision != KN_FP8_E4M3)
    return fail(KN_E_INVALID, "unknown precision %d", (int)precision);
  if (!s->march(precision)) return fail(KN_E_INVALID, "scene has no copy in precision %d", (int)precision);
  return KN_OK;
}

// Device buffers of one point query: records, per-cell counters (cell c at
// c * cs) and cursors, work items and the control block.
struct QueryBufs {
  RayRec* U;
  RayRec* S;
  uint32_t* counts;
  uint32_t* cursor;
  uint2* chunks;
  Ctrl* ctrl;
  uint32_t cs;
};

// Enqueues a point query (Sec. 3.3: the points binned by cell, then each
// cell's MLP on its batch): binning, scan, scatter, then the value kernel
// and/or the full kernel (value, gradient, feature).  kernels_only clears and
// restores counters with kernels instead of memset and memcpy nodes.
kn_status enqueue_query(kn_ctx* ctx, const KnScene* s, kn_precision precision, const float* points, uint64_t n,
                        float* d_out, float* grad_out, float* z_out, hipStream_t stream, const QueryBufs& b,
                        bool kernels_only) {
  const size_t cells = (size_t)s->N * s->N * s->N;
  const SoftplusK spk = softplus_consts(s->geom.beta);
  if (kernels_only) {
    KN_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t*>(b.ctrl), sizeof(Ctrl) / 4, 0u, stream));
    KN_HIP(ctx, launch_fill_u32(b.counts, cells * b.cs, 0u, stream));
  } else {
    KN_HIP(ctx, hipMemsetAsync(b.ctrl, 0, sizeof(Ctrl), stream));
    KN_HIP(ctx, hipMemsetAsync(b.counts, 0, cells * b.cs * 4, stream));
  }
  QueryBinArgs qb{s->geom, points, n, b.U, b.counts, b.cs};
  KN_HIP(ctx, launch_query_bin(qb, stream));
  ScanArgs sa{};
  sa.counts = b.counts;
  sa.cs = b.cs;
  sa.C = (uint32_t)cells;
  sa.T = kQueryChunk;
  sa.zero_counts = 0;
  sa.cursor = b.cursor;
  sa.chunks = b.chunks;
  sa.n_chunks = &b.ctrl->n_chunks[0];
  sa.grab = b.ctrl->grab;
  sa.grab0 = b.ctrl->grab0;
  sa.ticket = &b.ctrl->scan_ticket;
  sa.flags = b.ctrl->scan_flags;
  sa.err = &b.ctrl->scan_err;
  sa.zero_word = nullptr;
  KN_HIP(ctx, launch_scan(sa, stream));
  ScatterArgs sc{b.U, b.S, (uint32_t)n, nullptr, b.cursor, 0, b.cs};
  KN_HIP(ctx, launch_scatter(sc, (uint32_t)std::min<uint64_t>((n + 255) / 256, 65536), stream));
  QueryArgs qa{};
  qa.sg = s->geom;
  qa.S = b.S;
  qa.pts = points;
  qa.chunks = b.chunks;
  qa.n_chunks = &b.ctrl->n_chunks[0];
  qa.grab = b.ctrl->grab;
  qa.spk = spk;
  if (d_out) {
    qa.blocks = s->march(precision);
    qa.block_words = s->march_words(precision);
    qa.d_out = d_out;
    KN_HIP(ctx, launch_query_d(qa, s->H, (int)precision, persistent_grid(ctx, 2), stream));
  }
  if (grad_out || z_out) {
    if (kernels_only)
      KN_HIP(ctx, launch_copy_u32(b.ctrl->grab, b.ctrl->grab0, sizeof(b.ctrl->grab) / 4, stream));
    else
      KN_HIP(ctx, hipMemcpyAsync(b.ctrl->grab, b.ctrl->grab0, sizeof(b.ctrl->grab), hipMemcpyDeviceToDevice,
                                 stream));
    qa.blocks = s->shade;
    qa.block_words = s->shade_words;
    qa.d_out = nullptr;
    qa.grad_out = grad_out;
    qa.z_out = z_out;
    KN_HIP(ctx, launch_query_full(qa, s->H, persistent_grid(ctx, 2), stream));
  }
  return KN_OK;
}

}  // namespace

namespace {

// Waits until the scan of the round tagged `tag` has put its chunk count into
// the host-mapped ring (the count is stored by the scan itself, so no copy
// command sits between the rounds).  A stream that has failed, or finished
// without the entry, is an error.
kn_status wait_round(kn_ctx* ctx, hipStream_t stream, uint32_t tag, uint32_t* n) {
  volatile unsigned long long* slot = ctx->ring + tag % kRoundRing;
  const auto t0 = std::chrono::steady_clock::now();
  for (uint64_t it = 1;; ++it) {
    const unsigned long long v = *slot;
    if ((uint32_t)(v >> 32) == tag) {
      *n = (uint32_t)v;
      return KN_OK;
    }
    if ((it & 255u) == 0) {
      const hipError_t q = hipStreamQuery(stream);
      if (q == hipSuccess) {
        const unsigned long long v2 = *slot;
        if ((uint32_t)(v2 >> 32) == tag) {
          *n = (uint32_t)v2;
          return KN_OK;
        }
        ctx->poisoned = true;
        return fail(KN_E_DEVICE, "round %u: its chunk count never reached the host", tag & 2047u);
      }
      if (q != hipErrorNotReady) {
        ctx->poisoned = true;
        return fail(KN_E_DEVICE, "stream failed while rendering: %s", hipGetErrorString(q));
      }
      if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60)) {
        ctx->poisoned = true;
        return fail(KN_E_DEVICE, "round %u did not finish within 60 s", tag & 2047u);
      }
      std::this_thread::yield();
    }
  }
}

}  // namespace

namespace kn {

// Enqueues and runs one frame on `stream` as a one-request pool; the caller
// holds render_mu.  bounces > 0 path-traces spp paths per pixel.
kn_status render_frame(kn_ctx* ctx, KnScene* s, const kn_camera* c, const kn_frame* fr,
                       hipStream_t stream, kn_stats* stats) {
  const auto wall0 = std::chrono::steady_clock::now();
  const bool pt = c->bounces > 0;
  const uint32_t spp = pt ? c->spp : 1u;
  const size_t npix = (size_t)c->width * c->height;
  const size_t rays = npix * spp;
  const size_t cells = (size_t)s->N * s->N * s->N;
  const bool jumps = (c->flags & KN_CAMERA_UNCLAMPED_STEPS) != 0;
  const double early_frac = early_shade_fraction();

  // (frames timed kernel by kernel run their shading in one pass: their
  // per-launch times are not to be shared with a concurrent kernel)
  const bool early = !pt && rays >= kEarlyShadeMinRays && early_frac > 0.0 && !(stats && stats->kernel_times);
  kn_status st = ensure_pool(ctx, ctx->ws, rays, cells, pt, jumps, false, early);
  if (st != KN_OK) return st;
  Pool& w = ctx->ws;
  const bool split = (c->flags & KN_CAMERA_SPLIT_BF16_SHADING) && c->precision != KN_FP32;
  *ctx->h_scene = scene_entry(s, (int)c->precision, 0u, split);
  ReqEnt q{};
  q.out = out_ptrs(fr);
  if (!pt) q.out.seg = nullptr;   // segment records describe path-traced frames only
  q.eps = c->eps;
  q.max_steps = c->max_steps;
  q.npix = (uint32_t)npix;
  q.pt = pt ? 1u : 0u;
  q.spp = spp;
  q.bounces = c->bounces;
  q.seed_lo = (uint32_t)c->seed;
  q.seed_hi = (uint32_t)(c->seed >> 32);
  q.env = c->env_rgb;
  q.env_w = c->env_w;
  q.env_h = c->env_h;
  q.unclamped = jumps ? 1u : 0u;
  q.sample_offset = pt ? c->sample_offset : 0u;
  *ctx->h_req = q;
  RoundCfg cfg{s->H, (int)c->precision, 1u, ctx->h_scene->march_words, ctx->h_scene->shade_words, split,
               jumps, (uint32_t)cells, ctx->max_passes};
  if (!pt) {   // primary frames follow their rounds through the ring
    cfg.ring = ctx->ring_dev;
    cfg.tag0 = (ctx->frame_seq++ & 0x1FFFFFu) << 11;
  }

  const bool timed = stats && stats->kernel_times;
  std::vector<std::pair<int, int>> march_ev, shade_ev;   // event index pairs
  size_t next_ev = 0;
  auto ev = [&](hipEvent_t* e) -> kn_status {
    if (!timed) {
      *e = nullptr;
      return KN_OK;
    }
    if (next_ev == ctx->ev_kernel.size()) {
      hipEvent_t x;
      KN_HIP(ctx, hipEventCreate(&x));
      ctx->ev_kernel.push_back(x);
    }
    *e = ctx->ev_kernel[next_ev++];
    return KN_OK;
  };
  hipEvent_t e0, e1;

  KN_HIP(ctx, hipEventRecord(ctx->ev_start, stream));
  KN_HIP(ctx, hipMemcpyAsync(w.scenes, ctx->h_scene, sizeof(SceneEnt), hipMemcpyHostToDevice, stream));
  KN_HIP(ctx, hipMemcpyAsync(w.reqs, ctx->h_req, sizeof(ReqEnt), hipMemcpyHostToDevice, stream));
  KN_HIP(ctx, hipMemsetAsync(w.ctrl, 0, sizeof(Ctrl), stream));
  // both parities of the per-cell counts ([2][w.cells]) and the hit counts
  KN_HIP(ctx, hipMemsetAsync(w.counts, 0, 2 * w.cells * w.cs * 4, stream));
  KN_HIP(ctx, hipMemsetAsync(w.runs, 0, 2 * w.cells * w.cs * 4, stream));
  KN_HIP(ctx, hipMemsetAsync(w.hit_count, 0, w.cells * w.cs * 4, stream));
  KN_HIP(ctx, hipMemsetAsync(w.HL, 0xFF, rays * sizeof(RayRec), stream));
  if (early) {
    KN_HIP(ctx, hipMemsetAsync(w.ctrl2, 0, sizeof(Ctrl), stream));
    KN_HIP(ctx, hipMemsetAsync(w.hit_count2, 0, w.cells * w.cs * 4, stream));
  }
  bool forked = false;

  RaygenArgs rg{};
  rg.sg = ctx->h_scene->sg;
  camera_basis(c, rg);
  int rounds = 0;
  if (!pt) {
    rg.W = (int)c->width;
    rg.Hh = (int)c->height;
    rg.slot = 0;
    rg.rid_base = 0;
    rg.rs = w.rs;
    rg.U = w.Uin;
    rg.counts = w.counts;
    rg.cs = w.cs;
    rg.miss_done = &w.ctrl->miss_done[0];
    rg.out = q.out;
    KN_HIP(ctx, launch_raygen(rg, stream));
    // every round takes at least one SDF evaluation of every live ray
    const int max_rounds = (int)c->max_steps + 2;
    uint32_t peak = 0;
    for (int r = 0; r < max_rounds; ++r) {
      if ((st = ev(&e0)) != KN_OK || (st = ev(&e1)) != KN_OK) return st;
      if (timed) march_ev.push_back({(int)next_ev - 2, (int)next_ev - 1});
      st = enqueue_round(ctx, w, cfg, r, r == 0 ? (uint32_t)rays : 0u, stream, e0, e1);
      if (st != KN_OK) return st;
      ++rounds;
      // stop once the round kLag rounds back had no work (the rounds enqueued
      // after it find none and return at once); its count arrives through
      // the host-mapped ring while this round's work is queued behind it
      constexpr int kLag = 2;
      if (r >= kLag) {
        uint32_t n = 0;
        if ((st = wait_round(ctx, stream, cfg.tag0 + (uint32_t)(r - kLag), &n)) != KN_OK) return st;
        if (n == 0) break;
        peak = std::max(peak, n);
        // the rounds have thinned out: the hits so far (rounds 0..r) are
        // taken out of the hit list and binned here, then shaded on the
        // second stream, with two workgroups per CU, beside the remaining
        // rounds (whose hits are counted per cell in hit_count2)
        if (early && !forked && peak >= kEarlyShadeMinChunks && (double)n < early_frac * (double)peak) {
          const ShadeSet first{w.HL, w.hit_count, w.Uin, w.cursor2, w.chunk + 3 * w.chunks, w.ctrl2};
          st = enqueue_shade(ctx, w, cfg, (uint32_t)rays, stream, nullptr, nullptr, false, 0, &first, ctx->stream2,
                             2);
          if (st != KN_OK) return st;
          cfg.hit_count = w.hit_count2;
          forked = true;
        }
      }
    }
    if ((st = ev(&e0)) != KN_OK || (st = ev(&e1)) != KN_OK) return st;
    if (timed) shade_ev.push_back({(int)next_ev - 2, (int)next_ev - 1});
    const ShadeSet last = forked ? ShadeSet{w.HL, w.hit_count2, w.S, w.cursor, w.chunk + 2 * w.chunks, w.ctrl}
                                 : main_shade_set(w);
    st = enqueue_shade(ctx, w, cfg, (uint32_t)rays, stream, e0, e1, false, 0, &last);
    if (st != KN_OK) return st;
    if (forked) KN_HIP(ctx, hipStreamWaitEvent(stream, ctx->ev_join, 0));
  } else {
    RaygenPtArgs rp{};
    rp.sg = rg.sg;
    for (int k = 0; k < 3; ++k) {
      rp.eye[k] = rg.eye[k];
      rp.fwd[k] = rg.fwd[k];
      rp.right[k] = rg.right[k];
      rp.up[k] = rg.up[k];
    }
    rp.tx = rg.tx;
    rp.ty = rg.ty;
    rp.W = (int)c->width;
    rp.Hh = (int)c->height;
    rp.spp = spp;
    rp.bounces = c->bounces;
    rp.seed_lo = q.seed_lo;
    rp.seed_hi = q.seed_hi;
    rp.env = q.env;
    rp.env_w = q.env_w;
    rp.env_h = q.env_h;
    rp.jitter = fr->accum ? 1u : 0u;
    rp.sample_offset = q.sample_offset;
    rp.slot = 0;
    rp.rs = w.rs;
    rp.U = w.Uin;
    rp.path = w.path;
    rp.counts = w.counts;
    rp.cs = w.cs;
    rp.miss_done = &w.ctrl->miss_done[0];
    rp.out = q.out;
    KN_HIP(ctx, launch_raygen_pt(rp, stream));
    // groups of rounds, each followed by a shading pass that scatters the
    // hits into the next segments; stop when a round marched nothing and the
    // shading spawned nothing
    constexpr int kGroup = 4;
    const int max_groups = (int)((c->bounces + 1) * (c->max_steps + 2)) / kGroup + 4;
    int r = 0;
    for (int gi = 0;; ++gi) {
      if (gi >= max_groups) return fail(KN_E_DEVICE, "path tracing did not finish in %d round groups", gi);
      for (int k = 0; k < kGroup; ++k, ++r) {
        if ((st = ev(&e0)) != KN_OK || (st = ev(&e1)) != KN_OK) return st;
        if (timed) march_ev.push_back({(int)next_ev - 2, (int)next_ev - 1});
        const bool after_shade = k == 0 && r > 0;
        st = enqueue_round(ctx, w, cfg, r, r == 0 ? (uint32_t)rays : 0u, stream, e0, e1,
                           after_shade ? &w.ctrl->n_in : nullptr);
        if (st != KN_OK) return st;
        ++rounds;
      }
      if ((st = ev(&e0)) != KN_OK || (st = ev(&e1)) != KN_OK) return st;
      if (timed) shade_ev.push_back({(int)next_ev - 2, (int)next_ev - 1});
      st = enqueue_shade(ctx, w, cfg, (uint32_t)rays, stream, e0, e1, true, r);
      if (st != KN_OK) return st;
      KN_HIP(ctx, hipMemcpyAsync(&ctx->pinned[0], &w.ctrl->n_chunks[(r - 1) & 1], 4, hipMemcpyDeviceToHost,
                                 stream));
      KN_HIP(ctx, hipMemcpyAsync(&ctx->pinned[1], &w.ctrl->n_in, 4, hipMemcpyDeviceToHost, stream));
      KN_HIP(ctx, hipMemcpyAsync(&ctx->pinned[2], &w.ctrl->scan_err, 4, hipMemcpyDeviceToHost, stream));
      KN_HIP(ctx, hipEventRecord(ctx->ev_round[0], stream));
      KN_HIP(ctx, hipEventSynchronize(ctx->ev_round[0]));
      if ((st = check_scan(ctx, ctx->pinned[2])) != KN_OK) return st;
      if (ctx->pinned[0] == 0 && ctx->pinned[1] == 0) break;
    }
    ResolveArgs ra{w.path, (uint32_t)npix, spp, fr->rgb, fr->accum, q.sample_offset};
    KN_HIP(ctx, launch_resolve(ra, stream));
  }
  KN_HIP(ctx, hipMemcpyAsync(&ctx->pinned[kPinnedScanErr], &w.ctrl->scan_err, 4, hipMemcpyDeviceToHost, stream));
  if (forked)
    KN_HIP(ctx, hipMemcpyAsync(&ctx->pinned[kPinnedScanErr2], &w.ctrl2->scan_err, 4, hipMemcpyDeviceToHost, stream));
  KN_HIP(ctx, hipEventRecord(ctx->ev_end, stream));
  KN_HIP(ctx, hipEventSynchronize(ctx->ev_end));
  if ((st = check_scan(ctx, ctx->pinned[kPinnedScanErr])) != KN_OK) return st;
  if (forked && (st = check_scan(ctx, ctx->pinned[kPinnedScanErr2])) != KN_OK) return st;
  if (stats) {
    Ctrl hc;
    KN_HIP(ctx, hipMemcpy(&hc, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    if (forked) {
      uint32_t h2 = 0;
      KN_HIP(ctx, hipMemcpy(&h2, &w.ctrl2->n_hits, 4, hipMemcpyDeviceToHost));
      hc.n_hits += h2;
    }
    float ms = 0.0f;
    KN_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_end));
    stats->gpu_ms = ms;
    stats->wall_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0).count();
    stats->rays = rays;
    stats->evals = stats->march_tiles = stats->march_chunks = 0;
    for (uint32_t l = 0; l < kTallyLines; ++l) {
      stats->evals += hc.tally[l][0];
      stats->march_tiles += hc.tally[l][1];
      stats->march_chunks += hc.tally[l][2];
    }
    stats->hits = hc.n_hits;
    stats->rounds = (uint64_t)rounds;
    stats->march_launches = 0;
    stats->march_ms = stats->shade_ms = 0.0;
    if (timed) {
      for (auto& pr : march_ev) {
        float kms = 0.0f;
        KN_HIP(ctx, hipEventElapsedTime(&kms, ctx->ev_kernel[pr.first], ctx->ev_kernel[pr.second]));
        stats->march_ms += kms;
      }
      for (auto& pr : shade_ev) {
        float kms = 0.0f;
        KN_HIP(ctx, hipEventElapsedTime(&kms, ctx->ev_kernel[pr.first], ctx->ev_kernel[pr.second]));
        stats->shade_ms += kms;
      }
      stats->march_launches = (uint32_t)march_ev.size();
    }
  }
  return KN_OK;
}


// Enqueues and runs one frame of a world (Sec. 3.4, shared scenes) on
// `stream`; the caller holds render_mu.  The instances are the pool's scene
// table (one global cell range each).  Camera rays start in a world list;
// k_world_step takes each ray to its next object: primitive hits are shaded
// (and, path tracing, scattered) there, instance entries become march
// records of the next round.  Groups of rounds follow, each closed by a
// shading pass; rays that leave an instance's box, and paths scattered off
// instance surfaces, go to the group's world list, which the next
// k_world_step takes.
kn_status render_world(kn_ctx* ctx, KnWorld* wd, const kn_camera* c, const kn_frame* fr, hipStream_t stream,
                       kn_stats* stats) {
  const auto wall0 = std::chrono::steady_clock::now();
  const bool pt = c->bounces > 0;
  const uint32_t spp = pt ? c->spp : 1u;
  const size_t npix = (size_t)c->width * c->height;
  const size_t rays = npix * spp;
  const bool jumps = (c->flags & KN_CAMERA_UNCLAMPED_STEPS) != 0;
  const bool split = (c->flags & KN_CAMERA_SPLIT_BF16_SHADING) && c->precision != KN_FP32;
  const uint32_t n_inst = (uint32_t)wd->inst.size();
  int hmode = -1;
  uint32_t mw = 0, shw = 0, cells = 0;
  for (uint32_t k = 0; k < n_inst; ++k) {
    const KnScene* sc = wd->scenes[k];
    SceneEnt e = scene_entry(sc, (int)c->precision, cells, split);
    for (int a = 0; a < 3; ++a) e.wt[a] = wd->inst[k].translate[a];
    e.ws = wd->inst[k].scale;
    ctx->h_scene[k] = e;
    cells = e.cell_end;
    hmode = hmode < 0 ? sc->H : (hmode == sc->H ? hmode : 0);
    mw = std::max(mw, e.march_words);
    shw = std::max(shw, e.shade_words);
  }
  if (hmode < 0) hmode = 64;   // no instances: the rounds find no work
  if (jumps && hmode == 0)
    return fail(KN_E_UNSUPPORTED, "unclamped steps need instances of one MLP width");
  const uint32_t gcells = std::max<uint32_t>(cells, 1u);
  kn_status st = ensure_pool(ctx, ctx->ws, rays, gcells, pt, jumps, true);
  if (st != KN_OK) return st;
  Pool& w = ctx->ws;
  ReqEnt q{};
  q.out = out_ptrs(fr);
  q.out.seg = nullptr;   // no segment records in worlds
  q.eps = c->eps;
  q.max_steps = c->max_steps;
  q.npix = (uint32_t)npix;
  q.pt = pt ? 1u : 0u;
  q.spp = spp;
  q.bounces = c->bounces;
  q.seed_lo = (uint32_t)c->seed;
  q.seed_hi = (uint32_t)(c->seed >> 32);
  q.env = c->env_rgb;
  q.env_w = c->env_w;
  q.env_h = c->env_h;
  q.unclamped = jumps ? 1u : 0u;
  q.world = 1u;
  q.sample_offset = pt ? c->sample_offset : 0u;
  *ctx->h_req = q;
  RoundCfg cfg{hmode, (int)c->precision, n_inst, mw, shw, split, jumps, gcells, ctx->max_passes};

  const bool timed = stats && stats->kernel_times;
  std::vector<std::pair<int, int>> march_ev, shade_ev;
  size_t next_ev = 0;
  auto ev = [&](hipEvent_t* e) -> kn_status {
    if (!timed) {
      *e = nullptr;
      return KN_OK;
    }
    if (next_ev == ctx->ev_kernel.size()) {
      hipEvent_t x;
      KN_HIP(ctx, hipEventCreate(&x));
      ctx->ev_kernel.push_back(x);
    }
    *e = ctx->ev_kernel[next_ev++];
    return KN_OK;
  };
  hipEvent_t e0, e1;

  KN_HIP(ctx, hipEventRecord(ctx->ev_start, stream));
  if (n_inst)
    KN_HIP(ctx, hipMemcpyAsync(w.scenes, ctx->h_scene, n_inst * sizeof(SceneEnt), hipMemcpyHostToDevice, stream));
  KN_HIP(ctx, hipMemcpyAsync(w.reqs, ctx->h_req, sizeof(ReqEnt), hipMemcpyHostToDevice, stream));
  KN_HIP(ctx, hipMemsetAsync(w.ctrl, 0, sizeof(Ctrl), stream));
  KN_HIP(ctx, hipMemsetAsync(w.counts, 0, 2 * w.cells * w.cs * 4, stream));
  KN_HIP(ctx, hipMemsetAsync(w.runs, 0, 2 * w.cells * w.cs * 4, stream));
  KN_HIP(ctx, hipMemsetAsync(w.hit_count, 0, w.cells * w.cs * 4, stream));
  KN_HIP(ctx, hipMemsetAsync(w.HL, 0xFF, rays * sizeof(RayRec), stream));

  RaygenArgs rg{};
  camera_basis(c, rg);
  WorldRaygenArgs wr{};
  for (int k = 0; k < 3; ++k) {
    wr.eye[k] = rg.eye[k];
    wr.fwd[k] = rg.fwd[k];
    wr.right[k] = rg.right[k];
    wr.up[k] = rg.up[k];
  }
  wr.tx = rg.tx;
  wr.ty = rg.ty;
  wr.W = (int)c->width;
  wr.Hh = (int)c->height;
  wr.spp = spp;
  wr.jitter = fr->accum ? 1u : 0u;
  wr.sample_offset = q.sample_offset;
  wr.seed_lo = q.seed_lo;
  wr.seed_hi = q.seed_hi;
  wr.pt = pt;
  wr.path = w.path;
  wr.out = w.W + w.cap;   // list 1: group 0 appends to list 0
  KN_HIP(ctx, launch_world_raygen(wr, (uint32_t)rays, stream));

  WorldStepArgs ws{};
  ws.tabs = pool_tabs(w, n_inst);
  ws.prims = wd->prims;
  ws.n_prims = wd->n_prims;
  ws.rs = w.rs;
  ws.ws = w.WS;
  ws.spawn = w.Uin;
  ws.n_spawn = &w.ctrl->n_in;
  ws.cs = w.cs;
  // k_world_step over `n` records of list `in` (or *n_dev of them), into the
  // march records of round r
  auto world_step = [&](int list, uint32_t n, const uint32_t* n_dev, int r) -> kn_status {
    KN_HIP(ctx, launch_fill_u32(&w.ctrl->n_in, 1, 0u, stream));
    ws.in = w.W + (size_t)list * w.cap;
    ws.n = n;
    ws.n_dev = n_dev;
    ws.counts_next = w.counts + (size_t)(r & 1) * w.cells * w.cs;
    KN_HIP(ctx, launch_world_step(ws, persistent_grid(ctx, 4), stream));
    return KN_OK;
  };
  if ((st = world_step(1, (uint32_t)rays, nullptr, 0)) != KN_OK) return st;

  // a ray segment enters at most every instance once, each for at most
  // max_steps + 2 rounds, and waits at most a group at each box
  constexpr int kGroup = 4;
  const int max_groups =
      (int)((c->bounces + 1) * ((n_inst + 1) * (c->max_steps + 2 + kGroup) / kGroup + 2)) + 4;
  int r = 0, rounds = 0;
  for (int gi = 0;; ++gi) {
    if (gi >= max_groups) return fail(KN_E_DEVICE, "world render did not finish in %d round groups", gi);
    cfg.wpar = gi & 1;
    for (int k = 0; k < kGroup; ++k, ++r) {
      if ((st = ev(&e0)) != KN_OK || (st = ev(&e1)) != KN_OK) return st;
      if (timed) march_ev.push_back({(int)next_ev - 2, (int)next_ev - 1});
      cfg.wzero = k == 0;
      st = enqueue_round(ctx, w, cfg, r, 0u, stream, e0, e1, k == 0 ? &w.ctrl->n_in : nullptr);
      if (st != KN_OK) return st;
      ++rounds;
    }
    if ((st = ev(&e0)) != KN_OK || (st = ev(&e1)) != KN_OK) return st;
    if (timed) shade_ev.push_back({(int)next_ev - 2, (int)next_ev - 1});
    st = enqueue_shade(ctx, w, cfg, (uint32_t)rays, stream, e0, e1, pt, r);
    if (st != KN_OK) return st;
    if ((st = world_step(cfg.wpar, 0u, &w.ctrl->n_w[cfg.wpar], r)) != KN_OK) return st;
    KN_HIP(ctx, hipMemcpyAsync(&ctx->pinned[0], &w.ctrl->n_chunks[(r - 1) & 1], 4, hipMemcpyDeviceToHost,
                               stream));
    KN_HIP(ctx, hipMemcpyAsync(&ctx->pinned[1], &w.ctrl->n_in, 4, hipMemcpyDeviceToHost, stream));
    KN_HIP(ctx, hipMemcpyAsync(&ctx->pinned[2], &w.ctrl->scan_err, 4, hipMemcpyDeviceToHost, stream));
    KN_HIP(ctx, hipEventRecord(ctx->ev_round[0], stream));
    KN_HIP(ctx, hipEventSynchronize(ctx->ev_round[0]));
    if ((st = check_scan(ctx, ctx->pinned[2])) != KN_OK) return st;
    if (ctx->pinned[0] == 0 && ctx->pinned[1] == 0) break;
  }
  if (pt) {
    ResolveArgs ra{w.path, (uint32_t)npix, spp, fr->rgb, fr->accum, q.sample_offset};
    KN_HIP(ctx, launch_resolve(ra, stream));
  }
  KN_HIP(ctx, hipMemcpyAsync(&ctx->pinned[kPinnedScanErr], &w.ctrl->scan_err, 4, hipMemcpyDeviceToHost, stream));
  KN_HIP(ctx, hipEventRecord(ctx->ev_end, stream));
  KN_HIP(ctx, hipEventSynchronize(ctx->ev_end));
  if ((st = check_scan(ctx, ctx->pinned[kPinnedScanErr])) != KN_OK) return st;
  if (stats) {
    Ctrl hc;
    KN_HIP(ctx, hipMemcpy(&hc, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    float ms = 0.0f;
    KN_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_end));
    stats->gpu_ms = ms;
    stats->wall_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0).count();
    stats->rays = rays;
    stats->evals = stats->march_tiles = stats->march_chunks = 0;
    for (uint32_t l = 0; l < kTallyLines; ++l) {
      stats->evals += hc.tally[l][0];
      stats->march_tiles += hc.tally[l][1];
      stats->march_chunks += hc.tally[l][2];
    }
    stats->hits = hc.n_hits;
    stats->rounds = (uint64_t)rounds;
    stats->march_launches = 0;
    stats->march_ms = stats->shade_ms = 0.0;
    if (timed) {
      for (auto& pr : march_ev) {
        float kms = 0.0f;
        KN_HIP(ctx, hipEventElapsedTime(&kms, ctx->ev_kernel[pr.first], ctx->ev_kernel[pr.second]));
        stats->march_ms += kms;
      }
      for (auto& pr : shade_ev) {
        float kms = 0.0f;
        KN_HIP(ctx, hipEventElapsedTime(&kms, ctx->ev_kernel[pr.first], ctx->ev_kernel[pr.second]));
        stats->shade_ms += kms;
      }
      stats->march_launches = (uint32_t)march_ev.size();
    }
  }
  return KN_OK;
}

}  // namespace kn

extern "C" {

kn_status kn_render(kn_ctx* ctx, kn_scene_id scene, const kn_camera* cam, const kn_frame* frame,
                    kn_stats* stats) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  KnScene* s = find_scene(ctx, scene);
  if (!s) return fail(KN_E_NOT_FOUND, "scene %u not found", scene);
  st = validate_camera(cam, s);
  if (st != KN_OK) return st;
  if ((st = validate_frame(frame, cam)) != KN_OK) return st;
  std::lock_guard<std::mutex> lk(ctx->render_mu);
  KN_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t stream = frame->hip_stream ? (hipStream_t)frame->hip_stream : ctx->stream;
  s->refs++;
  st = render_frame(ctx, s, cam, frame, stream, stats);
  s->refs--;
  return st;
}

constexpr uint32_t kMaxWorldPrims = 256;

static kn_status check_primitive(const kn_primitive& p, uint32_t i) {
  for (float v : p.p)
    if (!std::isfinite(v)) return fail(KN_E_INVALID, "primitive %u: non-finite parameter", i);
  for (float v : p.albedo)
    if (!(v >= 0.0f && v <= 1.0f)) return fail(KN_E_INVALID, "primitive %u: albedo outside [0, 1]", i);
  if (p.kind == KN_PRIM_SPHERE) {
    if (!(p.p[3] > 0.0f)) return fail(KN_E_INVALID, "primitive %u: sphere radius must be positive", i);
  } else if (p.kind == KN_PRIM_BOX) {
    for (int a = 0; a < 3; ++a)
      if (!(p.p[a] < p.p[3 + a])) return fail(KN_E_INVALID, "primitive %u: box min not below max on axis %d", i, a);
  } else if (p.kind == KN_PRIM_TRIANGLE) {
    const double e1[3] = {(double)p.p[3] - p.p[0], (double)p.p[4] - p.p[1], (double)p.p[5] - p.p[2]};
    const double e2[3] = {(double)p.p[6] - p.p[0], (double)p.p[7] - p.p[1], (double)p.p[8] - p.p[2]};
    const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                 cz = e1[0] * e2[1] - e1[1] * e2[0];
    if (!(cx * cx + cy * cy + cz * cz > 0.0)) return fail(KN_E_INVALID, "primitive %u: degenerate triangle", i);
  } else {
    return fail(KN_E_INVALID, "primitive %u: unknown kind %u", i, p.kind);
  }
  return KN_OK;
}

kn_status kn_world_create(kn_ctx* ctx, const kn_world_desc* d, kn_world_id* out) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  if (!d || !out) return fail(KN_E_INVALID, "desc or out is NULL");
  if (d->n_instances > (uint32_t)kMaxScenes)
    return fail(KN_E_INVALID, "%u instances, at most %d", d->n_instances, kMaxScenes);
  if (d->n_primitives > kMaxWorldPrims)
    return fail(KN_E_INVALID, "%u primitives, at most %u", d->n_primitives, kMaxWorldPrims);
  if ((d->n_instances && !d->instances) || (d->n_primitives && !d->primitives))
    return fail(KN_E_INVALID, "instances or primitives is NULL");
  for (uint32_t i = 0; i < d->n_primitives; ++i)
    if ((st = check_primitive(d->primitives[i], i)) != KN_OK) return st;
  std::unique_ptr<KnWorld> w(new KnWorld());
  std::vector<std::array<double, 6>> boxes;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    uint64_t cells = 0;
    for (uint32_t k = 0; k < d->n_instances; ++k) {
      const kn_instance& in = d->instances[k];
      auto it = ctx->scenes.find(in.scene);
      if (it == ctx->scenes.end()) return fail(KN_E_NOT_FOUND, "instance %u: scene %u not found", k, in.scene);
      if (!(in.scale > 0.0f) || !std::isfinite(in.scale))
        return fail(KN_E_INVALID, "instance %u: scale must be positive and finite", k);
      for (float v : in.translate)
        if (!std::isfinite(v)) return fail(KN_E_INVALID, "instance %u: non-finite translation", k);
      const KnScene* sc = it->second;
      std::array<double, 6> b;
      for (int a = 0; a < 3; ++a) {
        b[a] = (double)in.translate[a] + (double)in.scale * sc->geom.bmin[a];
        b[3 + a] = (double)in.translate[a] + (double)in.scale * sc->geom.bmax[a];
      }
      for (uint32_t j = 0; j < k; ++j) {
        bool overlap = true;
        for (int a = 0; a < 3; ++a) overlap = overlap && b[a] < boxes[j][3 + a] && boxes[j][a] < b[3 + a];
        if (overlap) return fail(KN_E_INVALID, "instances %u and %u have overlapping boxes", j, k);
      }
      boxes.push_back(b);
      cells += (uint64_t)sc->N * sc->N * sc->N;
      w->inst.push_back(in);
      w->scenes.push_back(it->second);
    }
    if (cells > kCellMask)
      return fail(KN_E_INVALID, "instances hold %llu cells, at most %u", (unsigned long long)cells, kCellMask);
    w->cells = (uint32_t)cells;
  }
  w->n_prims = d->n_primitives;
  w->bytes = (size_t)std::max<uint32_t>(d->n_primitives, 1u) * sizeof(PrimDev);
  if (ctx->used.load() + w->bytes > ctx->budget) return fail(KN_E_NOMEM, "world exceeds the HBM budget");
  std::vector<PrimDev> hp(std::max<uint32_t>(d->n_primitives, 1u), PrimDev{0u, {}, {}});
  for (uint32_t i = 0; i < d->n_primitives; ++i) {
    hp[i].kind = d->primitives[i].kind;
    for (int k = 0; k < 9; ++k) hp[i].p[k] = d->primitives[i].p[k];
    for (int k = 0; k < 3; ++k) hp[i].albedo[k] = d->primitives[i].albedo[k];
  }
  KN_HIP(ctx, hipSetDevice(ctx->device));
  KN_HIP(ctx, hipMalloc(&w->prims, hp.size() * sizeof(PrimDev)));
  {
    const hipError_t e = hipMemcpy(w->prims, hp.data(), hp.size() * sizeof(PrimDev), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(w->prims);
      ctx->poisoned = true;
      return fail(KN_E_DEVICE, "hipMemcpy of the primitives failed: %s", hipGetErrorString(e));
    }
  }
  ctx->used += w->bytes;
  std::lock_guard<std::mutex> lk(ctx->mu);
  // the scenes may have gone between the two locks
  for (uint32_t k = 0; k < d->n_instances; ++k) {
    auto it = ctx->scenes.find(d->instances[k].scene);
    if (it == ctx->scenes.end() || it->second != w->scenes[k]) {
      (void)hipFree(w->prims);
      ctx->used -= w->bytes;
      return fail(KN_E_NOT_FOUND, "instance %u: scene %u was destroyed", k, d->instances[k].scene);
    }
  }
  for (KnScene* sc : w->scenes) sc->world_refs++;
  KnWorld* wp = w.release();
  wp->id = ctx->next_world++;
  ctx->worlds[wp->id] = wp;
  *out = wp->id;
  return KN_OK;
}

kn_status kn_world_destroy(kn_ctx* ctx, kn_world_id id) {
  if (!ctx) return fail(KN_E_INVALID, "ctx is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->worlds.find(id);
  if (it == ctx->worlds.end()) return fail(KN_E_NOT_FOUND, "world %u not found", id);
  KnWorld* w = it->second;
  if (w->refs.load() > 0) return fail(KN_E_BUSY, "world %u is being rendered", id);
  std::lock_guard<std::mutex> rk(ctx->render_mu);
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (KnScene* sc : w->scenes) sc->world_refs--;
  if (w->prims) (void)hipFree(w->prims);
  ctx->used -= w->bytes;
  delete w;
  ctx->worlds.erase(it);
  return KN_OK;
}

kn_status kn_render_world(kn_ctx* ctx, kn_world_id world, const kn_camera* cam, const kn_frame* frame,
                          kn_stats* stats) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  KnWorld* w;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->worlds.find(world);
    if (it == ctx->worlds.end()) return fail(KN_E_NOT_FOUND, "world %u not found", world);
    w = it->second;
    st = validate_camera(cam, nullptr);
    if (st != KN_OK) return st;
    for (size_t k = 0; k < w->scenes.size(); ++k)
      if (!w->scenes[k]->march(cam->precision))
        return fail(KN_E_INVALID, "instance %zu: its scene has no copy in precision %d", k, (int)cam->precision);
    w->refs++;
  }
  if ((st = validate_frame(frame, cam)) != KN_OK) {
    w->refs--;
    return st;
  }
  {
    std::lock_guard<std::mutex> rk(ctx->render_mu);
    const hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) {
      w->refs--;
      ctx->poisoned = true;
      return fail(KN_E_DEVICE, "hipSetDevice failed: %s", hipGetErrorString(e));
    }
    hipStream_t stream = frame->hip_stream ? (hipStream_t)frame->hip_stream : ctx->stream;
    st = render_world(ctx, w, cam, frame, stream, stats);
  }
  w->refs--;
  return st;
}

kn_status kn_query(kn_ctx* ctx, kn_scene_id scene, kn_precision precision, const float* points,
                   uint64_t n, float* d_out, float* grad_out, float* z_out, void* hip_stream) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  KnScene* s = find_scene(ctx, scene);
  if (!s) return fail(KN_E_NOT_FOUND, "scene %u not found", scene);
  if (n == 0) return KN_OK;
  if ((st = validate_query(s, precision, points, n)) != KN_OK) return st;
  std::lock_guard<std::mutex> lk(ctx->render_mu);
  KN_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t stream = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
  const size_t cells = (size_t)s->N * s->N * s->N;
  st = ensure_pool(ctx, ctx->ws, n, cells);
  if (st != KN_OK) return st;
  Pool& w = ctx->ws;
  const QueryBufs b{w.U, w.S, w.counts, w.cursor, w.chunk, w.ctrl, w.cs};
  st = enqueue_query(ctx, s, precision, points, n, d_out, grad_out, z_out, stream, b, false);
  if (st != KN_OK) return st;
  KN_HIP(ctx, hipMemcpyAsync(&ctx->pinned[kPinnedScanErr], &w.ctrl->scan_err, 4, hipMemcpyDeviceToHost, stream));
  KN_HIP(ctx, hipStreamSynchronize(stream));
  return check_scan(ctx, ctx->pinned[kPinnedScanErr]);
}

kn_status kn_query_noalloc(kn_ctx* ctx, kn_scene_id scene, kn_precision precision, const float* points,
                           uint64_t n, float* d_out, float* grad_out, float* z_out, void* hip_stream) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  KnScene* s = find_scene(ctx, scene);
  if (!s) return fail(KN_E_NOT_FOUND, "scene %u not found", scene);
  if (n == 0) return KN_OK;
  if ((st = validate_query(s, precision, points, n)) != KN_OK) return st;
  if (n > kNoAllocMaxPoints)
    return fail(KN_E_INVALID, "%llu points exceed the allocation-free query's limit of %u (use kn_query)",
                (unsigned long long)n, kNoAllocMaxPoints);
  const size_t cells = (size_t)s->N * s->N * s->N;
  if (cells > kNoAllocMaxCells)
    return fail(KN_E_INVALID, "%zu cells exceed the allocation-free query's limit of %u", cells, kNoAllocMaxCells);
  if (!ctx->scratch)
    return fail(KN_E_DEVICE, "no address of the scratch array on device %d: %s", ctx->device,
                hipGetErrorString(ctx->scratch_err));
  // the device's one scratch array: calls of this process on the device are
  // serialised here (the call returns after its work is done)
  std::lock_guard<std::mutex> lk(scratch_mutex(ctx->device));
  KN_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t stream = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
  const NoAllocLayout L = noalloc_layout();
  uint8_t* base = ctx->scratch;
  const QueryBufs b{reinterpret_cast<RayRec*>(base + L.U), reinterpret_cast<RayRec*>(base + L.S),
                    reinterpret_cast<uint32_t*>(base + L.counts), reinterpret_cast<uint32_t*>(base + L.cursor),
                    reinterpret_cast<uint2*>(base + L.chunks), reinterpret_cast<Ctrl*>(base + L.ctrl), 1u};
  s->refs++;
  st = enqueue_query(ctx, s, precision, points, n, d_out, grad_out, z_out, stream, b, true);
  if (st == KN_OK) {
    if (hipMemcpyAsync(&ctx->pinned[kPinnedScanErrNoAlloc], &b.ctrl->scan_err, 4, hipMemcpyDeviceToHost,
                       stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
      ctx->poisoned = true;
      st = fail(KN_E_DEVICE, "allocation-free query: %s", hipGetErrorString(hipGetLastError()));
    } else {
      st = check_scan(ctx, ctx->pinned[kPinnedScanErrNoAlloc]);
    }
  }
  s->refs--;
  return st;
}

kn_status kn_grid_sample(kn_ctx* ctx, kn_scene_id scene, kn_precision precision, uint32_t R, float* d_out,
                         float* grad_out, void* hip_stream) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  KnScene* s = find_scene(ctx, scene);
  if (!s) return fail(KN_E_NOT_FOUND, "scene %u not found", scene);
  if (!d_out) return fail(KN_E_INVALID, "d_out is NULL");
  if (R < 2 || R > kGridMaxR) return fail(KN_E_INVALID, "lattice size R = %u outside [2, %u]", R, kGridMaxR);
  if (precision != KN_FP32 && precision != KN_BF16 && precision != KN_FP8_E4M3)
    return fail(KN_E_INVALID, "unknown precision %d", (int)precision);
  if (grad_out && precision != KN_FP32)
    return fail(KN_E_INVALID, "gradients are computed with the float32 weights (precision KN_FP32)");
  if (!s->march(precision)) return fail(KN_E_INVALID, "scene has no copy in precision %d", (int)precision);
  // work items per cell: enough 256-point parts for the largest cell
  const uint32_t N = s->N;
  uint32_t nmax = 0;
  for (uint32_t c = 0; c < N; ++c) {
    const uint32_t lo = (uint32_t)(((uint64_t)c * (R - 1u) + N - 1u) / N);
    const uint32_t hi = c + 1u >= N ? R : (uint32_t)(((uint64_t)(c + 1u) * (R - 1u) + N - 1u) / N);
    nmax = std::max(nmax, hi - lo);
  }
  const uint64_t per_cell = (uint64_t)nmax * nmax * nmax;
  if (per_cell >= (1ull << 31))
    return fail(KN_E_INVALID, "%llu lattice points in one cell exceed the limit of 2^31",
                (unsigned long long)per_cell);
  const uint64_t K = (per_cell + 255u) / 256u;
  std::lock_guard<std::mutex> lk(ctx->render_mu);
  KN_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t stream = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
  GridArgs ga{};
  ga.sg = s->geom;
  ga.spk = softplus_consts(s->geom.beta);
  ga.R = R;
  ga.K = (uint32_t)K;
  ga.rm1 = (float)(R - 1u);
  ga.d_out = d_out;
  s->refs++;
  hipError_t e;
  if (grad_out) {
    ga.blocks = s->shade;
    ga.block_words = s->shade_words;
    ga.grad_out = grad_out;
    e = launch_grid_full(ga, s->H, persistent_grid(ctx, 2), stream);
  } else {
    ga.blocks = s->march(precision);
    ga.block_words = s->march_words(precision);
    e = launch_grid_d(ga, s->H, (int)precision, persistent_grid(ctx, 2), stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  s->refs--;
  if (e != hipSuccess) {
    ctx->poisoned = true;
    return fail(KN_E_DEVICE, "lattice sampling: %s", hipGetErrorString(e));
  }
  return KN_OK;
}

kn_status kn_eikonal_fd(kn_ctx* ctx, kn_scene_id scene, kn_precision precision, const float* points, uint64_t n,
                        float delta, float* gnorm_out, float* stencil_out, double* loss_out, void* hip_stream) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  KnScene* s = find_scene(ctx, scene);
  if (!s) return fail(KN_E_NOT_FOUND, "scene %u not found", scene);
  if (!gnorm_out) return fail(KN_E_INVALID, "gnorm_out is NULL");
  if (!(delta > 0.0f) || !std::isfinite(delta)) return fail(KN_E_INVALID, "delta must be positive and finite");
  if (n == 0) return KN_OK;
  if (n > kEikMaxPoints)
    return fail(KN_E_INVALID, "%llu points exceed the limit of %llu", (unsigned long long)n,
                (unsigned long long)kEikMaxPoints);
  if ((st = validate_query(s, precision, points, 6u * n)) != KN_OK) return st;
  std::lock_guard<std::mutex> lk(ctx->render_mu);
  KN_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t stream = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
  const size_t cells = (size_t)s->N * s->N * s->N;
  const uint64_t ns = 6u * n, nparts = (n + 255u) / 256u;
  // work buffer: stencil points, stencil values (unless the caller keeps
  // them), per-workgroup partial sums
  const size_t off_val = align256(ns * 3u * 4u), off_part = off_val + align256(ns * 4u);
  if ((st = ensure_aux(ctx, off_part + nparts * 8u)) != KN_OK) return st;
  if ((st = ensure_pool(ctx, ctx->ws, ns, cells)) != KN_OK) return st;
  uint8_t* aux = static_cast<uint8_t*>(ctx->aux);
  EikArgs ea{};
  ea.pts = points;
  ea.n = n;
  ea.delta = delta;
  ea.stencil_pts = reinterpret_cast<float*>(aux);
  float* vals = stencil_out ? stencil_out : reinterpret_cast<float*>(aux + off_val);
  ea.stencil = vals;
  ea.gnorm = gnorm_out;
  ea.partial = reinterpret_cast<double*>(aux + off_part);
  ea.loss = loss_out;
  s->refs++;
  hipError_t e = launch_eik_points(ea, stream);
  if (e != hipSuccess) {
    s->refs--;
    ctx->poisoned = true;
    return fail(KN_E_DEVICE, "eikonal stencil: %s", hipGetErrorString(e));
  }
  Pool& w = ctx->ws;
  const QueryBufs b{w.U, w.S, w.counts, w.cursor, w.chunk, w.ctrl, w.cs};
  st = enqueue_query(ctx, s, precision, ea.stencil_pts, ns, vals, nullptr, nullptr, stream, b, false);
  s->refs--;
  if (st != KN_OK) return st;
  KN_HIP(ctx, launch_eik_combine(ea, stream));
  KN_HIP(ctx, hipMemcpyAsync(&ctx->pinned[kPinnedScanErr], &w.ctrl->scan_err, 4, hipMemcpyDeviceToHost, stream));
  KN_HIP(ctx, hipStreamSynchronize(stream));
  return check_scan(ctx, ctx->pinned[kPinnedScanErr]);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// serving: continuous batching of render requests in one shared ray pool
// ---------------------------------------------------------------------------
namespace kn {

struct Request {
  enum State { kQueued, kRunning, kDone, kFailed };
  kn_request_id id = 0;
  KnScene* scene = nullptr;
  kn_camera cam{};
  OutPtrs out{};
  uint32_t npix = 0;
  int slot = -1;
  size_t base = 0;          // first pool ray id
  int64_t admit_group = -1; // round group whose rays started it
  State state = kQueued;
  uint32_t hits = 0;
  uint64_t rounds = 0;
  std::chrono::steady_clock::time_point t_submit, t_admit, t_done;
};

// The loop thread owns the pool, its stream and the tables.  Between groups
// of kGroupRounds rounds it admits queued requests in arrival order while a
// request slot and a contiguous range of pool ray ids are free (the pool is
// the HBM budget of ray state), generates their rays into the next round,
// runs the rounds and a shading pass over the pool, and retires requests
// whose rays have all finished (per-slot miss and hit counters, read back
// one group late so the host never waits on the group in flight).
class ServeLoop {
 public:
  static constexpr int kGroupRounds = 4;

  ServeLoop(kn_ctx* c, uint32_t mi, kn_precision p) : ctx(c), max_inflight(mi), prec(p) {}
  kn_precision precision() const { return prec; }

  kn_status start(size_t cap, size_t cell_cap) {
    KN_HIP(ctx, hipSetDevice(ctx->device));
    kn_status st = ensure_pool(ctx, pool, cap, cell_cap);
    if (st != KN_OK) return st;
    this->cell_cap = cell_cap;
    KN_HIP(ctx, hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    for (auto& e : ev) KN_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    KN_HIP(ctx, hipHostMalloc((void**)&head, 4 * (size_t)kCtrlHead, hipHostMallocDefault));
    KN_HIP(ctx, hipHostMalloc((void**)&h_scenes, kMaxScenes * sizeof(SceneEnt), hipHostMallocDefault));
    KN_HIP(ctx, hipHostMalloc((void**)&h_reqs, kMaxSlots * sizeof(ReqEnt), hipHostMallocDefault));
    KN_HIP(ctx, hipMemsetAsync(pool.ctrl, 0, sizeof(Ctrl), stream));
    KN_HIP(ctx, hipMemsetAsync(pool.counts, 0, 2 * pool.cells * pool.cs * 4, stream));
    KN_HIP(ctx, hipMemsetAsync(pool.runs, 0, 2 * pool.cells * pool.cs * 4, stream));
    KN_HIP(ctx, hipMemsetAsync(pool.hit_count, 0, pool.cells * pool.cs * 4, stream));
    KN_HIP(ctx, hipStreamSynchronize(stream));
    free_ranges[0] = pool.cap;
    th = std::thread([this] { run(); });
    return KN_OK;
  }

  // drains every submitted request, then stops the thread and frees the pool
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stopping = true;
    }
    cv_work.notify_all();
    if (th.joinable()) th.join();
    (void)hipSetDevice(ctx->device);
    if (stream) (void)hipStreamSynchronize(stream);
    ctx->used -= pool.bytes;
    free_pool(pool);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (stream) (void)hipStreamDestroy(stream);
    if (head) (void)hipHostFree(head);
    if (h_scenes) (void)hipHostFree(h_scenes);
    if (h_reqs) (void)hipHostFree(h_reqs);
    std::lock_guard<std::mutex> lk(mu);
    for (auto& kv : reqs)
      if (kv.second->state == Request::kQueued || kv.second->state == Request::kRunning) {
        kv.second->state = Request::kFailed;
        kv.second->scene->refs--;
      }
    cv_done.notify_all();
  }

  kn_status submit(KnScene* s, const kn_camera* cam, const kn_frame* fr, kn_request_id* out) {
    const uint32_t npix = cam->width * cam->height;
    if (npix > pool.cap)
      return fail(KN_E_NOMEM, "request of %u rays exceeds the serving pool (%zu rays)", npix, pool.cap);
    std::unique_ptr<Request> q(new Request());
    q->scene = s;
    q->cam = *cam;
    q->out = out_ptrs(fr);
    q->out.seg = nullptr;   // primary rays only: no path segments
    q->npix = npix;
    q->t_submit = std::chrono::steady_clock::now();
    {
      std::lock_guard<std::mutex> lk(mu);
      if (stopping || failed) return fail(KN_E_SHUTDOWN, "serving loop is stopping");
      q->id = next_id++;
      *out = q->id;
      queue.push_back(q.get());
      reqs[q->id] = std::move(q);
    }
    cv_work.notify_all();
    return KN_OK;
  }

  kn_status poll(kn_request_id id, int64_t timeout_us, kn_stats* stats) {
    std::unique_lock<std::mutex> lk(mu);
    auto it = reqs.find(id);
    if (it == reqs.end()) return fail(KN_E_NOT_FOUND, "request %llu not found", (unsigned long long)id);
    Request* q = it->second.get();
    auto finished = [q] { return q->state == Request::kDone || q->state == Request::kFailed; };
    if (!finished()) {
      if (timeout_us == 0) return KN_PENDING;
      if (timeout_us < 0) cv_done.wait(lk, finished);
      else if (!cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), finished))
        return fail(KN_E_TIMEOUT, "request %llu not finished", (unsigned long long)id);
    }
    if (q->state == Request::kFailed) {
      reqs.erase(it);
      return fail(KN_E_DEVICE, "request failed: %s", fail_msg.empty() ? "serving stopped" : fail_msg.c_str());
    }
    if (stats) {
      const uint32_t keep = stats->kernel_times;
      *stats = kn_stats{};
      stats->kernel_times = keep;
      stats->wall_ms = std::chrono::duration<double, std::milli>(q->t_done - q->t_submit).count();
      stats->gpu_ms = std::chrono::duration<double, std::milli>(q->t_done - q->t_admit).count();
      stats->rays = q->npix;
      stats->hits = q->hits;
      stats->rounds = q->rounds;
    }
    reqs.erase(it);
    return KN_OK;
  }

 private:
  struct TabEnt {
    kn_scene_id id;
    uint32_t base, cells, march_words, shade_words;
    int H;
  };

  kn_ctx* ctx;
  uint32_t max_inflight;
  kn_precision prec;
  Pool pool;
  size_t cell_cap = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  uint8_t* head = nullptr;       // pinned readback of the Ctrl head, one slot per group (mod 4)
  SceneEnt* h_scenes = nullptr;  // pinned staging of the tables
  ReqEnt* h_reqs = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::map<kn_request_id, std::unique_ptr<Request>> reqs;
  Request* slots[kMaxSlots] = {};
  uint32_t inflight = 0;
  std::map<size_t, size_t> free_ranges;  // begin -> end of free pool ray ids
  kn_request_id next_id = 1;
  bool stopping = false, failed = false;
  std::string fail_msg;
  std::vector<TabEnt> table;     // loop thread only
  uint32_t cells_used = 0;       // loop thread only

  bool alloc_range(size_t n, size_t* base) {
    for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
      if (it->second - it->first >= n) {
        *base = it->first;
        const size_t end = it->second;
        free_ranges.erase(it);
        if (*base + n < end) free_ranges[*base + n] = end;
        return true;
      }
    }
    return false;
  }

  void free_range(size_t base, size_t n) {
    size_t b = base, e = base + n;
    auto it = free_ranges.lower_bound(b);
    if (it != free_ranges.end() && it->first == e) {
      e = it->second;
      it = free_ranges.erase(it);
    }
    if (it != free_ranges.begin()) {
      auto pv = std::prev(it);
      if (pv->second == b) {
        b = pv->first;
        free_ranges.erase(pv);
      }
    }
    free_ranges[b] = e;
  }

  // table index of a scene, adding it (and uploading its entry) if needed;
  // -1 when the table is full
  int table_index(KnScene* s) {
    for (size_t k = 0; k < table.size(); ++k)
      if (table[k].id == s->id) return (int)k;
    const uint32_t cells = (uint32_t)(s->N * s->N * s->N);
    if (table.size() >= (size_t)kMaxScenes || (size_t)cells_used + cells > cell_cap) return -1;
    const int k = (int)table.size();
    h_scenes[k] = scene_entry(s, (int)prec, cells_used, false);
    if (hipMemcpyAsync(pool.scenes + k, h_scenes + k, sizeof(SceneEnt), hipMemcpyHostToDevice, stream) !=
        hipSuccess)
      return -2;
    table.push_back(TabEnt{s->id, cells_used, cells, h_scenes[k].march_words, h_scenes[k].shade_words, s->H});
    cells_used += cells;
    return k;
  }

  // end of the highest pool ray-id range in use (the hits the shading pass
  // looks at); ranges of retired requests hold no hits
  uint32_t ray_extent() {
    std::lock_guard<std::mutex> lk(mu);
    size_t e = 0;
    for (Request* q : slots)
      if (q) e = std::max(e, q->base + q->npix);
    return (uint32_t)e;
  }

  RoundCfg round_cfg() const {
    RoundCfg c{};
    c.hmode = table.empty() ? 32 : table[0].H;
    for (const TabEnt& e : table) {
      if (e.H != c.hmode) c.hmode = 0;
      c.march_words = std::max(c.march_words, e.march_words);
      c.shade_words = std::max(c.shade_words, e.shade_words);
    }
    c.prec = (int)prec;
    c.split = false;
    c.n_scenes = (uint32_t)table.size();
    c.cells = cells_used;
    c.max_passes = ctx->max_passes;
    return c;
  }

  // admits requests in arrival order; returns them (caller enqueues their rays)
  std::vector<Request*> admit(int64_t group) {
    std::vector<Request*> adm;
    while (!queue.empty() && inflight < max_inflight) {
      Request* q = queue.front();
      int slot = -1;
      for (int i = 0; i < kMaxSlots; ++i)
        if (!slots[i]) {
          slot = i;
          break;
        }
      if (slot < 0) break;
      size_t base = 0;
      if (!alloc_range(q->npix, &base)) break;
      int k = table_index(q->scene);
      if (k == -1 && inflight == 0 && adm.empty()) {
        // idle pool with a full scene table: start a fresh table
        (void)hipStreamSynchronize(stream);
        table.clear();
        cells_used = 0;
        k = table_index(q->scene);
      }
      if (k < 0) {
        free_range(base, q->npix);
        break;
      }
      q->slot = slot;
      q->base = base;
      q->admit_group = group;
      q->state = Request::kRunning;
      q->t_admit = std::chrono::steady_clock::now();
      slots[slot] = q;
      ++inflight;
      queue.pop_front();
      adm.push_back(q);
    }
    return adm;
  }

  // enqueues the rays of an admitted request into Uin at offset *n_new
  kn_status start_request(Request* q, int r, uint32_t* n_new) {
    const int k = table_index(q->scene);
    if (k < 0) return fail(KN_E_DEVICE, "scene table lookup failed");
    h_reqs[q->slot] = ReqEnt{q->out, q->cam.eps, q->cam.max_steps, q->npix, 0u};
    KN_HIP(ctx, hipMemcpyAsync(pool.reqs + q->slot, h_reqs + q->slot, sizeof(ReqEnt), hipMemcpyHostToDevice,
                               stream));
    KN_HIP(ctx, hipMemsetAsync(&pool.ctrl->miss_done[q->slot], 0, 4, stream));
    KN_HIP(ctx, hipMemsetAsync(&pool.ctrl->hit_done[q->slot], 0, 4, stream));
    RaygenArgs rg{};
    rg.sg = h_scenes[k].sg;
    camera_basis(&q->cam, rg);
    rg.W = (int)q->cam.width;
    rg.Hh = (int)q->cam.height;
    rg.slot = (uint32_t)q->slot;
    rg.rid_base = (uint32_t)q->base;
    rg.rs = pool.rs;
    rg.U = pool.Uin + *n_new;
    rg.counts = pool.counts + (r & 1) * pool.cells * pool.cs;
    rg.cs = pool.cs;
    rg.miss_done = &pool.ctrl->miss_done[0];
    rg.out = q->out;
    KN_HIP(ctx, launch_raygen(rg, stream));
    *n_new += q->npix;
    return KN_OK;
  }

  // Counters of group `g`'s readback of the Ctrl head.  The slots are
  // kCtrlHead bytes apart, which is not the alignment of a whole Ctrl, so the
  // words are copied out rather than read through a Ctrl pointer.
  struct Head {
    uint32_t scan_err;
    uint32_t miss_done[kMaxSlots];
    uint32_t hit_done[kMaxSlots];
  };
  Head read_head(int64_t g) const {
    static_assert(offsetof(Ctrl, hit_done) + sizeof(Ctrl::hit_done) <= (size_t)kCtrlHead, "head size");
    const uint8_t* p = head + (size_t)(g & 3) * kCtrlHead;
    Head h;
    std::memcpy(&h.scan_err, p + offsetof(Ctrl, scan_err), sizeof h.scan_err);
    std::memcpy(h.miss_done, p + offsetof(Ctrl, miss_done), sizeof h.miss_done);
    std::memcpy(h.hit_done, p + offsetof(Ctrl, hit_done), sizeof h.hit_done);
    return h;
  }

  // retires the requests that group `g`'s readback shows finished
  void retire(int64_t g) {
    const Head hd = read_head(g);
    const Head* h = &hd;
    const auto now = std::chrono::steady_clock::now();
    bool any = false;
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < kMaxSlots; ++i) {
      Request* q = slots[i];
      if (!q || q->admit_group > g) continue;
      if ((uint64_t)h->miss_done[i] + h->hit_done[i] >= q->npix) {
        q->hits = h->hit_done[i];
        q->rounds = (uint64_t)(g - q->admit_group + 1) * kGroupRounds;
        q->t_done = now;
        q->state = Request::kDone;
        slots[i] = nullptr;
        free_range(q->base, q->npix);
        --inflight;
        q->scene->refs--;
        any = true;
      }
    }
    if (any) cv_done.notify_all();
  }

  kn_status loop() {
    KN_HIP(ctx, hipSetDevice(ctx->device));
    int r = 0;
    int64_t group = 0;
    for (;;) {
      std::vector<Request*> adm;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [this] { return stopping || !queue.empty() || inflight > 0; });
        if (stopping && queue.empty() && inflight == 0) break;
        adm = admit(group);
      }
      uint32_t n_new = 0;
      for (Request* q : adm) {
        kn_status st = start_request(q, r, &n_new);
        if (st != KN_OK) return st;
      }
      const RoundCfg cfg = round_cfg();
      for (int k = 0; k < kGroupRounds; ++k, ++r) {
        kn_status st = enqueue_round(ctx, pool, cfg, r, k == 0 ? n_new : 0u, stream, nullptr, nullptr);
        if (st != KN_OK) return st;
      }
      kn_status st = enqueue_shade(ctx, pool, cfg, ray_extent(), stream, nullptr, nullptr);
      if (st != KN_OK) return st;
      KN_HIP(ctx, hipMemcpyAsync(head + (size_t)(group & 3) * kCtrlHead, pool.ctrl, kCtrlHead,
                                 hipMemcpyDeviceToHost, stream));
      KN_HIP(ctx, hipEventRecord(ev[group & 3], stream));
      if (group > 0) {
        KN_HIP(ctx, hipEventSynchronize(ev[(group - 1) & 3]));
        // the flag is sticky in the serving pool: every request in flight
        // may have been binned wrongly, so all of them fail
        if ((st = check_scan(ctx, read_head(group - 1).scan_err)) != KN_OK) return st;
        retire(group - 1);
      }
      ++group;
    }
    return KN_OK;
  }

  void run() {
    const kn_status st = loop();
    if (st != KN_OK) {
      std::lock_guard<std::mutex> lk(mu);
      failed = true;
      fail_msg = kn_last_error();
      for (auto& kv : reqs)
        if (kv.second->state == Request::kQueued || kv.second->state == Request::kRunning) {
          kv.second->state = Request::kFailed;
          kv.second->scene->refs--;
        }
      for (auto& q : slots) q = nullptr;
      queue.clear();
      inflight = 0;
      cv_done.notify_all();
    }
  }
};

}  // namespace kn

extern "C" {

kn_status kn_serve_start(kn_ctx* ctx, uint32_t max_inflight, kn_precision precision) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  if (max_inflight < 1 || max_inflight > (uint32_t)kMaxSlots)
    return fail(KN_E_INVALID, "max_inflight %u not in 1..%d", max_inflight, kMaxSlots);
  if (precision != KN_FP32 && precision != KN_BF16 && precision != KN_FP8_E4M3)
    return fail(KN_E_INVALID, "unknown precision %d", (int)precision);
  std::lock_guard<std::mutex> lk(ctx->serve_mu);
  if (ctx->serve) return fail(KN_E_BUSY, "serving loop already running");
  // ray state: what the budget leaves, at most 32 M rays
  const size_t cell_cap = (size_t)1 << 18;
  const size_t fixed = pool_bytes(0, cell_cap, cell_cap + 2);
  // bytes per pool ray, from the pool's own size formula (rounded up)
  const size_t probe = (size_t)1 << 20;
  const size_t per_ray = (pool_bytes(probe, cell_cap, probe / kShadeChunk + cell_cap + 2) - fixed) / probe + 1;
  uint64_t used = ctx->used.load();
  uint64_t avail = ctx->budget > used ? ctx->budget - used : 0;
  if (avail < fixed + probe * per_ray && ctx->ws.ctrl) {
    // the workspace of kn_render is grow-only; its memory goes to the
    // serving pool (the next kn_render allocates a workspace again)
    std::lock_guard<std::mutex> rk(ctx->render_mu);
    KN_HIP(ctx, hipDeviceSynchronize());
    ctx->used -= ctx->ws.bytes;
    free_pool(ctx->ws);
    used = ctx->used.load();
    avail = ctx->budget > used ? ctx->budget - used : 0;
  }
  if (avail < fixed + probe * per_ray) return fail(KN_E_NOMEM, "HBM budget leaves no room for a serving pool");
  const size_t cap = std::min<size_t>((avail - fixed) / per_ray, (size_t)32 << 20);
  std::shared_ptr<kn::ServeLoop> loop(new kn::ServeLoop(ctx, max_inflight, precision));
  st = loop->start(cap, cell_cap);
  if (st != KN_OK) {
    loop->stop();
    return st;
  }
  ctx->serve = std::move(loop);
  return KN_OK;
}

kn_status kn_serve_submit(kn_ctx* ctx, kn_scene_id scene, const kn_camera* cam, const kn_frame* frame,
                          kn_request_id* out) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  if (!out) return fail(KN_E_INVALID, "out is NULL");
  if (!frame || !frame->rgb) return fail(KN_E_INVALID, "frame or frame->rgb is NULL");
  std::lock_guard<std::mutex> sk(ctx->serve_mu);
  if (!ctx->serve) return fail(KN_E_SHUTDOWN, "serving loop not running");
  KnScene* s;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->scenes.find(scene);
    if (it == ctx->scenes.end()) return fail(KN_E_NOT_FOUND, "scene %u not found", scene);
    s = it->second;
    st = validate_camera(cam, s);
    if (st != KN_OK) return st;
    if ((st = validate_frame(frame, cam)) != KN_OK) return st;
    if (cam->bounces != 0) return fail(KN_E_UNSUPPORTED, "the serving loop renders primary rays (bounces 0)");
    if (cam->flags & KN_CAMERA_SPLIT_BF16_SHADING)
      return fail(KN_E_UNSUPPORTED, "the serving loop refines and shades with float32 weights");
    if (cam->flags & KN_CAMERA_UNCLAMPED_STEPS)
      return fail(KN_E_UNSUPPORTED, "the serving loop takes cell-clamped steps");
    if (cam->precision != ctx->serve->precision())
      return fail(KN_E_INVALID, "camera precision %d differs from the serving loop's %d", (int)cam->precision,
                  (int)ctx->serve->precision());
    s->refs++;
  }
  st = ctx->serve->submit(s, cam, frame, out);
  if (st != KN_OK) s->refs--;
  return st;
}

kn_status kn_serve_poll(kn_ctx* ctx, kn_request_id req, int64_t timeout_us, kn_stats* stats_opt) {
  if (!ctx) return fail(KN_E_INVALID, "ctx is NULL");
  std::shared_ptr<kn::ServeLoop> loop;
  {
    std::lock_guard<std::mutex> sk(ctx->serve_mu);
    if (!ctx->serve) return fail(KN_E_SHUTDOWN, "serving loop not running");
    loop = ctx->serve;
  }
  return loop->poll(req, timeout_us, stats_opt);
}

kn_status kn_serve_stop(kn_ctx* ctx) {
  if (!ctx) return fail(KN_E_INVALID, "ctx is NULL");
  std::shared_ptr<kn::ServeLoop> loop;
  {
    std::lock_guard<std::mutex> sk(ctx->serve_mu);
    loop = std::move(ctx->serve);
  }
  if (loop) loop->stop();
  return KN_OK;
}

}  // extern "C"
