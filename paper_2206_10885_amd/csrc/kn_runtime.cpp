// Host runtime of the C ABI (include/kn.h): contexts, scene packing, the
// per-frame round driver, the point query, and the serving loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
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
#include "kn_serve.h"

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

constexpr uint32_t kMarchChunk = 128;   // rays per march work item
constexpr uint32_t kShadeChunk = 64;    // hits per shading work item
constexpr uint32_t kQueryChunk = 256;   // points per query work item

uint16_t bf16_bits(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  const uint32_t r = ((u >> 16) & 1u) + 0x7fffu;
  return (uint16_t)((u + r) >> 16);
}
float bf16_value(float x) {
  uint32_t u = (uint32_t)bf16_bits(x) << 16;
  float y;
  memcpy(&y, &u, 4);
  return y;
}

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
        val = w.W2[(16 * b + m) * H + unit_f32(q, g)];
      }
      out[(s / 4) * 256 + lane * 4 + (s % 4)] = val;
    }
  }
  float* vec = out + 64 * SF;
  for (int j = 0; j < H; ++j) {
    vec[j] = w.b1[j];
    vec[H + j] = w.b2[j];
    vec[2 * H + j] = w.W3[j];
  }
  vec[3 * H] = w.b3[0];
  vec[3 * H + 1] = vec[3 * H + 2] = vec[3 * H + 3] = 0.0f;
}

static void pack_march_bf16(const float* blk, int H, float* out_words) {
  const SdfView w = sdf_view(blk, H);
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
          val = idx < 0 ? 0.0f : w.W1[(16 * b + m) * kSdfIn + idx];
        } else {
          const int f2 = f - F1, b = f2 / (H / 32), c = f2 % (H / 32);
          val = w.W2[(16 * b + m) * H + unit_bf16(c, g, i)];
        }
        out[((size_t)f * 64 + lane) * 8 + i] = bf16_bits(val);
      }
    }
  }
  float* vec = out_words + 64 * 4 * NF;
  for (int j = 0; j < H; ++j) {
    vec[j] = w.b1[j];
    vec[H + j] = w.b2[j];
    vec[2 * H + j] = bf16_value(w.W3[j]);
  }
  vec[3 * H] = w.b3[0];
  vec[3 * H + 1] = vec[3 * H + 2] = vec[3 * H + 3] = 0.0f;
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
  float* shade = nullptr;
  uint32_t march_f32_words = 0, march_bf16_words = 0, shade_words = 0;
  size_t bytes = 0;
  std::atomic<int> refs{0};
};

struct Workspace {
  size_t rays = 0, cells = 0, chunks = 0;
  RayStatic* rs = nullptr;
  RayRec* U = nullptr;
  RayRec* S = nullptr;
  RayRec* HL = nullptr;
  uint32_t* counts = nullptr;      // [2][cells]
  uint32_t* hit_count = nullptr;   // [cells]
  uint32_t* cursor = nullptr;      // [cells]
  uint2* chunk = nullptr;          // [2][chunks]
  uint4* chunk_out = nullptr;      // [2][chunks][2]
  Ctrl* ctrl = nullptr;
  size_t bytes = 0;
};

struct kn_ctx {
  int device = 0;
  int num_cu = 256;
  hipStream_t stream = nullptr;
  uint64_t budget = 0;
  std::atomic<uint64_t> used{0};
  std::mutex mu;              // scenes map
  std::mutex render_mu;       // one render / query at a time on the workspace
  std::map<kn_scene_id, KnScene*> scenes;
  kn_scene_id next_id = 1;
  std::atomic<bool> poisoned{false};
  Workspace ws;
  uint32_t* pinned = nullptr;  // round counters read back by the host
  hipEvent_t ev_start = nullptr, ev_end = nullptr;
  hipEvent_t ev_round[4] = {nullptr, nullptr, nullptr, nullptr};
  int max_passes = 4;          // in-cell passes of a march chunk per round
  std::vector<hipEvent_t> ev_kernel;  // pairs around timed kernel launches
  std::unique_ptr<kn::ServeLoop> serve;
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

void free_ws(Workspace& w) {
  void* ptrs[] = {w.rs, w.U, w.S, w.HL, w.counts, w.hit_count, w.cursor, w.chunk, w.chunk_out, w.ctrl};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  w = Workspace{};
}

// grow-only workspace for `rays` records over `cells` cells; work chunks of
// at least `min_chunk` records
kn_status ensure_ws(kn_ctx* ctx, size_t rays, size_t cells, uint32_t min_chunk) {
  Workspace& w = ctx->ws;
  const size_t chunks = rays / min_chunk + cells + 2;
  if (w.rays >= rays && w.cells >= cells && w.chunks >= chunks && w.ctrl) return KN_OK;
  const size_t R = std::max(w.rays, rays), C = std::max(w.cells, cells),
               K = std::max(w.chunks, chunks);
  const size_t bytes = R * (sizeof(RayStatic) + 3 * sizeof(RayRec)) + C * 4 * 4 + K * 2 * (8 + 32) +
                       sizeof(Ctrl);
  const uint64_t other = ctx->used.load() - w.bytes;
  if (other + bytes > ctx->budget)
    return fail(KN_E_NOMEM, "ray workspace of %zu bytes exceeds the HBM budget", bytes);
  ctx->used -= w.bytes;
  free_ws(w);
  Workspace n;
  n.rays = R;
  n.cells = C;
  n.chunks = K;
  n.bytes = bytes;
  KN_HIP(ctx, hipMalloc(&n.rs, R * sizeof(RayStatic)));
  KN_HIP(ctx, hipMalloc(&n.U, R * sizeof(RayRec)));
  KN_HIP(ctx, hipMalloc(&n.S, R * sizeof(RayRec)));
  KN_HIP(ctx, hipMalloc(&n.HL, R * sizeof(RayRec)));
  KN_HIP(ctx, hipMalloc(&n.counts, 2 * C * 4));
  KN_HIP(ctx, hipMalloc(&n.hit_count, C * 4));
  KN_HIP(ctx, hipMalloc(&n.cursor, C * 4));
  KN_HIP(ctx, hipMalloc(&n.chunk, 2 * K * 8));
  KN_HIP(ctx, hipMalloc(&n.chunk_out, 2 * K * 32));
  KN_HIP(ctx, hipMalloc(&n.ctrl, sizeof(Ctrl)));
  w = n;
  ctx->used += bytes;
  return KN_OK;
}

SoftplusK softplus_consts(float beta) {
  return SoftplusK{(float)(-(double)beta / std::log(2.0)), (float)(std::log(2.0) / (double)beta)};
}

uint32_t persistent_grid(kn_ctx* ctx, uint32_t per_cu) { return (uint32_t)ctx->num_cu * per_cu; }

}  // namespace

extern "C" {

const char* kn_last_error(void) { return g_err.c_str(); }

kn_status kn_ctx_create(int hip_device, uint64_t hbm_budget_bytes, kn_ctx** out) {
  if (!out) return fail(KN_E_INVALID, "out is NULL");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(KN_E_DEVICE, "no HIP device");
  if (hip_device < 0 || hip_device >= n) return fail(KN_E_INVALID, "device %d out of range", hip_device);
  std::unique_ptr<kn_ctx> ctx(new kn_ctx());
  ctx->device = hip_device;
  KN_HIP(ctx, hipSetDevice(hip_device));
  hipDeviceProp_t prop;
  KN_HIP(ctx, hipGetDeviceProperties(&prop, hip_device));
  ctx->num_cu = prop.multiProcessorCount;
  size_t freeb = 0, total = 0;
  KN_HIP(ctx, hipMemGetInfo(&freeb, &total));
  ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)freeb);
  KN_HIP(ctx, hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
  KN_HIP(ctx, hipHostMalloc((void**)&ctx->pinned, 64 * sizeof(uint32_t), hipHostMallocDefault));
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
  for (auto& kv : ctx->scenes) {
    KnScene* s = kv.second;
    if (s->march_f32) (void)hipFree(s->march_f32);
    if (s->march_bf16) (void)hipFree(s->march_bf16);
    if (s->shade) (void)hipFree(s->shade);
    delete s;
  }
  free_ws(ctx->ws);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->ev_start) (void)hipEventDestroy(ctx->ev_start);
  if (ctx->ev_end) (void)hipEventDestroy(ctx->ev_end);
  for (auto& e : ctx->ev_round)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->ev_kernel) (void)hipEventDestroy(e);
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
  if (d->precisions & (1u << KN_FP8_E4M3))
    return fail(KN_E_UNSUPPORTED, "fp8 scene copies are not built yet");

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
  s->march_f32_words = (uint32_t)march_block_words(H, 0);
  s->march_bf16_words = (uint32_t)march_block_words(H, 1);
  s->shade_words = (uint32_t)shade_block_words(H);
  const bool want_bf16 = (d->precisions >> KN_BF16) & 1u;
  const size_t bytes = cells * 4 * ((size_t)s->march_f32_words + s->shade_words +
                                    (want_bf16 ? s->march_bf16_words : 0));
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
    st = upload(&s->march_bf16, s->march_bf16_words,
                [&](size_t c, float* o) { pack_march_bf16(d->sdf_params + c * psdf, H, o); });
    if (st != KN_OK) return st;
  }
  st = upload(&s->shade, s->shade_words, [&](size_t c, float* o) {
    pack_shade(d->sdf_params + c * psdf, d->col_params + c * pcol, H, o);
  });
  if (st != KN_OK) return st;
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
  std::lock_guard<std::mutex> rk(ctx->render_mu);
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (s->march_f32) (void)hipFree(s->march_f32);
  if (s->march_bf16) (void)hipFree(s->march_bf16);
  if (s->shade) (void)hipFree(s->shade);
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

kn_status validate_camera(const kn_camera* c, const KnScene* s) {
  if (!c) return fail(KN_E_INVALID, "camera is NULL");
  if (c->width == 0 || c->height == 0) return fail(KN_E_INVALID, "empty image %ux%u", c->width, c->height);
  if ((uint64_t)c->width * c->height > (1ull << 28))
    return fail(KN_E_INVALID, "image %ux%u too large", c->width, c->height);
  if (c->max_steps < 1 || c->max_steps > (uint32_t)kMaxSteps)
    return fail(KN_E_INVALID, "max_steps %u not in 1..%d", c->max_steps, kMaxSteps);
  if (!(c->eps > 0.0f) || !std::isfinite(c->eps)) return fail(KN_E_INVALID, "eps must be positive");
  if (c->spp != 1 || c->bounces != 0)
    return fail(KN_E_UNSUPPORTED, "only spp = 1 primary casts are implemented (spp %u, bounces %u)",
                c->spp, c->bounces);
  if (c->precision == KN_BF16 && !s->march_bf16)
    return fail(KN_E_INVALID, "scene has no bf16 copy (set precisions bit KN_BF16)");
  if (c->precision != KN_FP32 && c->precision != KN_BF16)
    return fail(KN_E_UNSUPPORTED, "precision %d not available", (int)c->precision);
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

}  // namespace

namespace kn {

// Enqueues and runs one frame on `stream`; the caller holds render_mu.
kn_status render_frame(kn_ctx* ctx, KnScene* s, const kn_camera* c, const kn_frame* fr,
                       hipStream_t stream, kn_stats* stats) {
  const auto wall0 = std::chrono::steady_clock::now();
  const size_t rays = (size_t)c->width * c->height;
  const size_t cells = (size_t)s->N * s->N * s->N;
  kn_status st = ensure_ws(ctx, rays, cells, std::min(kMarchChunk, kShadeChunk));
  if (st != KN_OK) return st;
  Workspace& w = ctx->ws;
  OutPtrs out{fr->rgb, fr->depth, fr->normal, fr->hit, fr->steps,
              reinterpret_cast<TraceRec*>(fr->trace), {0.0f, 0.0f, 0.0f}};
  const bool bf = c->precision == KN_BF16;
  const SoftplusK spk = softplus_consts(s->geom.beta);

  const bool timed = stats && stats->kernel_times;
  const size_t need_ev = 2 * ((size_t)c->max_steps + 3);
  while (timed && ctx->ev_kernel.size() < need_ev) {
    hipEvent_t e;
    KN_HIP(ctx, hipEventCreate(&e));
    ctx->ev_kernel.push_back(e);
  }
  KN_HIP(ctx, hipEventRecord(ctx->ev_start, stream));
  KN_HIP(ctx, hipMemsetAsync(w.ctrl, 0, sizeof(Ctrl), stream));
  KN_HIP(ctx, hipMemsetAsync(w.counts, 0, 2 * cells * 4, stream));
  KN_HIP(ctx, hipMemsetAsync(w.hit_count, 0, cells * 4, stream));
  KN_HIP(ctx, hipMemsetAsync(w.HL, 0xFF, rays * sizeof(RayRec), stream));

  RaygenArgs rg{};
  rg.sg = s->geom;
  camera_basis(c, rg);
  rg.W = (int)c->width;
  rg.Hh = (int)c->height;
  rg.rs = w.rs;
  rg.U = w.U;
  rg.counts = w.counts;
  rg.out = out;
  KN_HIP(ctx, launch_raygen(rg, stream));

  const uint32_t scatter_grid = (uint32_t)std::min<size_t>((rays + 255) / 256, 4096);
  const uint32_t march_grid = persistent_grid(ctx, 4);
  // every round takes at least one SDF evaluation of every live ray
  const int max_rounds = (int)c->max_steps + 2;
  int rounds = 0;
  for (int r = 0; r < max_rounds; ++r) {
    const int par = r & 1;
    uint2* chunks = w.chunk + (size_t)par * w.chunks;
    uint4* chunk_out = w.chunk_out + (size_t)par * w.chunks * 2;
    ScanArgs sa{};
    sa.counts = w.counts + par * cells;
    sa.C = (uint32_t)cells;
    sa.T = kChunk;
    sa.zero_counts = 1;
    sa.cursor = w.cursor;
    sa.chunks = chunks;
    sa.n_chunks = &w.ctrl->n_chunks[par];
    sa.grab = w.ctrl->grab;
    sa.grab0 = w.ctrl->grab0;
    sa.zero_word = nullptr;
    KN_HIP(ctx, launch_scan(sa, stream));
    if (r == 0) {
      ScatterArgs sc{w.U, w.S, (uint32_t)rays, w.cursor};
      KN_HIP(ctx, launch_scatter(sc, scatter_grid, stream));
    } else {
      ScatterChunksArgs sc{s->geom,
                           w.chunk + (size_t)(par ^ 1) * w.chunks,
                           w.chunk_out + (size_t)(par ^ 1) * w.chunks * 2,
                           &w.ctrl->n_chunks[par ^ 1],
                           w.U,
                           w.S,
                           w.cursor};
      KN_HIP(ctx, launch_scatter_chunks(sc, persistent_grid(ctx, 4), stream));
    }
    MarchArgs ma{};
    ma.sg = s->geom;
    ma.blocks = bf ? s->march_bf16 : s->march_f32;
    ma.block_words = bf ? s->march_bf16_words : s->march_f32_words;
    ma.S = w.S;
    ma.rs = w.rs;
    ma.chunks = chunks;
    ma.n_chunks = &w.ctrl->n_chunks[par];
    ma.grab = w.ctrl->grab;
    ma.chunk_out = chunk_out;
    ma.U = w.U;
    ma.counts_next = w.counts + (par ^ 1) * cells;
    ma.HL = w.HL;
    ma.hit_count = w.hit_count;
    ma.evals = &w.ctrl->evals;
    ma.max_steps = (int)c->max_steps;
    ma.max_passes = ctx->max_passes;
    ma.eps = c->eps;
    ma.spk = spk;
    ma.out = out;
    if (timed) KN_HIP(ctx, hipEventRecord(ctx->ev_kernel[2 * r], stream));
    KN_HIP(ctx, launch_march(ma, s->H, bf ? 1 : 0, march_grid, stream));
    if (timed) KN_HIP(ctx, hipEventRecord(ctx->ev_kernel[2 * r + 1], stream));
    ++rounds;
    // every kReadback rounds, read back how many chunks the round had; stop
    // once an earlier readback shows an empty round (rounds enqueued after
    // it find no work and return at once)
    constexpr int kReadback = 4;
    if (r % kReadback == kReadback - 1) {
      const int slot = (r / kReadback) & 3;
      KN_HIP(ctx, hipMemcpyAsync(&ctx->pinned[slot], &w.ctrl->n_chunks[par], 4, hipMemcpyDeviceToHost,
                                 stream));
      KN_HIP(ctx, hipEventRecord(ctx->ev_round[slot], stream));
      if (r >= 2 * kReadback - 1) {
        const int prev = ((r / kReadback) - 1) & 3;
        KN_HIP(ctx, hipEventSynchronize(ctx->ev_round[prev]));
        if (ctx->pinned[prev] == 0) break;
      }
    }
  }

  // shade the hits, binned by cell
  {
    ScanArgs sa{};
    sa.counts = w.hit_count;
    sa.C = (uint32_t)cells;
    sa.T = kShadeChunk;
    sa.zero_counts = 0;
    sa.cursor = w.cursor;
    sa.chunks = w.chunk;
    sa.n_chunks = &w.ctrl->n_chunks[2];
    sa.grab = w.ctrl->grab;
    sa.grab0 = w.ctrl->grab0;
    sa.zero_word = nullptr;
    sa.total = &w.ctrl->n_hits;
    KN_HIP(ctx, launch_scan(sa, stream));
    ScatterArgs sc{w.HL, w.S, (uint32_t)rays, w.cursor};
    KN_HIP(ctx, launch_scatter(sc, scatter_grid, stream));
    ShadeArgs sh{};
    sh.sg = s->geom;
    sh.blocks = s->shade;
    sh.block_words = s->shade_words;
    sh.S = w.S;
    sh.rs = w.rs;
    sh.chunks = w.chunk;
    sh.n_chunks = &w.ctrl->n_chunks[2];
    sh.grab = w.ctrl->grab;
    sh.spk = spk;
    sh.out = out;
    if (timed) KN_HIP(ctx, hipEventRecord(ctx->ev_kernel[need_ev - 2], stream));
    KN_HIP(ctx, launch_shade(sh, s->H, persistent_grid(ctx, 2), stream));
    if (timed) KN_HIP(ctx, hipEventRecord(ctx->ev_kernel[need_ev - 1], stream));
  }
  KN_HIP(ctx, hipEventRecord(ctx->ev_end, stream));
  KN_HIP(ctx, hipEventSynchronize(ctx->ev_end));
  if (stats) {
    Ctrl hc;
    KN_HIP(ctx, hipMemcpy(&hc, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    float ms = 0.0f;
    KN_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_end));
    stats->gpu_ms = ms;
    stats->wall_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0).count();
    stats->rays = rays;
    stats->evals = hc.evals;
    stats->march_tiles = hc.tiles;
    stats->march_chunks = hc.chunks;
    stats->hits = hc.n_hits;
    stats->rounds = (uint64_t)rounds;
    stats->march_launches = 0;
    stats->march_ms = stats->shade_ms = 0.0;
    if (timed) {
      for (int r = 0; r < rounds; ++r) {
        float kms = 0.0f;
        KN_HIP(ctx, hipEventElapsedTime(&kms, ctx->ev_kernel[2 * r], ctx->ev_kernel[2 * r + 1]));
        stats->march_ms += kms;
      }
      stats->march_launches = (uint32_t)rounds;
      float kms = 0.0f;
      KN_HIP(ctx, hipEventElapsedTime(&kms, ctx->ev_kernel[need_ev - 2], ctx->ev_kernel[need_ev - 1]));
      stats->shade_ms = kms;
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
  if (!frame || !frame->rgb) return fail(KN_E_INVALID, "frame or frame->rgb is NULL");
  if (cam->env_rgb) return fail(KN_E_UNSUPPORTED, "environment maps are used by path tracing only");
  std::lock_guard<std::mutex> lk(ctx->render_mu);
  KN_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t stream = frame->hip_stream ? (hipStream_t)frame->hip_stream : ctx->stream;
  s->refs++;
  st = render_frame(ctx, s, cam, frame, stream, stats);
  s->refs--;
  return st;
}

kn_status kn_query(kn_ctx* ctx, kn_scene_id scene, kn_precision precision, const float* points,
                   uint64_t n, float* d_out, float* grad_out, float* z_out, void* hip_stream) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  KnScene* s = find_scene(ctx, scene);
  if (!s) return fail(KN_E_NOT_FOUND, "scene %u not found", scene);
  if (n == 0) return KN_OK;
  if (!points) return fail(KN_E_INVALID, "points is NULL");
  if (n > (1ull << 28)) return fail(KN_E_INVALID, "too many points (%llu)", (unsigned long long)n);
  if (precision != KN_FP32 && precision != KN_BF16)
    return fail(KN_E_UNSUPPORTED, "precision %d not available", (int)precision);
  if (precision == KN_BF16 && !s->march_bf16) return fail(KN_E_INVALID, "scene has no bf16 copy");
  std::lock_guard<std::mutex> lk(ctx->render_mu);
  KN_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t stream = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
  const size_t cells = (size_t)s->N * s->N * s->N;
  st = ensure_ws(ctx, n, cells, 16);
  if (st != KN_OK) return st;
  Workspace& w = ctx->ws;
  const SoftplusK spk = softplus_consts(s->geom.beta);
  KN_HIP(ctx, hipMemsetAsync(w.ctrl, 0, sizeof(Ctrl), stream));
  KN_HIP(ctx, hipMemsetAsync(w.counts, 0, cells * 4, stream));
  QueryBinArgs qb{s->geom, points, n, w.U, w.counts};
  KN_HIP(ctx, launch_query_bin(qb, stream));
  ScanArgs sa{};
  sa.counts = w.counts;
  sa.C = (uint32_t)cells;
  sa.T = kQueryChunk;
  sa.zero_counts = 0;
  sa.cursor = w.cursor;
  sa.chunks = w.chunk;
  sa.n_chunks = &w.ctrl->n_chunks[0];
  sa.grab = w.ctrl->grab;
    sa.grab0 = w.ctrl->grab0;
  sa.zero_word = nullptr;
  KN_HIP(ctx, launch_scan(sa, stream));
  ScatterArgs sc{w.U, w.S, (uint32_t)n, w.cursor};
  KN_HIP(ctx, launch_scatter(sc, (uint32_t)std::min<uint64_t>((n + 255) / 256, 4096), stream));
  QueryArgs qa{};
  qa.sg = s->geom;
  qa.S = w.S;
  qa.pts = points;
  qa.chunks = w.chunk;
  qa.n_chunks = &w.ctrl->n_chunks[0];
  qa.grab = w.ctrl->grab;
  qa.spk = spk;
  if (d_out) {
    const bool bf = precision == KN_BF16;
    qa.blocks = bf ? s->march_bf16 : s->march_f32;
    qa.block_words = bf ? s->march_bf16_words : s->march_f32_words;
    qa.d_out = d_out;
    KN_HIP(ctx, launch_query_d(qa, s->H, bf ? 1 : 0, persistent_grid(ctx, 2), stream));
  }
  if (grad_out || z_out) {
    KN_HIP(ctx, hipMemcpyAsync(w.ctrl->grab, w.ctrl->grab0, sizeof(w.ctrl->grab), hipMemcpyDeviceToDevice,
                               stream));
    qa.blocks = s->shade;
    qa.block_words = s->shade_words;
    qa.d_out = nullptr;
    qa.grad_out = grad_out;
    qa.z_out = z_out;
    KN_HIP(ctx, launch_query_full(qa, s->H, persistent_grid(ctx, 2), stream));
  }
  KN_HIP(ctx, hipStreamSynchronize(stream));
  return KN_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// serving (continuous batching) -- not built yet
// ---------------------------------------------------------------------------
namespace kn {
class ServeLoop {};
}  // namespace kn

extern "C" {

kn_status kn_serve_start(kn_ctx* ctx, uint32_t, kn_precision) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  return fail(KN_E_UNSUPPORTED, "serving loop not built yet");
}
kn_status kn_serve_submit(kn_ctx* ctx, kn_scene_id, const kn_camera*, const kn_frame*, kn_request_id*) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  return fail(KN_E_SHUTDOWN, "serving loop not running");
}
kn_status kn_serve_poll(kn_ctx* ctx, kn_request_id, int64_t, kn_stats*) {
  kn_status st = check_ctx(ctx);
  if (st != KN_OK) return st;
  return fail(KN_E_SHUTDOWN, "serving loop not running");
}
kn_status kn_serve_stop(kn_ctx* ctx) {
  if (!ctx) return fail(KN_E_INVALID, "ctx is NULL");
  ctx->serve.reset();
  return KN_OK;
}

}  // extern "C"
