// Host runtime of the C ABI (kn_runtime.cpp) driven on the CPU against the
// host-only HIP stand-in, built with the address and undefined-behaviour
// sanitizers: scene creation and packing at several grid and MLP sizes in
// every precision, argument validation, frames, point queries and the serving
// loop, and the treatment of the scan's look-back overrun flag.  Each check
// prints one line; any failure, sanitizer report or leak ends the process
// with a non-zero status.  Usage: driver <case>.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "kn.h"

namespace {

int g_fail = 0;

void expect(bool ok, const char* what) {
  std::printf("%s %s\n", ok ? "ok  " : "FAIL", what);
  if (!ok) ++g_fail;
}

// scene parameters: any finite values do for the host runtime
struct HostScene {
  uint32_t N, H;
  std::vector<float> sdf, col;
};

HostScene make_scene(uint32_t N, uint32_t H, uint32_t seed) {
  HostScene s{N, H, {}, {}};
  const size_t cells = (size_t)N * N * N;
  const size_t psdf = 39 * H + H + H * H + H + 16 * H + 16, pcol = 48 * 32 + 32 + 3 * 32 + 3;
  s.sdf.resize(cells * psdf);
  s.col.resize(cells * pcol);
  uint32_t x = seed * 2654435761u + 1u;
  auto next = [&x]() {
    x = x * 1664525u + 1013904223u;
    return (float)(x >> 8) / 16777216.0f - 0.5f;
  };
  for (float& v : s.sdf) v = next();
  for (float& v : s.col) v = next();
  return s;
}

kn_scene_desc desc_of(const HostScene& s, uint32_t precisions) {
  kn_scene_desc d{};
  d.abi_version = KN_ABI_VERSION;
  d.grid_n = s.N;
  for (int k = 0; k < 3; ++k) {
    d.bbox_min[k] = -1.0f;
    d.bbox_max[k] = 1.0f;
  }
  d.pos_freqs = 6;
  d.dir_freqs = 4;
  d.sdf_hidden = s.H;
  d.sdf_layers = 2;
  d.feat_dim = 15;
  d.col_hidden = 32;
  d.col_layers = 1;
  d.col_in_has_x = 1;
  d.softplus_beta = 100.0f;
  d.sdf_params = s.sdf.data();
  d.col_params = s.col.data();
  d.precisions = precisions;
  return d;
}

kn_camera camera(uint32_t W, uint32_t H, kn_precision p) {
  kn_camera c{};
  c.eye[2] = 2.5f;
  c.up[1] = 1.0f;
  c.width = W;
  c.height = H;
  c.spp = 1;
  c.max_steps = 64;
  c.eps = 1e-4f;
  c.precision = p;
  return c;
}

struct DevFrame {
  kn_frame f{};
  explicit DevFrame(size_t npix) {
    (void)hipMalloc((void**)&f.rgb, npix * 12);
    (void)hipMalloc((void**)&f.depth, npix * 4);
    (void)hipMalloc((void**)&f.normal, npix * 12);
    (void)hipMalloc((void**)&f.hit, npix);
    (void)hipMalloc((void**)&f.steps, npix * 2);
  }
  ~DevFrame() {
    (void)hipFree(f.rgb);
    (void)hipFree(f.depth);
    (void)hipFree(f.normal);
    (void)hipFree(f.hit);
    (void)hipFree(f.steps);
  }
};

const uint32_t kAll = (1u << KN_BF16) | (1u << KN_FP8_E4M3);

void case_scenes() {
  kn_ctx* ctx = nullptr;
  expect(kn_ctx_create(0, 0, &ctx) == KN_OK, "ctx create");
  const uint32_t sizes[][2] = {{1, 32}, {1, 64}, {3, 32}, {4, 64}, {8, 64}, {16, 32}, {12, 64}};
  for (auto& nh : sizes) {
    HostScene s = make_scene(nh[0], nh[1], nh[0] * 100 + nh[1]);
    for (uint32_t prec : {0u, 1u << KN_BF16, 1u << KN_FP8_E4M3, kAll}) {
      kn_scene_desc d = desc_of(s, prec);
      kn_scene_id id = 0;
      char what[96];
      std::snprintf(what, sizeof what, "scene N=%u H=%u precisions=%u created", nh[0], nh[1], prec);
      expect(kn_scene_create(ctx, &d, &id) == KN_OK, what);
      std::snprintf(what, sizeof what, "scene N=%u H=%u precisions=%u destroyed", nh[0], nh[1], prec);
      expect(kn_scene_destroy(ctx, id) == KN_OK, what);
    }
  }
  // a scene left for kn_ctx_destroy to free (every resident copy)
  HostScene s = make_scene(4, 64, 7);
  kn_scene_desc d = desc_of(s, kAll);
  kn_scene_id id = 0;
  expect(kn_scene_create(ctx, &d, &id) == KN_OK, "scene kept until the context is destroyed");
  expect(kn_ctx_destroy(ctx) == KN_OK, "ctx destroy frees the remaining scene");
}

void case_validation() {
  kn_ctx* ctx = nullptr;
  expect(kn_ctx_create(0, 0, &ctx) == KN_OK, "ctx create");
  HostScene s = make_scene(2, 32, 3);
  kn_scene_id id = 0;
  kn_scene_desc d = desc_of(s, kAll);
  d.grid_n = 0;
  expect(kn_scene_create(ctx, &d, &id) == KN_E_UNSUPPORTED, "grid_n 0 unsupported");
  d = desc_of(s, kAll);
  d.sdf_hidden = 48;
  expect(kn_scene_create(ctx, &d, &id) == KN_E_UNSUPPORTED, "sdf_hidden 48 unsupported");
  d = desc_of(s, kAll);
  d.abi_version = 99;
  expect(kn_scene_create(ctx, &d, &id) == KN_E_INVALID, "wrong abi_version");
  d = desc_of(s, 1u << 5);
  expect(kn_scene_create(ctx, &d, &id) == KN_E_INVALID, "unknown precision bit");
  s.sdf[s.sdf.size() - 1] = NAN;
  d = desc_of(s, kAll);
  expect(kn_scene_create(ctx, &d, &id) == KN_E_INVALID, "NaN in the last SDF parameter");
  expect(std::strstr(kn_last_error(), "non-finite") != nullptr, "message names the parameter");
  expect(kn_ctx_destroy(ctx) == KN_OK, "ctx destroy");
}

void case_render_query(bool scan_err) {
  kn_ctx* ctx = nullptr;
  expect(kn_ctx_create(0, 0, &ctx) == KN_OK, "ctx create");
  HostScene s = make_scene(4, 32, 11);
  kn_scene_desc d = desc_of(s, kAll);
  kn_scene_id id = 0;
  expect(kn_scene_create(ctx, &d, &id) == KN_OK, "scene create");
  const kn_status want = scan_err ? KN_E_DEVICE : KN_OK;
  for (kn_precision p : {KN_FP32, KN_BF16, KN_FP8_E4M3}) {
    DevFrame fr(97 * 61);
    kn_camera c = camera(97, 61, p);
    kn_stats st{};
    const kn_status r = kn_render(ctx, id, &c, &fr.f, (p == KN_BF16) ? &st : nullptr);
    expect(r == want, scan_err ? "render reports the scan overrun" : "render");
    if (scan_err) {
      expect(kn_render(ctx, id, &c, &fr.f, nullptr) == KN_E_DEVICE, "context poisoned afterwards");
      break;
    }
  }
  if (!scan_err) {
    DevFrame fr(64 * 48);
    kn_camera c = camera(64, 48, KN_BF16);
    c.bounces = 3;
    c.spp = 4;
    expect(kn_render(ctx, id, &c, &fr.f, nullptr) == KN_OK, "path-traced render");
    c.flags = KN_CAMERA_UNCLAMPED_STEPS;
    expect(kn_render(ctx, id, &c, &fr.f, nullptr) == KN_OK, "path-traced render, unclamped steps");
    kn_camera cu = camera(64, 48, KN_FP32);
    cu.flags = KN_CAMERA_UNCLAMPED_STEPS;
    expect(kn_render(ctx, id, &cu, &fr.f, nullptr) == KN_OK, "render, unclamped steps");
    cu.flags = 4u;
    expect(kn_render(ctx, id, &cu, &fr.f, nullptr) == KN_E_INVALID, "unknown camera flag refused");
    float* pts = nullptr;
    float *dd = nullptr, *gg = nullptr, *zz = nullptr;
    const uint64_t n = 5000;
    (void)hipMalloc((void**)&pts, n * 12);
    (void)hipMalloc((void**)&dd, n * 4);
    (void)hipMalloc((void**)&gg, n * 12);
    (void)hipMalloc((void**)&zz, n * 60);
    expect(kn_query(ctx, id, KN_BF16, pts, n, dd, gg, zz, nullptr) == KN_OK, "query");
    (void)hipFree(pts);
    (void)hipFree(dd);
    (void)hipFree(gg);
    (void)hipFree(zz);
  }
  kn_scene_destroy(ctx, id);
  expect(kn_ctx_destroy(ctx) == KN_OK, "ctx destroy");
}

void case_noalloc() {
  kn_ctx* ctx = nullptr;
  expect(kn_ctx_create(0, 0, &ctx) == KN_OK, "ctx create");
  HostScene s = make_scene(16, 64, 13);
  kn_scene_desc d = desc_of(s, kAll);
  kn_scene_id id = 0;
  expect(kn_scene_create(ctx, &d, &id) == KN_OK, "scene create");
  const uint64_t nmax = 1u << 18;
  float *pts = nullptr, *dd = nullptr, *gg = nullptr, *zz = nullptr;
  (void)hipMalloc((void**)&pts, (nmax + 1) * 12);
  (void)hipMalloc((void**)&dd, (nmax + 1) * 4);
  (void)hipMalloc((void**)&gg, (nmax + 1) * 12);
  (void)hipMalloc((void**)&zz, (nmax + 1) * 60);
  for (kn_precision p : {KN_FP32, KN_BF16, KN_FP8_E4M3})
    expect(kn_query_noalloc(ctx, id, p, pts, nmax, dd, gg, zz, nullptr) == KN_OK, "no-alloc query at the limit");
  expect(kn_query_noalloc(ctx, id, KN_BF16, pts, 333, dd, nullptr, nullptr, nullptr) == KN_OK,
         "no-alloc query, small");
  expect(kn_query_noalloc(ctx, id, KN_BF16, pts, nmax + 1, dd, nullptr, nullptr, nullptr) == KN_E_INVALID,
         "no-alloc query above the limit");
  expect(std::strstr(kn_last_error(), "limit") != nullptr, "message names the limit");
  (void)hipFree(pts);
  (void)hipFree(dd);
  (void)hipFree(gg);
  (void)hipFree(zz);
  expect(kn_ctx_destroy(ctx) == KN_OK, "ctx destroy");
}

void case_grid_eikonal() {
  kn_ctx* ctx = nullptr;
  expect(kn_ctx_create(0, 0, &ctx) == KN_OK, "ctx create");
  HostScene s = make_scene(4, 32, 14);
  kn_scene_desc d = desc_of(s, kAll);
  kn_scene_id id = 0;
  expect(kn_scene_create(ctx, &d, &id) == KN_OK, "scene create");
  const uint32_t R = 37;
  float *dd = nullptr, *gg = nullptr;
  (void)hipMalloc((void**)&dd, (size_t)R * R * R * 4);
  (void)hipMalloc((void**)&gg, (size_t)R * R * R * 12);
  for (kn_precision p : {KN_FP32, KN_BF16, KN_FP8_E4M3})
    expect(kn_grid_sample(ctx, id, p, R, dd, nullptr, nullptr) == KN_OK, "lattice values");
  expect(kn_grid_sample(ctx, id, KN_FP32, R, dd, gg, nullptr) == KN_OK, "lattice gradients");
  expect(kn_grid_sample(ctx, id, KN_BF16, R, dd, gg, nullptr) == KN_E_INVALID, "bf16 gradients refused");
  expect(kn_grid_sample(ctx, id, KN_FP32, 1, dd, nullptr, nullptr) == KN_E_INVALID, "R = 1 refused");
  expect(kn_grid_sample(ctx, id, KN_FP32, R, nullptr, nullptr, nullptr) == KN_E_INVALID, "NULL d_out refused");
  const uint64_t n = 3000;
  float *pts = nullptr, *gn = nullptr, *st = nullptr;
  double* loss = nullptr;
  (void)hipMalloc((void**)&pts, 2 * n * 12);
  (void)hipMalloc((void**)&gn, 2 * n * 4);
  (void)hipMalloc((void**)&st, n * 24);
  (void)hipMalloc((void**)&loss, 8);
  for (kn_precision p : {KN_FP32, KN_BF16, KN_FP8_E4M3})
    expect(kn_eikonal_fd(ctx, id, p, pts, n, 1e-3f, gn, st, loss, nullptr) == KN_OK, "eikonal");
  expect(kn_eikonal_fd(ctx, id, KN_FP32, pts, n, 1e-3f, gn, nullptr, nullptr, nullptr) == KN_OK,
         "eikonal without stencil or loss");
  expect(kn_eikonal_fd(ctx, id, KN_FP32, pts, 2 * n, 1e-3f, gn, nullptr, nullptr, nullptr) == KN_OK,
         "eikonal, work buffer grown");
  expect(kn_eikonal_fd(ctx, id, KN_FP32, pts, n, 0.0f, gn, nullptr, nullptr, nullptr) == KN_E_INVALID,
         "delta 0 refused");
  expect(kn_eikonal_fd(ctx, id, KN_FP32, pts, n, 1e-3f, nullptr, nullptr, nullptr, nullptr) == KN_E_INVALID,
         "NULL gnorm refused");
  (void)hipFree(dd);
  (void)hipFree(gg);
  (void)hipFree(pts);
  (void)hipFree(gn);
  (void)hipFree(st);
  (void)hipFree(loss);
  kn_scene_destroy(ctx, id);
  expect(kn_ctx_destroy(ctx) == KN_OK, "ctx destroy");
}

void case_world() {
  kn_ctx* ctx = nullptr;
  expect(kn_ctx_create(0, (uint64_t)1 << 30, &ctx) == KN_OK, "ctx create");
  HostScene s1 = make_scene(4, 64, 31), s2 = make_scene(8, 32, 32);
  kn_scene_desc d1 = desc_of(s1, kAll), d2 = desc_of(s2, 1u << KN_BF16);
  kn_scene_id a = 0, b = 0;
  expect(kn_scene_create(ctx, &d1, &a) == KN_OK && kn_scene_create(ctx, &d2, &b) == KN_OK, "scenes create");
  kn_instance inst[3] = {{a, {0.0f, 0.0f, 0.0f}, 1.0f}, {b, {3.0f, 0.0f, 0.0f}, 0.5f}, {a, {0.0f, 0.0f, -4.0f}, 2.0f}};
  kn_primitive prim[3] = {{KN_PRIM_SPHERE, {0.0f, -3.0f, 0.0f, 1.0f}, {0.5f, 0.5f, 0.5f}},
                          {KN_PRIM_BOX, {-5.0f, -6.0f, -5.0f, 5.0f, -5.0f, 5.0f}, {0.8f, 0.7f, 0.6f}},
                          {KN_PRIM_TRIANGLE, {0.0f, 3.0f, 0.0f, 1.0f, 3.0f, 0.0f, 0.0f, 4.0f, 0.0f}, {1.0f, 0.0f, 0.0f}}};
  kn_world_desc wd{3, inst, 3, prim};
  kn_world_id w = 0;
  expect(kn_world_create(ctx, &wd, &w) == KN_OK, "world create (3 instances, 3 primitives)");
  expect(kn_scene_destroy(ctx, a) == KN_E_BUSY, "scene placed in a world is busy");
  DevFrame fr(97 * 61);
  for (kn_precision p : {KN_FP32, KN_BF16}) {
    kn_camera c = camera(97, 61, p);
    c.eye[2] = 9.0f;
    kn_stats st{};
    expect(kn_render_world(ctx, w, &c, &fr.f, &st) == KN_OK, "world render");
  }
  kn_camera c8 = camera(97, 61, KN_FP8_E4M3);
  expect(kn_render_world(ctx, w, &c8, &fr.f, nullptr) == KN_E_INVALID, "instance without an fp8 copy refused");
  float* acc = nullptr;
  (void)hipMalloc((void**)&acc, 97 * 61 * 12);
  kn_camera cp = camera(97, 61, KN_BF16);
  cp.bounces = 2;
  cp.spp = 2;
  fr.f.accum = acc;
  expect(kn_render_world(ctx, w, &cp, &fr.f, nullptr) == KN_OK, "path-traced world render with accumulation");
  cp.sample_offset = 2;
  expect(kn_render_world(ctx, w, &cp, &fr.f, nullptr) == KN_OK, "accumulation, second call");
  expect(kn_render(ctx, a, &cp, &fr.f, nullptr) == KN_OK, "single-scene render with accumulation");
  kn_camera c0 = camera(97, 61, KN_BF16);
  expect(kn_render(ctx, a, &c0, &fr.f, nullptr) == KN_E_UNSUPPORTED, "accumulation without path tracing refused");
  fr.f.accum = nullptr;
  c0.sample_offset = 3;
  expect(kn_render(ctx, a, &c0, &fr.f, nullptr) == KN_E_INVALID, "sample_offset without path tracing refused");
  (void)hipFree(acc);
  kn_camera cu = camera(33, 17, KN_BF16);
  cu.flags = KN_CAMERA_UNCLAMPED_STEPS;
  expect(kn_render_world(ctx, w, &cu, &fr.f, nullptr) == KN_E_UNSUPPORTED,
         "unclamped steps in a world of mixed widths refused");
  expect(kn_render_world(ctx, w + 77, &cu, &fr.f, nullptr) == KN_E_NOT_FOUND, "unknown world");
  // validation
  kn_instance ov[2] = {{a, {0.0f, 0.0f, 0.0f}, 1.0f}, {b, {1.5f, 0.0f, 0.0f}, 1.0f}};
  kn_world_desc bad{2, ov, 0, nullptr};
  kn_world_id wx = 0;
  expect(kn_world_create(ctx, &bad, &wx) == KN_E_INVALID, "overlapping instance boxes refused");
  kn_instance sc0[1] = {{a, {0.0f, 0.0f, 0.0f}, 0.0f}};
  bad = kn_world_desc{1, sc0, 0, nullptr};
  expect(kn_world_create(ctx, &bad, &wx) == KN_E_INVALID, "zero scale refused");
  kn_instance nf[1] = {{a + 99, {0.0f, 0.0f, 0.0f}, 1.0f}};
  bad = kn_world_desc{1, nf, 0, nullptr};
  expect(kn_world_create(ctx, &bad, &wx) == KN_E_NOT_FOUND, "unknown scene refused");
  kn_primitive bp[4] = {{KN_PRIM_SPHERE, {0.0f, 0.0f, 0.0f, -1.0f}, {0.5f, 0.5f, 0.5f}},
                        {KN_PRIM_BOX, {0.0f, 0.0f, 0.0f, 1.0f, 0.0f, 1.0f}, {0.5f, 0.5f, 0.5f}},
                        {KN_PRIM_TRIANGLE, {0.0f, 0.0f, 0.0f, 1.0f, 1.0f, 1.0f, 2.0f, 2.0f, 2.0f}, {0.5f, 0.5f, 0.5f}},
                        {KN_PRIM_SPHERE, {0.0f, 0.0f, 0.0f, 1.0f}, {1.5f, 0.5f, 0.5f}}};
  for (int i = 0; i < 4; ++i) {
    bad = kn_world_desc{0, nullptr, 1, bp + i};
    expect(kn_world_create(ctx, &bad, &wx) == KN_E_INVALID, "bad primitive refused");
  }
  // primitives only, then no objects at all
  kn_world_desc po{0, nullptr, 1, prim};
  kn_world_id wp = 0;
  expect(kn_world_create(ctx, &po, &wp) == KN_OK, "world of primitives only");
  kn_camera c1 = camera(40, 30, KN_FP32);
  c1.eye[1] = -0.5f;
  c1.eye[2] = 6.0f;
  expect(kn_render_world(ctx, wp, &c1, &fr.f, nullptr) == KN_OK, "render a world of primitives");
  expect(kn_world_destroy(ctx, wp) == KN_OK, "world destroy");
  kn_world_desc none{0, nullptr, 0, nullptr};
  expect(kn_world_create(ctx, &none, &wp) == KN_OK, "empty world");
  expect(kn_render_world(ctx, wp, &c1, &fr.f, nullptr) == KN_OK, "render an empty world");
  expect(kn_world_destroy(ctx, w) == KN_OK, "world destroy releases its scenes");
  expect(kn_scene_destroy(ctx, b) == KN_OK, "scene destroy after its world");
  // a world and a scene left for kn_ctx_destroy
  kn_world_desc keep{1, inst, 1, prim};
  expect(kn_world_create(ctx, &keep, &wx) == KN_OK, "world kept until the context is destroyed");
  expect(kn_ctx_destroy(ctx) == KN_OK, "ctx destroy frees the remaining worlds");
}

// a primary frame large enough for early shading (the fake's round counts
// fall, so the first shading pass is forked onto the second stream)
void case_render_early() {
  kn_ctx* ctx = nullptr;
  expect(kn_ctx_create(0, (uint64_t)2 << 30, &ctx) == KN_OK, "ctx create");
  HostScene s = make_scene(4, 64, 17);
  kn_scene_desc d = desc_of(s, kAll);
  kn_scene_id id = 0;
  expect(kn_scene_create(ctx, &d, &id) == KN_OK, "scene create");
  for (kn_precision p : {KN_BF16, KN_FP32}) {
    DevFrame fr((size_t)1024 * 512);
    kn_camera c = camera(1024, 512, p);
    kn_stats st{};
    st.kernel_times = 1;
    expect(kn_render(ctx, id, &c, &fr.f, &st) == KN_OK, "large frame with early shading");
    expect(st.rounds >= 9, "rounds went on past the fork");
  }
  kn_scene_destroy(ctx, id);
  expect(kn_ctx_destroy(ctx) == KN_OK, "ctx destroy");
}

// a budget the render workspace of a large frame leaves too little of for
// a serving pool: kn_serve_start releases the workspace, and rendering
// afterwards allocates it again
void case_serve_release() {
  kn_ctx* ctx = nullptr;
  expect(kn_ctx_create(0, (uint64_t)480 << 20, &ctx) == KN_OK, "ctx create");
  HostScene s = make_scene(4, 32, 19);
  kn_scene_desc d = desc_of(s, 1u << KN_BF16);
  kn_scene_id id = 0;
  expect(kn_scene_create(ctx, &d, &id) == KN_OK, "scene create");
  {
    DevFrame fr((size_t)2048 * 2048);
    kn_camera c = camera(2048, 2048, KN_BF16);
    expect(kn_render(ctx, id, &c, &fr.f, nullptr) == KN_OK, "large frame (workspace grows)");
  }
  expect(kn_serve_start(ctx, 4, KN_BF16) == KN_OK, "serve start after releasing the workspace");
  DevFrame fr(64 * 48);
  kn_camera c = camera(64, 48, KN_BF16);
  kn_request_id r = 0;
  expect(kn_serve_submit(ctx, id, &c, &fr.f, &r) == KN_OK && kn_serve_poll(ctx, r, -1, nullptr) == KN_OK,
         "served frame");
  expect(kn_serve_stop(ctx) == KN_OK, "serve stop");
  expect(kn_render(ctx, id, &c, &fr.f, nullptr) == KN_OK, "render after serving (workspace allocated again)");
  kn_scene_destroy(ctx, id);
  expect(kn_ctx_destroy(ctx) == KN_OK, "ctx destroy");
}

void case_query_scan_err() {
  kn_ctx* ctx = nullptr;
  expect(kn_ctx_create(0, 0, &ctx) == KN_OK, "ctx create");
  HostScene s = make_scene(4, 32, 12);
  kn_scene_desc d = desc_of(s, 0);
  kn_scene_id id = 0;
  expect(kn_scene_create(ctx, &d, &id) == KN_OK, "scene create");
  float *pts = nullptr, *dd = nullptr;
  (void)hipMalloc((void**)&pts, 300 * 12);
  (void)hipMalloc((void**)&dd, 300 * 4);
  expect(kn_query(ctx, id, KN_FP32, pts, 300, dd, nullptr, nullptr, nullptr) == KN_E_DEVICE,
         "query reports the scan overrun");
  (void)hipFree(pts);
  (void)hipFree(dd);
  expect(kn_ctx_destroy(ctx) == KN_OK, "ctx destroy");
}

void case_serve(bool scan_err) {
  kn_ctx* ctx = nullptr;
  // a small budget keeps the fake's host-memory pool small
  expect(kn_ctx_create(0, (uint64_t)1 << 30, &ctx) == KN_OK, "ctx create");
  std::vector<kn_scene_id> ids;
  for (uint32_t k = 0; k < 3; ++k) {
    HostScene s = make_scene(2 + 2 * k, k % 2 ? 64 : 32, 20 + k);
    kn_scene_desc d = desc_of(s, 1u << KN_BF16);
    kn_scene_id id = 0;
    expect(kn_scene_create(ctx, &d, &id) == KN_OK, "scene create");
    ids.push_back(id);
  }
  expect(kn_serve_start(ctx, 8, KN_BF16) == KN_OK, "serve start");
  std::vector<DevFrame*> frames;
  std::vector<kn_request_id> reqs;
  int refused = 0;
  for (int i = 0; i < 12; ++i) {
    const uint32_t W = 16 + 8 * (i % 5), H = 9 + 4 * (i % 3);
    frames.push_back(new DevFrame((size_t)W * H));
    kn_camera c = camera(W, H, KN_BF16);
    kn_request_id r = 0;
    const kn_status s = kn_serve_submit(ctx, ids[i % 3], &c, &frames.back()->f, &r);
    if (s == KN_OK) reqs.push_back(r);
    else if (scan_err && (s == KN_E_DEVICE || s == KN_E_SHUTDOWN)) ++refused;   // the loop has failed
    else expect(false, "submit");
  }
  const kn_status want = scan_err ? KN_E_DEVICE : KN_OK;
  int ok = 0;
  for (kn_request_id r : reqs) ok += kn_serve_poll(ctx, r, -1, nullptr) == want;
  expect(!reqs.empty() && ok == (int)reqs.size(),
         scan_err ? "every accepted request fails on the scan overrun" : "every request done");
  if (scan_err) {
    kn_camera c = camera(8, 8, KN_BF16);
    kn_request_id r = 0;
    expect(kn_serve_submit(ctx, ids[0], &c, &frames[0]->f, &r) == KN_E_DEVICE,
           "later submits find the context poisoned");
  }
  expect(kn_serve_stop(ctx) == KN_OK, "serve stop");
  for (DevFrame* f : frames) delete f;
  for (kn_scene_id id : ids) kn_scene_destroy(ctx, id);
  expect(kn_ctx_destroy(ctx) == KN_OK, "ctx destroy");
}

}  // namespace

int main(int argc, char** argv) {
  const std::string c = argc > 1 ? argv[1] : "";
  if (c == "scenes") case_scenes();
  else if (c == "validation") case_validation();
  else if (c == "render") case_render_query(false);
  else if (c == "render_scan_err") case_render_query(true);
  else if (c == "query_scan_err") case_query_scan_err();
  else if (c == "grid_eikonal") case_grid_eikonal();
  else if (c == "world") case_world();
  else if (c == "render_early") case_render_early();
  else if (c == "serve_release") case_serve_release();
  else if (c == "noalloc") case_noalloc();
  else if (c == "serve") case_serve(false);
  else if (c == "serve_scan_err") case_serve(true);
  else {
    std::fprintf(stderr, "unknown case '%s'\n", c.c_str());
    return 2;
  }
  return g_fail ? 1 : 0;
}
