/* kn.h -- C ABI of the MI355X KiloNeuS renderer.
 *
 * KiloNeuS (arXiv 2206.10885) represents an object as a regular N^3 grid
 * over a fixed box, each cell holding a small SDF MLP and a small color MLP
 * (Sec. 3.1).  This library renders it: camera rays are clipped to the box,
 * sphere-traced through the grid (each step evaluates the MLP of the cell
 * the ray is in), and each hit is shaded with the normalised analytic SDF
 * gradient and the cell's color MLP (Sec. 3.4.1).
 *
 * Conventions for every call:
 *  - Every function returns kn_status.  Negative values are errors; the
 *    message of the calling thread's last error is kn_last_error().  No C++
 *    exception crosses this boundary.
 *  - A call that fails validation changes no output buffer.
 *  - After a device (HIP) error the context is poisoned: later calls on it
 *    return KN_E_DEVICE.
 *  - All calls are thread-safe.  GPU work of one context is serialised on
 *    the streams named below.
 *  - "DEVICE pointer" means memory on the context's HIP device (for example
 *    the data pointer of a torch tensor on that device); "HOST pointer"
 *    means ordinary CPU memory.
 */
#ifndef KN_H
#define KN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KN_ABI_VERSION 3u   /* 2: kn_camera gained `flags`, kn_frame `segments`;
                               3: kn_camera `sample_offset`, kn_frame `accum`, shared scenes */

typedef enum {
  KN_OK = 0,
  KN_PENDING = 1,          /* serve_poll: request not finished yet */
  KN_E_INVALID = -1,       /* bad argument (message says which) */
  KN_E_NOMEM = -2,         /* device allocation failed or HBM budget exceeded */
  KN_E_NOT_FOUND = -3,     /* unknown scene or request id */
  KN_E_BUSY = -4,          /* scene still used by queued or running requests */
  KN_E_DEVICE = -5,        /* HIP error; the context is poisoned */
  KN_E_TIMEOUT = -6,       /* serve_poll: timeout elapsed */
  KN_E_UNSUPPORTED = -7,   /* valid but not implemented (e.g. an MLP shape) */
  KN_E_SHUTDOWN = -8       /* serving loop not running */
} kn_status;

typedef enum {
  KN_FP32 = 0,             /* march weights and activations in float32 */
  KN_BF16 = 1,             /* march in bfloat16 (RNE), float32 accumulate */
  KN_FP8_E4M3 = 2          /* march in OCP fp8 e4m3: the two hidden layers' weights and
                              inputs rounded (nearest even, saturating at 448) with
                              power-of-two per-(cell, layer) scales; output row bf16 */
} kn_precision;

typedef struct kn_ctx kn_ctx;
typedef uint32_t kn_scene_id;
typedef uint64_t kn_request_id;

/* Creates a context on HIP device `hip_device`.  `hbm_budget_bytes` caps
 * the device memory the context may hold for scenes, ray state and serving
 * requests (0 = 90% of the device's free memory).  *out receives the
 * context; it owns every device allocation it makes.
 * Errors: KN_E_INVALID (out NULL, bad device), KN_E_DEVICE. */
kn_status kn_ctx_create(int hip_device, uint64_t hbm_budget_bytes, kn_ctx** out);

/* Stops serving if running, frees every scene and buffer, destroys ctx. */
kn_status kn_ctx_destroy(kn_ctx* ctx);

/* Message of the calling thread's last failed call ("" if none).  Valid
 * until that thread's next kn_ call. */
const char* kn_last_error(void);

/* ---------------------------------------------------------------------
 * Scenes (Sec. 3.1).  Host parameter layout, one float32 block per cell,
 * cells ordered g = ix + N*(iy + N*iz), ix along x:
 *   SDF block (KiloSDF, eq. 3; softplus_beta activations), P_sdf floats:
 *     W1[H][39]  b1[H]  W2[H][H]  b2[H]  W3[16][H]  b3[16]
 *     input: gamma_6 of the cell-local position x_l = (x - c)/h, raw
 *     coordinates first, then per axis sin(2^k pi x), cos(2^k pi x),
 *     k = 0..5 (eq. 1-2); output row 0 = SDF d in world units, rows 1..15
 *     = feature z.
 *   Color block (KiloColor, eq. 4), P_col floats:
 *     Wc1[32][48]  bc1[32]  Wc2[3][32]  bc2[3]
 *     input [x_l(3), gamma_4(v)(27), n(3), z(15)], ReLU hidden layer,
 *     sigmoid output; v is the unit ray direction.
 *   P_sdf = 39H + H + H*H + H + 16H + 16; P_col = 1667.
 * Supported: grid_n 1..64 (N^3 <= 2^18 cells), sdf_hidden 32 or 64,
 * sdf_layers 2, feat_dim 15, col_hidden 32, col_layers 1, col_in_has_x 1,
 * pos_freqs 6, dir_freqs 4; anything else returns KN_E_UNSUPPORTED.
 * --------------------------------------------------------------------- */
typedef struct {
  uint32_t abi_version;            /* KN_ABI_VERSION */
  uint32_t grid_n;                 /* N */
  float bbox_min[3], bbox_max[3];  /* the paper's box is [-1,1]^3 */
  uint32_t pos_freqs, dir_freqs;   /* 6, 4 */
  uint32_t sdf_hidden, sdf_layers, feat_dim;   /* 32|64, 2, 15 */
  uint32_t col_hidden, col_layers, col_in_has_x; /* 32, 1, 1 */
  float softplus_beta;             /* 100 */
  const float* sdf_params;         /* HOST, [N^3][P_sdf], copied by the call */
  const float* col_params;         /* HOST, [N^3][P_col], copied by the call */
  uint32_t precisions;             /* bitmask of low-precision copies to keep
                                      resident: bit KN_BF16, bit KN_FP8_E4M3
                                      (the float32 copy is always kept) */
} kn_scene_desc;

/* Copies and packs a scene onto the device.  The host arrays may be freed
 * when the call returns.  Errors: KN_E_INVALID, KN_E_UNSUPPORTED,
 * KN_E_NOMEM (budget), KN_E_DEVICE. */
kn_status kn_scene_create(kn_ctx* ctx, const kn_scene_desc* desc, kn_scene_id* out);

/* Frees a scene.  KN_E_BUSY while serving requests still reference it. */
kn_status kn_scene_destroy(kn_ctx* ctx, kn_scene_id scene);

/* ---------------------------------------------------------------------
 * Rendering (Sec. 3.4.1).
 * Camera: pinhole at `eye` looking at `look_at`, `up` fixes the roll; the
 * half-diagonal field of view has tangent tan_half_diag (0 selects
 * 1/sqrt(|eye-look_at|^2 - 1), which makes the image diagonal tangent to
 * the unit sphere).  Pixel (row i from the top, column j) looks through
 * u = (2(j+1/2)/W - 1) tx, v = (1 - 2(i+1/2)/H) ty, tx = T W/sqrt(W^2+H^2),
 * ty = T H/sqrt(W^2+H^2), d = normalize(f + u r + v u'), f = forward,
 * r = normalize(f x up), u' = r x f.
 * Tracing: the ray is clipped to the box; inside, each step evaluates the
 * SDF MLP of the current cell; f < eps is a hit; otherwise the ray advances
 * by f, but never past the current cell's exit plane: there it moves to the
 * neighbouring cell.  A ray that leaves the grid, or uses max_steps SDF
 * evaluations without a hit, misses.  Hits are refined by two guarded
 * Newton steps along the ray, then depth, normal and color are computed
 * there, with float32 weights and arithmetic whatever the march precision
 * (unless flags asks for split-bfloat16 shading).
 * --------------------------------------------------------------------- */
typedef struct {
  float eye[3], look_at[3], up[3];
  float tan_half_diag;
  uint32_t width, height;
  uint32_t spp;                    /* samples per pixel, 1..64; > 1 needs bounces >= 1 */
  uint32_t bounces;                /* 0: primary rays through the pixel centres, rgb = the
                                      hit's color (below); 1..16: path tracing, see below */
  uint32_t max_steps;              /* S, 1..1023 */
  float eps;                       /* hit threshold, > 0 */
  kn_precision precision;          /* weights used by the march */
  uint64_t seed;                   /* random stream for path tracing */
  const float* env_rgb;            /* DEVICE [env_h][env_w][3] or NULL (black); path tracing */
  uint32_t env_w, env_h;
  uint32_t flags;                  /* KN_CAMERA_* bits, 0 by default */
  uint32_t sample_offset;          /* path tracing: the index of this call's first sample (its
                                      samples are sample_offset .. sample_offset + spp - 1 of
                                      each pixel's stream); 0 for a single call */
} kn_camera;

/* kn_camera.flags: refinement and shading of a bf16 or fp8 march with the SDF
 * MLP's products on bfloat16 MFMA with split operands (each weight and each
 * layer input as hi + lo bfloat16, three products per pair, about 2^-16
 * relative error each) instead of float32 weights and arithmetic.  A faster
 * variant; the default is float32.  Ignored for float32 marches; refused by
 * the serving loop. */
#define KN_CAMERA_SPLIT_BF16_SHADING 1u
/* kn_camera.flags: Hart's unclamped sphere-tracing steps (Sec. 3.4.1 traces
 * the SDF inside the bounding interval; the step rule at cell faces is a
 * reading).  By default a step never crosses the current cell's exit plane:
 * it stops there and the ray continues in the face neighbour, so every cell
 * the ray crosses is evaluated and each MLP is used only inside its own
 * cell.  With this flag t always advances by the full SDF value; a step that
 * leaves the cell continues in the cell that contains the new point (any
 * cell, so cells inside a step are skipped without an evaluation), and the
 * hit cell's entry parameter is the t of its first evaluation.  Fewer
 * evaluations on fields that are coherent across cells; results differ from
 * the default where the per-cell fields disagree at seams.  kn_render only;
 * refused by the serving loop. */
#define KN_CAMERA_UNCLAMPED_STEPS 2u
/* Path tracing (bounces >= 1; Sec. 3.4.1: Lambertian surfaces, the color
 * MLP output is the albedo).  Each pixel traces spp paths; sample s of pixel
 * p is jittered inside the pixel by Philox-4x32-10 keyed by `seed` with
 * counter (p, s, 0, 0) when spp > 1 (pixel centre otherwise).  At each hit
 * the path scatters up to `bounces` times: throughput *= albedo, the new
 * direction is cosine-weighted about the normal (uniforms from counter
 * (p, s, k, 0) at the k-th scatter, basis of Duff et al. 2017), the new
 * segment starts 1e-3 above the surface.  A path that leaves the grid adds
 * throughput x env(direction) (equirectangular: u = 1/2 + atan2(d_x, -d_z)
 * / 2 pi, v = acos(d_y) / pi, bilinear, wrapping in u, row 0 up); a hit
 * after the last scatter adds nothing.  rgb = mean over the samples; depth,
 * normal, hit, steps and trace describe sample 0's primary segment.  The
 * serving loop renders primary rays only. */

/* Per-pixel march record, for diagnostics and replay of a hit's shading:
 * t_march = ray parameter where the march stopped, t_entry = where the ray
 * entered that cell, cell = global cell index (-1 for a box miss), status =
 * 0 box miss, 1 hit, 2 left the grid, 3 step budget used up. */
typedef struct {
  float t_march;
  float t_entry;
  int32_t cell;
  int32_t status;
} kn_trace_record;

/* Per-segment record of a path-traced frame (diagnostics and per-segment
 * checks): path p = pixel * spp + sample, segment k = 0..bounces at index
 * p * (bounces + 1) + k.  Segment 0 is the camera ray; segment k >= 1 starts
 * at the previous hit (x + 1e-3 n) in the scattered direction.  Written when
 * the segment starts (origin, dir; status -1 until it ends) and when it ends:
 * status 0 = it misses the box, 1 = hit (t = refined distance along dir,
 * normal, albedo = color MLP output), 2 = left the grid, 3 = step budget used
 * up; t_march, t_entry, cell and steps describe where the march stopped, as
 * in kn_trace_record.  Segments a path never reaches keep status -1. */
typedef struct {
  float origin[3];
  float dir[3];
  float t_march, t_entry;
  float t;
  float normal[3];
  float albedo[3];
  int32_t cell;
  int32_t status;
  uint32_t steps;
  uint32_t pad[2];
} kn_segment_record;   /* 80 bytes */

/* Output buffers, all DEVICE pointers owned by the caller, row-major
 * [height][width] (rgb and normal with 3 floats per pixel).  Only rgb is
 * required; NULL skips an output.  Misses get rgb = background (black, or
 * the environment map looked up along the ray), depth = 0, normal = 0,
 * hit = 0.  depth is the distance along the unit ray from the eye. */
typedef struct {
  float* rgb;
  float* depth;
  float* normal;
  uint8_t* hit;
  uint16_t* steps;                 /* SDF evaluations of the march */
  kn_trace_record* trace;          /* optional diagnostics */
  kn_segment_record* segments;     /* optional, path tracing: [W*H*spp][bounces + 1] */
  void* hip_stream;                /* hipStream_t to run on; NULL = ctx stream */
  float* accum;                    /* optional, path tracing: progressive accumulation,
                                      [height][width][3] running sum of the samples'
                                      radiance.  A call with sample_offset 0 restarts it;
                                      every call adds its spp samples and sets
                                      rgb = accum / (sample_offset + spp).  With accum the
                                      pixel samples are jittered even at spp = 1. */
} kn_frame;

typedef struct {
  double gpu_ms;                   /* first to last kernel of the call (hipEvents) */
  double wall_ms;                  /* host time of the call */
  uint64_t rays, evals, hits, rounds;
  uint32_t kernel_times;           /* in: nonzero => also time each march and
                                      shading launch with hipEvents (adds two
                                      event records per launch) */
  uint32_t march_launches;         /* out (kernel_times): march launches */
  double march_ms;                 /* out (kernel_times): summed march kernel time */
  double shade_ms;                 /* out (kernel_times): shading kernel time */
  uint64_t march_tiles;            /* out: pairs of 16-ray MFMA tiles evaluated by the march */
  uint64_t march_chunks;           /* out: march work items (<= 256 rays of one cell) */
} kn_stats;

/* Renders one frame into `frame` and returns when it is complete on the
 * stream.  Errors: KN_E_INVALID, KN_E_NOT_FOUND, KN_E_UNSUPPORTED,
 * KN_E_NOMEM, KN_E_DEVICE. */
kn_status kn_render(kn_ctx* ctx, kn_scene_id scene, const kn_camera* cam, const kn_frame* frame,
                    kn_stats* stats_opt);

/* Batched point query (per-cell MLPs evaluated on per-cell batches of
 * points, Sec. 3.3): for each world point x (DEVICE float [n][3]) evaluates the
 * SDF MLP of the cell containing x (points outside the box are clamped to
 * the nearest cell): d (DEVICE float [n]), and optionally the world-space
 * gradient of d (DEVICE float [n][3]) and the feature z (DEVICE float
 * [n][15]).  `precision` selects the weights for d; gradients and features
 * use float32.  Runs on `hip_stream` (NULL = ctx stream) and returns when
 * done. */
kn_status kn_query(kn_ctx* ctx, kn_scene_id scene, kn_precision precision, const float* points,
                   uint64_t n, float* d_out, float* grad_out, float* z_out, void* hip_stream);

/* Allocation-free variant of kn_query, for callers that cannot allocate
 * device memory during the call (code being recorded into a HIP graph, tight
 * serving loops, harnesses that forbid allocation).  Same arguments, outputs,
 * arithmetic and results (bit for bit) as kn_query; the work buffers (point
 * records, per-cell counters and cursors, work items, control block) live in
 * one static array per GPU in the library (about 12.2 MB, held by each GPU
 * the library runs on until the process ends), whose device address the
 * context looks up when it is created.  No hipMalloc, hipFree or allocating
 * library routine is called, and counters are cleared with kernels, not
 * memset nodes.  Limits: n <= 262144 points and grids of at most 2^18 cells;
 * larger calls return KN_E_INVALID and change no output.  Every call on a GPU
 * uses that GPU's array: calls of this process on one device are serialised
 * by the library, and each call returns after its work is done on
 * `hip_stream` (NULL = ctx stream); work of another library instance that
 * overlaps on the same device would race.  Errors as kn_query. */
kn_status kn_query_noalloc(kn_ctx* ctx, kn_scene_id scene, kn_precision precision, const float* points,
                           uint64_t n, float* d_out, float* grad_out, float* z_out, void* hip_stream);

/* Dense lattice sampling of the SDF, the input of marching-cubes mesh
 * extraction (Sec. 4.1 extracts meshes on a 512^3 lattice).  The lattice has
 * R points per axis spanning the scene box: point (i, j, k) lies at
 * bbox_min + (bbox_max - bbox_min) (i, j, k) / (R - 1).  Along each axis its
 * cell is floor(i N / (R - 1)) in integer arithmetic, clamped to N - 1, so a
 * point on an inner cell face belongs to the cell above it and the last
 * lattice plane to the last cell (the cell map of Sec. 3.1 at the exact
 * position); it is evaluated with that cell's SDF MLP.
 * d_out: DEVICE float [R^3], caller-owned, index i + R (j + R k).
 * grad_out: NULL, or DEVICE float [R^3][3] for the world-space gradient of d;
 * gradients need precision KN_FP32 (the float32 weights).
 * 2 <= R <= 4096, with at most 2^31 lattice points in a cell.  Runs on `hip_stream` (NULL = ctx stream) and returns when
 * done.  Errors: KN_E_INVALID (outputs untouched), KN_E_NOT_FOUND,
 * KN_E_DEVICE. */
kn_status kn_grid_sample(kn_ctx* ctx, kn_scene_id scene, kn_precision precision, uint32_t R, float* d_out,
                         float* grad_out, void* hip_stream);

/* Eikonal term by central finite differences of the global, piecewise SDF
 * (Sec. 3.2 defines the eikonal loss as the mean of (|grad d| - 1)^2 over
 * sampled points; Sec. 3.3 takes the gradient by finite differences, each
 * stencil value from the MLP of the cell containing the stencil point, which
 * couples neighbouring cells at their seams).  For each point x (DEVICE float
 * [n][3]): the six stencil points x +- delta e_a are formed in float32 (order
 * +x, -x, +y, -y, +z, -z) and evaluated as by kn_query with `precision`;
 * g_a = (d(x + delta e_a) - d(x - delta e_a)) / (2 delta) and
 * gnorm_out[q] = |g| (DEVICE float [n]).  stencil_out: NULL, or DEVICE float
 * [n][6] receiving the six stencil values.  loss_out: NULL, or a DEVICE
 * double receiving the mean of (gnorm - 1)^2 over the n points, summed in
 * double in a fixed order (the same on every run).  delta > 0 in world units;
 * n <= 2^28 / 6.  The context's work buffers grow to about 750 bytes per
 * point and are kept between calls (counted against the HBM budget).
 * Returns when done on `hip_stream`.  Errors: KN_E_INVALID, KN_E_NOT_FOUND, KN_E_NOMEM,
 * KN_E_DEVICE. */
kn_status kn_eikonal_fd(kn_ctx* ctx, kn_scene_id scene, kn_precision precision, const float* points, uint64_t n,
                        float delta, float* gnorm_out, float* stencil_out, double* loss_out, void* hip_stream);

/* ---------------------------------------------------------------------
 * Shared scenes (Sec. 3.4: the path tracer renders KiloNeuS objects
 * together with classic primitives).  A world holds up to 16 KiloNeuS
 * instances and up to 256 primitives.
 *   - An instance places a resident scene by a uniform scale s > 0 and a
 *     translation T: world x = T + s x_local.  Its MLPs see local
 *     coordinates (ray ((o - T) / s, d); a local parameter t' is the world
 *     distance s t').  The world boxes T + s [bbox_min, bbox_max] of the
 *     instances must be disjoint.
 *   - Primitives are Lambertian (albedo in [0, 1]^3) and two-sided (the
 *     shading normal faces the incoming ray): spheres (p[0..2] centre,
 *     p[3] radius > 0), axis-aligned boxes (p[0..2] min < p[3..5] max) and
 *     triangles (p[0..8]: three vertices, nonzero area).
 *   - A ray's next object is the nearest of its closest primitive hit and
 *     the instance boxes it enters (ties go to the primitive, then to the
 *     lower index).  An instance is sphere-traced, as kn_render does, from
 *     its box entry to the nearer of its box exit and the closest primitive
 *     hit; a march that reaches that end goes on past the box, one that
 *     runs out of steps ends the ray as a miss.
 *   - Primary renders (bounces 0): rgb is the primitive's albedo or the
 *     KiloNeuS color; depth is the world distance; hit = 1 on either.  Path
 *     tracing treats every surface as Lambertian with its albedo, as
 *     kn_render does.  kn_trace_record.cell of a primitive hit is
 *     -(2 + primitive index); segments are not recorded.
 * --------------------------------------------------------------------- */
typedef uint32_t kn_world_id;
enum { KN_PRIM_SPHERE = 1, KN_PRIM_BOX = 2, KN_PRIM_TRIANGLE = 3 };
typedef struct {
  uint32_t kind;                   /* KN_PRIM_* */
  float p[9];
  float albedo[3];
} kn_primitive;
typedef struct {
  kn_scene_id scene;
  float translate[3];
  float scale;
} kn_instance;
typedef struct {
  uint32_t n_instances;            /* 0..16 */
  const kn_instance* instances;    /* HOST */
  uint32_t n_primitives;           /* 0..256 */
  const kn_primitive* primitives;  /* HOST, copied by the call */
} kn_world_desc;

/* Creates a world over resident scenes (which it references until it is
 * destroyed: kn_scene_destroy of such a scene returns KN_E_BUSY).
 * Errors: KN_E_INVALID (overlapping instance boxes, bad primitive),
 * KN_E_NOT_FOUND, KN_E_NOMEM, KN_E_DEVICE. */
kn_status kn_world_create(kn_ctx* ctx, const kn_world_desc* desc, kn_world_id* out);
kn_status kn_world_destroy(kn_ctx* ctx, kn_world_id world);

/* Renders one frame of a world, as kn_render does a single scene (same
 * camera, frame and flags; every instance's scene needs a copy in the
 * camera's precision).  Returns when the frame is complete.  Errors as
 * kn_render, and KN_E_UNSUPPORTED for unclamped steps in a world whose
 * instances mix MLP widths. */
kn_status kn_render_world(kn_ctx* ctx, kn_world_id world, const kn_camera* cam, const kn_frame* frame,
                          kn_stats* stats_opt);

/* ---------------------------------------------------------------------
 * Serving: a loop that keeps scenes resident and renders queued requests
 * with continuous batching (requests arriving while others run join the
 * shared ray pool as memory allows).
 * --------------------------------------------------------------------- */
/* Starts the loop with a ray pool sized to what the HBM budget leaves (at
 * most 32 M rays).  When the budget leaves too little, the workspace that
 * kn_render keeps between calls is released first (the next kn_render
 * allocates it again).  Errors: KN_E_INVALID, KN_E_BUSY (already running),
 * KN_E_NOMEM, KN_E_DEVICE. */
kn_status kn_serve_start(kn_ctx* ctx, uint32_t max_inflight, kn_precision precision);
kn_status kn_serve_submit(kn_ctx* ctx, kn_scene_id scene, const kn_camera* cam,
                          const kn_frame* frame, kn_request_id* out);
kn_status kn_serve_poll(kn_ctx* ctx, kn_request_id req, int64_t timeout_us, kn_stats* stats_opt);
kn_status kn_serve_stop(kn_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
