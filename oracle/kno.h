/* FP64 CPU oracle for the KiloNeuS rendering hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the tests, the package's smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no source with the HIP
 * path: encoding, MLPs, camera, box clip, cell stepping, refinement and
 * shading are written out here again, plainly, in double precision.
 *
 * Paper: "KiloNeuS: A Versatile Neural Implicit Surface Representation for
 * Real-Time Rendering" (arXiv 2206.10885).
 *   - Sec. 3.1, eq. 1-2: Fourier encoding gamma_L, raw input included,
 *     R^n -> R^{n+2nL}; L = 6 for positions, L = 4 for view directions.
 *   - Sec. 3.1, eq. 3-4: d(x) = f(gamma_6(x); Theta^d_{m(x)}),
 *     c = sigmoid(g(x, gamma_4(v), n, z; Theta^c_{m(x)})); softplus for the
 *     SDF MLP, ReLU for the color MLP; n = grad d / |grad d|.
 *   - Sec. 3.1: m : R^3 -> [N]^3 picks the cell's MLP pair.
 *   - Sec. 3.4.1: closest bounding-volume hit, sphere tracing inside the
 *     interval until it reaches the 0-level set, then normal from the
 *     normalised SDF gradient and color from the color MLP at the hit;
 *     Lambertian surfaces.
 * Readings of points the paper leaves open (cell-boundary stepping, local
 * cell coordinates, Newton refinement, camera model, ...) are listed in the
 * design notes of the repository and restated at each function below.
 */
#ifndef KNO_H
#define KNO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t N;            /* grid resolution per axis; cell g = ix + N*(iy + N*iz) */
  int32_t H;            /* SDF hidden width */
  int32_t pos_freqs;    /* 6 */
  int32_t dir_freqs;    /* 4 */
  double beta;          /* softplus beta (100) */
  double bmin[3], bmax[3];
  const float* sdf;     /* [N^3][P_sdf]: W1[H][39] b1[H] W2[H][H] b2[H] W3[16][H] b3[16] */
  const float* col;     /* [N^3][P_col]: Wc1[32][48] bc1[32] Wc2[3][32] bc2[3] */
} kno_scene;

typedef struct {
  double eye[3], look_at[3], up[3];
  double tan_half_diag;   /* 0 => 1/sqrt(|eye - look_at|^2 - 1) */
  int32_t width, height;
  int32_t max_steps;      /* S: SDF evaluations allowed per ray */
  double eps;             /* hit threshold */
  double background[3];   /* rgb of rays that miss */
  int32_t step_mode;      /* KNO_STEP_CLAMPED or KNO_STEP_UNCLAMPED */
} kno_camera;

/* sphere-tracing step rule: clamp each step at the cell's exit plane and
 * move to the face neighbour, or take Hart's full step across cells */
enum { KNO_STEP_CLAMPED = 0, KNO_STEP_UNCLAMPED = 1 };

/* march outcome */
enum { KNO_BOX_MISS = 0, KNO_HIT = 1, KNO_EXIT_MISS = 2, KNO_BUDGET_MISS = 3 };

typedef struct {
  int32_t status;       /* KNO_* */
  int32_t steps;        /* SDF evaluations used by the march */
  int32_t cell[3];      /* hit cell (status == KNO_HIT) */
  double t;             /* march t at the hit (before refinement) */
  double t_entry;       /* t where the ray entered the hit cell */
  double fmin;          /* smallest SDF value seen along the march */
} kno_trace_result;

int kno_sdf_params(int H);
int kno_col_params(void);

void kno_encode(const double* p, int n, int L, double* out);
double kno_softplus(double u, double beta);
void kno_sdf_eval(const kno_scene* s, int cell, const double xl[3], double out[16],
                  double grad_xl[3]);
void kno_color_eval(const kno_scene* s, int cell, const double xl[3], const double v[3],
                    const double n[3], const double z[15], double rgb[3]);
void kno_camera_ray(const kno_camera* c, int row, int colm, double xi1, double xi2,
                    double o[3], double d[3]);
int kno_slab(const kno_scene* s, const double o[3], const double d[3], double* t_near,
             double* t_far);
int kno_cells_along_ray(const kno_scene* s, const double o[3], const double d[3], int max_cells,
                        int32_t* cells, double* t_enter);
void kno_trace(const kno_scene* s, const double o[3], const double d[3], int max_steps,
               double eps, kno_trace_result* r);
void kno_trace_mode(const kno_scene* s, const double o[3], const double d[3], int max_steps,
                    double eps, int step_mode, kno_trace_result* r);
void kno_shade(const kno_scene* s, const double o[3], const double d[3],
               const kno_trace_result* r, double* depth, double normal[3], double rgb[3],
               double z[15]);
void kno_render(const kno_scene* s, const kno_camera* c, const int64_t* pixels, int64_t npix,
                double* rgb, double* depth, double* normal, uint8_t* hit, int32_t* steps,
                int32_t* status, double* fmin, int nthreads);

/* path tracing (Sec. 3.4.1) */
typedef struct {
  const float* rgb;       /* [h][w][3] equirectangular map, or NULL (black) */
  int32_t w, h;
} kno_env;

typedef struct {
  int32_t spp;            /* samples per pixel (1: through the pixel centre) */
  int32_t bounces;        /* scatters per path */
  uint64_t seed;          /* Philox key */
  kno_env env;
  int32_t jitter;         /* pixel jitter even at spp = 1 (progressive accumulation) */
} kno_pt;

void kno_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void kno_onb(const double n[3], double b1[3], double b2[3]);
void kno_cosine_dir(const double n[3], double u1, double u2, double out[3]);
void kno_env_lookup(const kno_env* e, const double d[3], double rgb[3]);
void kno_path_trace(const kno_scene* s, const kno_camera* c, const kno_pt* pt, const int64_t* pixels,
                    int64_t npix, double* rgb, double* depth, double* normal, uint8_t* hit, int nthreads);

/* shared scenes (Sec. 3.4: KiloNeuS objects with classic primitives):
 * Lambertian spheres, axis-aligned boxes and triangles, and KiloNeuS
 * instances placed by a uniform scale and a translation */
enum { KNO_PRIM_SPHERE = 1, KNO_PRIM_BOX = 2, KNO_PRIM_TRIANGLE = 3 };
typedef struct {
  int32_t kind;           /* KNO_PRIM_* */
  double p[9];            /* sphere: centre, radius; box: min, max; triangle: 3 vertices */
  double albedo[3];
} kno_prim;

typedef struct {
  const kno_scene* scene; /* its box [bmin, bmax] in the instance's own frame */
  double translate[3];    /* world = translate + scale * local */
  double scale;
} kno_instance;

typedef struct {
  int32_t n_inst;
  const kno_instance* inst;
  int32_t n_prim;
  const kno_prim* prim;
} kno_world;

/* outcome of a world ray */
enum { KNO_OBJ_NONE = 0, KNO_OBJ_PRIM = 1, KNO_OBJ_INST = 2 };

int kno_prim_hit(const kno_prim* p, const double o[3], const double d[3], double t_min, double* t,
                 double n[3]);
void kno_world_render(const kno_world* w, const kno_camera* c, const int64_t* pixels, int64_t npix,
                      double* rgb, double* depth, double* normal, uint8_t* hit, int32_t* object,
                      int nthreads);
void kno_world_path_trace(const kno_world* w, const kno_camera* c, const kno_pt* pt, const int64_t* pixels,
                          int64_t npix, double* rgb, double* depth, double* normal, uint8_t* hit,
                          int nthreads);

/* point-query workloads (Sec. 3.3): the global piecewise SDF at world
 * points, on a dense lattice (mesh extraction, Sec. 4.1) and the eikonal
 * term by central finite differences (Sec. 3.2, 3.3) */
void kno_query(const kno_scene* s, const double* pts, int64_t n, double* d, double* grad, double* z,
               int nthreads);
void kno_grid_sample(const kno_scene* s, int R, const int64_t* lin, int64_t n, double* d, double* grad,
                     double* z, int nthreads);
void kno_eikonal_fd(const kno_scene* s, const double* pts, int64_t n, double delta, double* gnorm,
                    double* stencil, double* loss, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
