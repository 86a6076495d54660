/* FP64 CPU oracle for the KiloNeuS rendering hot path -- implementation.
 *
 * TEST INFRASTRUCTURE ONLY (see kno.h).  Plain per-ray loops in double
 * precision with libm; no blocking, fusion or reordering beyond what each
 * definition states.  Parameters are float32 in the scene and are promoted
 * exactly to double.
 */
#include "kno.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FEAT 15
#define KNO_MAX_H 256   /* widest SDF hidden layer the oracle accepts */
#define COL_HID 32

static const double PI = 3.14159265358979323846;

int kno_sdf_params(int H) {
  int din = 3 + 6 * 6;
  return din * H + H + H * H + H + (1 + FEAT) * H + (1 + FEAT);
}

int kno_col_params(void) {
  int cin = 3 + (3 + 6 * 4) + 3 + FEAT;
  return cin * COL_HID + COL_HID + 3 * COL_HID + 3;
}

/* Sec. 3.1, eq. 1-2: gamma_L(p) for p in R^n.  Raw coordinates first, then
 * for every coordinate p_a the pairs sin(2^k pi p_a), cos(2^k pi p_a) for
 * k = 0..L-1 (the raw input is kept because the paper states the encoding
 * maps R^n to R^{n+2nL}).  out has n + 2nL entries. */
void kno_encode(const double* p, int n, int L, double* out) {
  for (int a = 0; a < n; ++a) out[a] = p[a];
  for (int a = 0; a < n; ++a) {
    for (int k = 0; k < L; ++k) {
      double w = ldexp(PI, k) * p[a];
      out[n + a * 2 * L + 2 * k] = sin(w);
      out[n + a * 2 * L + 2 * k + 1] = cos(w);
    }
  }
}

/* softplus with sharpness beta, log(1 + exp(beta u)) / beta, written in its
 * overflow-free form max(u, 0) + log1p(exp(-beta |u|)) / beta. */
double kno_softplus(double u, double beta) {
  return fmax(u, 0.0) + log1p(exp(-beta * fabs(u))) / beta;
}

/* logistic function, d softplus_beta(u) / du = sigmoid(beta u) */
static double sigmoid(double x) {
  if (x >= 0) return 1.0 / (1.0 + exp(-x));
  double e = exp(x);
  return e / (1.0 + e);
}

typedef struct {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
} sdf_view;

static sdf_view sdf_block(const kno_scene* s, int cell) {
  const int H = s->H, din = 3 + 6 * s->pos_freqs;
  const float* p = s->sdf + (size_t)cell * (size_t)kno_sdf_params(H);
  sdf_view v;
  v.W1 = p; p += din * H;
  v.b1 = p; p += H;
  v.W2 = p; p += H * H;
  v.b2 = p; p += H;
  v.W3 = p; p += (1 + FEAT) * H;
  v.b3 = p;
  return v;
}

/* KiloSDF MLP of one cell (Sec. 3.1, eq. 3): e = gamma_6(x_local),
 * a1 = softplus(W1 e + b1), a2 = softplus(W2 a1 + b2), y = W3 a2 + b3;
 * out[0] = d (world units), out[1..15] = feature z.
 * If grad_xl is not NULL, the gradient of out[0] with respect to the local
 * coordinates x_local is computed by the chain rule backwards through the
 * layers and the encoding: d/dp sin(w p) = w cos(w p), d/dp cos(w p) =
 * -w sin(w p), softplus' = sigmoid(beta u). */
void kno_sdf_eval(const kno_scene* s, int cell, const double xl[3], double out[16],
                  double grad_xl[3]) {
  const int H = s->H, L = s->pos_freqs, din = 3 + 6 * L;
  sdf_view w = sdf_block(s, cell);
  double e[3 + 6 * 16];
  kno_encode(xl, 3, L, e);
  double u1[KNO_MAX_H], a1[KNO_MAX_H], u2[KNO_MAX_H], a2[KNO_MAX_H];
  for (int j = 0; j < H; ++j) {
    double acc = w.b1[j];
    for (int k = 0; k < din; ++k) acc += (double)w.W1[j * din + k] * e[k];
    u1[j] = acc;
    a1[j] = kno_softplus(acc, s->beta);
  }
  for (int j = 0; j < H; ++j) {
    double acc = w.b2[j];
    for (int k = 0; k < H; ++k) acc += (double)w.W2[j * H + k] * a1[k];
    u2[j] = acc;
    a2[j] = kno_softplus(acc, s->beta);
  }
  for (int o = 0; o < 1 + FEAT; ++o) {
    double acc = w.b3[o];
    for (int k = 0; k < H; ++k) acc += (double)w.W3[o * H + k] * a2[k];
    out[o] = acc;
  }
  if (grad_xl) {
    double d2[KNO_MAX_H], d1[KNO_MAX_H];
    for (int j = 0; j < H; ++j) d2[j] = (double)w.W3[j] * sigmoid(s->beta * u2[j]);
    for (int k = 0; k < H; ++k) {
      double acc = 0;
      for (int j = 0; j < H; ++j) acc += (double)w.W2[j * H + k] * d2[j];
      d1[k] = acc * sigmoid(s->beta * u1[k]);
    }
    double ge[3 + 6 * 16];
    for (int m = 0; m < din; ++m) {
      double acc = 0;
      for (int k = 0; k < H; ++k) acc += (double)w.W1[k * din + m] * d1[k];
      ge[m] = acc;
    }
    for (int a = 0; a < 3; ++a) {
      double g = ge[a];
      for (int k = 0; k < L; ++k) {
        double wk = ldexp(PI, k);
        double gs = ge[3 + a * 2 * L + 2 * k], gc = ge[3 + a * 2 * L + 2 * k + 1];
        g += wk * (gs * cos(wk * xl[a]) - gc * sin(wk * xl[a]));
      }
      grad_xl[a] = g;
    }
  }
}

/* KiloColor MLP of one cell (Sec. 3.1, eq. 4): input
 * [x_local(3), gamma_4(v)(27), n(3), z(15)] -> ReLU(32) -> sigmoid(3). */
void kno_color_eval(const kno_scene* s, int cell, const double xl[3], const double v[3],
                    const double n[3], const double z[15], double rgb[3]) {
  const int L = s->dir_freqs;
  const int cin = 3 + (3 + 6 * L) + 3 + FEAT;
  const float* p = s->col + (size_t)cell * (size_t)kno_col_params();
  const float *Wc1 = p, *bc1 = p + cin * COL_HID, *Wc2 = bc1 + COL_HID, *bc2 = Wc2 + 3 * COL_HID;
  double in[3 + 3 + 6 * 16 + 3 + FEAT];
  int q = 0;
  for (int a = 0; a < 3; ++a) in[q++] = xl[a];
  kno_encode(v, 3, L, in + q);
  q += 3 + 6 * L;
  for (int a = 0; a < 3; ++a) in[q++] = n[a];
  for (int i = 0; i < FEAT; ++i) in[q++] = z[i];
  double hid[COL_HID];
  for (int j = 0; j < COL_HID; ++j) {
    double acc = bc1[j];
    for (int k = 0; k < cin; ++k) acc += (double)Wc1[j * cin + k] * in[k];
    hid[j] = acc > 0 ? acc : 0.0;
  }
  for (int c = 0; c < 3; ++c) {
    double acc = bc2[c];
    for (int k = 0; k < COL_HID; ++k) acc += (double)Wc2[c * COL_HID + k] * hid[k];
    rgb[c] = sigmoid(acc);
  }
}

static void normalize3(double v[3]) {
  double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  v[0] /= l; v[1] /= l; v[2] /= l;
}

static void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Pinhole camera.  The paper only states that the object sits in front of
 * the camera with every ray meeting its bounding volume (Sec. 4.2); this
 * model is the repository's reading: forward = normalize(look_at - eye),
 * right = normalize(forward x up), up' = right x forward; the half-diagonal
 * field of view has tangent T (0 selects 1/sqrt(D^2 - 1), D = |eye - look_at|,
 * so the diagonal is tangent to the unit sphere).  Pixel (row, col) with
 * sub-pixel offset (xi1, xi2): u = (2 (col + xi1)/W - 1) tx,
 * v = (1 - 2 (row + xi2)/H) ty, tx = T W / sqrt(W^2 + H^2),
 * ty = T H / sqrt(W^2 + H^2); d = normalize(forward + u right + v up'). */
void kno_camera_ray(const kno_camera* c, int row, int colm, double xi1, double xi2,
                    double o[3], double d[3]) {
  double fwd[3] = {c->look_at[0] - c->eye[0], c->look_at[1] - c->eye[1],
                   c->look_at[2] - c->eye[2]};
  double dist2 = fwd[0] * fwd[0] + fwd[1] * fwd[1] + fwd[2] * fwd[2];
  normalize3(fwd);
  double right[3], upp[3];
  cross3(fwd, c->up, right);
  normalize3(right);
  cross3(right, fwd, upp);
  double T = c->tan_half_diag > 0 ? c->tan_half_diag : 1.0 / sqrt(dist2 - 1.0);
  double W = c->width, Hh = c->height;
  double diag = sqrt(W * W + Hh * Hh);
  double tx = T * W / diag, ty = T * Hh / diag;
  double u = (2.0 * (colm + xi1) / W - 1.0) * tx;
  double v = (1.0 - 2.0 * (row + xi2) / Hh) * ty;
  for (int a = 0; a < 3; ++a) {
    o[a] = c->eye[a];
    d[a] = fwd[a] + u * right[a] + v * upp[a];
  }
  normalize3(d);
}

/* Closest bounding-volume hit (Sec. 3.4.1), slab method on the box.
 * Returns 1 and [t_near, t_far] when the ray meets the box ahead of it. */
int kno_slab(const kno_scene* s, const double o[3], const double d[3], double* t_near,
             double* t_far) {
  double tn = -INFINITY, tf = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (d[a] != 0.0) {
      double t1 = (s->bmin[a] - o[a]) / d[a], t2 = (s->bmax[a] - o[a]) / d[a];
      tn = fmax(tn, fmin(t1, t2));
      tf = fmin(tf, fmax(t1, t2));
    } else if (o[a] < s->bmin[a] || o[a] > s->bmax[a]) {
      return 0;
    }
  }
  *t_near = tn;
  *t_far = tf;
  return (tn <= tf && tf > 0.0) ? 1 : 0;
}

static double cell_side(const kno_scene* s, int a) { return (s->bmax[a] - s->bmin[a]) / s->N; }

/* Cell map m (Sec. 3.1) at parameter t: floor of the box-relative position
 * over the cell side, clamped to the grid. */
static void cell_at(const kno_scene* s, const double o[3], const double d[3], double t, int idx[3]) {
  for (int a = 0; a < 3; ++a) {
    double x = o[a] + t * d[a];
    int i = (int)floor((x - s->bmin[a]) / cell_side(s, a));
    idx[a] = i < 0 ? 0 : (i > s->N - 1 ? s->N - 1 : i);
  }
}

/* Parameter where the ray leaves cell idx: the nearest of the three exit
 * planes (the far plane along each axis the ray moves on).  *axis gets the
 * plane's axis, ties going to the lowest axis. */
static double cell_exit(const kno_scene* s, const double o[3], const double d[3], const int idx[3],
                        int* axis) {
  double best = INFINITY;
  int ba = 0;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) continue;
    double plane = s->bmin[a] + (idx[a] + (d[a] > 0 ? 1 : 0)) * cell_side(s, a);
    double ta = (plane - o[a]) / d[a];
    if (ta < best) { best = ta; ba = a; }
  }
  if (axis) *axis = ba;
  return best;
}

static int cell_index(const kno_scene* s, const int idx[3]) {
  return idx[0] + s->N * (idx[1] + s->N * idx[2]);
}

static void local_coords(const kno_scene* s, const int idx[3], const double x[3], double xl[3]) {
  for (int a = 0; a < 3; ++a) {
    double side = cell_side(s, a);
    double c = s->bmin[a] + (idx[a] + 0.5) * side;
    xl[a] = (x[a] - c) / (0.5 * side);
  }
}

/* Cells the ray passes through inside the box, in order, by the same
 * cell-exit stepping the march uses (no SDF queries).  Returns the count. */
int kno_cells_along_ray(const kno_scene* s, const double o[3], const double d[3], int max_cells,
                        int32_t* cells, double* t_enter) {
  double tn, tf;
  if (!kno_slab(s, o, d, &tn, &tf)) return 0;
  double t = fmax(tn, 0.0);
  int idx[3];
  cell_at(s, o, d, t, idx);
  int n = 0;
  while (n < max_cells) {
    cells[n] = cell_index(s, idx);
    t_enter[n] = t;
    ++n;
    int ax;
    double te = fmax(t, cell_exit(s, o, d, idx, &ax));
    t = te;
    idx[ax] += d[ax] > 0 ? 1 : -1;
    if (idx[ax] < 0 || idx[ax] >= s->N || t > tf) break;
  }
  return n;
}

/* Sphere tracing inside the box interval (Sec. 3.4.1; Hart's rule: advance
 * by the SDF value).  Each step queries the MLP of the cell the ray is in,
 * in that cell's local frame.  A step that would cross the cell's exit plane
 * stops on the plane instead and the ray moves to the neighbouring cell
 * (cell-boundary stepping: a cell's MLP is only evaluated inside its cell).
 * HIT when the SDF is below eps (negative values included); MISS when the
 * ray leaves the grid or the box interval, or after max_steps evaluations. */
void kno_trace(const kno_scene* s, const double o[3], const double d[3], int max_steps,
               double eps, kno_trace_result* r) {
  kno_trace_mode(s, o, d, max_steps, eps, KNO_STEP_CLAMPED, r);
}

/* The same march with a choice of step rule.  KNO_STEP_UNCLAMPED is Hart's
 * rule without the cell-boundary clamp: t always advances by the SDF value;
 * when the new point lies past the current cell's exit plane the ray goes on
 * in the cell that contains the new point (cell map m of Sec. 3.1), which
 * need not be a neighbour, so cells inside a step are never evaluated.  The
 * cell's entry parameter (the refinement's lower bound) is the t of its
 * first evaluation. */
static void trace_interval(const kno_scene* s, const double o[3], const double d[3], double t0, double tf,
                           int max_steps, double eps, int step_mode, kno_trace_result* r);

void kno_trace_mode(const kno_scene* s, const double o[3], const double d[3], int max_steps,
                    double eps, int step_mode, kno_trace_result* r) {
  double tn, tf;
  if (!kno_slab(s, o, d, &tn, &tf)) {
    memset(r, 0, sizeof(*r));
    r->fmin = INFINITY;
    r->status = KNO_BOX_MISS;
    return;
  }
  trace_interval(s, o, d, fmax(tn, 0.0), tf, max_steps, eps, step_mode, r);
}

/* The march over the parameter interval [t0, tf] inside the box: the entry
 * cell is the one containing o + t0 d, and a step past tf ends the march as
 * a miss wherever it lands (for the whole box interval, tf is the box exit,
 * which no in-cell step can pass). */
static void trace_interval(const kno_scene* s, const double o[3], const double d[3], double t0, double tf,
                           int max_steps, double eps, int step_mode, kno_trace_result* r) {
  memset(r, 0, sizeof(*r));
  r->fmin = INFINITY;
  double t = t0;
  int idx[3];
  cell_at(s, o, d, t, idx);
  double t_entry = t;
  for (int k = 0; k < max_steps; ++k) {
    double x[3], xl[3], y[16];
    for (int a = 0; a < 3; ++a) x[a] = o[a] + t * d[a];
    local_coords(s, idx, x, xl);
    kno_sdf_eval(s, cell_index(s, idx), xl, y, NULL);
    double f = y[0];
    r->steps = k + 1;
    if (f < r->fmin) r->fmin = f;
    if (f < eps) {
      r->status = KNO_HIT;
      r->t = t;
      r->t_entry = t_entry;
      memcpy(r->cell, idx, sizeof(idx));
      return;
    }
    int ax;
    double t_exit = fmax(t, cell_exit(s, o, d, idx, &ax));
    if (t + f < t_exit) {
      t = t + f;
      if (t > tf) {   /* past the end of the interval inside a cell (an interval cut short) */
        r->status = KNO_EXIT_MISS;
        r->t = t;
        return;
      }
    } else if (step_mode == KNO_STEP_UNCLAMPED) {
      t = t + f;
      t_entry = t;
      if (t > tf) {
        r->status = KNO_EXIT_MISS;
        r->t = t;
        return;
      }
      cell_at(s, o, d, t, idx);
    } else {
      t = t_exit;
      idx[ax] += d[ax] > 0 ? 1 : -1;
      t_entry = t;
      if (idx[ax] < 0 || idx[ax] >= s->N || t > tf) {
        r->status = KNO_EXIT_MISS;
        r->t = t;
        return;
      }
    }
  }
  r->status = KNO_BUDGET_MISS;
  r->t = t;
}

/* Shading of a hit (Sec. 3.4.1).  Two guarded Newton steps along the ray on
 * f(o + t d) refine the hit inside its cell (t stays within the cell's
 * [entry, exit] interval; a step is taken only when the directional
 * derivative is below -1e-3).  At the refined point: depth = t, the normal
 * is the normalised world-space SDF gradient of the hit cell's MLP (-d if
 * the gradient vanishes), and the color MLP gets x_local, gamma_4(d), n, z. */
void kno_shade(const kno_scene* s, const double o[3], const double d[3],
               const kno_trace_result* r, double* depth, double normal[3], double rgb[3],
               double z[15]) {
  const int idx[3] = {r->cell[0], r->cell[1], r->cell[2]};
  const int cell = cell_index(s, idx);
  double half[3];
  for (int a = 0; a < 3; ++a) half[a] = 0.5 * cell_side(s, a);
  double t = r->t;
  double t_exit = cell_exit(s, o, d, idx, NULL);
  double x[3], xl[3], y[16], gl[3], g[3];
  for (int it = 0; it < 2; ++it) {
    for (int a = 0; a < 3; ++a) x[a] = o[a] + t * d[a];
    local_coords(s, idx, x, xl);
    kno_sdf_eval(s, cell, xl, y, gl);
    double gd = 0;
    for (int a = 0; a < 3; ++a) gd += gl[a] / half[a] * d[a];
    if (gd < -1e-3) {
      double tn = t - y[0] / gd;
      tn = fmax(tn, r->t_entry);
      tn = fmin(tn, t_exit);
      t = tn;
    }
  }
  for (int a = 0; a < 3; ++a) x[a] = o[a] + t * d[a];
  local_coords(s, idx, x, xl);
  kno_sdf_eval(s, cell, xl, y, gl);
  for (int a = 0; a < 3; ++a) g[a] = gl[a] / half[a];
  double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  if (gn < 1e-20) {
    for (int a = 0; a < 3; ++a) normal[a] = -d[a];
  } else {
    for (int a = 0; a < 3; ++a) normal[a] = g[a] / gn;
  }
  for (int i = 0; i < FEAT; ++i) z[i] = y[1 + i];
  kno_color_eval(s, cell, xl, d, normal, z, rgb);
  *depth = t;
}

/* One primary ray per pixel through the pixel center; outputs laid out
 * row-major, rgb and normal as [npix][3].  pixels == NULL renders the whole
 * image (npix must be width*height); otherwise only the listed pixels. */
void kno_render(const kno_scene* s, const kno_camera* c, const int64_t* pixels, int64_t npix,
                double* rgb, double* depth, double* normal, uint8_t* hit, int32_t* steps,
                int32_t* status, double* fmin, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t q = 0; q < npix; ++q) {
    int64_t p = pixels ? pixels[q] : q;
    int row = (int)(p / c->width), colm = (int)(p % c->width);
    double o[3], d[3];
    kno_camera_ray(c, row, colm, 0.5, 0.5, o, d);
    kno_trace_result r;
    kno_trace_mode(s, o, d, c->max_steps, c->eps, c->step_mode, &r);
    double dep = 0, n[3] = {0, 0, 0}, col[3], z[15];
    if (r.status == KNO_HIT) {
      kno_shade(s, o, d, &r, &dep, n, col, z);
    } else {
      for (int a = 0; a < 3; ++a) col[a] = c->background[a];
    }
    for (int a = 0; a < 3; ++a) {
      if (rgb) rgb[q * 3 + a] = col[a];
      if (normal) normal[q * 3 + a] = n[a];
    }
    if (depth) depth[q] = dep;
    if (hit) hit[q] = r.status == KNO_HIT;
    if (steps) steps[q] = r.steps;
    if (status) status[q] = r.status;
    if (fmin) fmin[q] = r.fmin;
  }
}

/* ------------------------------------------------------------------------
 * Path tracing (Sec. 3.4.1: the renderer is a path tracer; surfaces are
 * Lambertian, with the color MLP output as albedo).  Readings: cosine-
 * weighted scattering about the normal, throughput times albedo at each
 * scatter, at most `bounces` scatters, an escaping ray adds throughput times
 * the environment, a hit after the last scatter adds nothing; the pixel is
 * the mean of its samples.
 * ------------------------------------------------------------------------ */

/* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): ten rounds; each round multiplies counter
 * words 0 and 2 by the two round constants, keeps the low halves, and xors
 * the high halves with the other two words and the key; the key advances by
 * the two Weyl constants between rounds. */
void kno_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* uniform in [0, 1) from the top 24 bits */
static double u01(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* two uniforms of path (pixel, sample) at event k: Philox keyed by the seed,
 * counter (pixel, sample, k, 0); k = 0 is the pixel jitter, k >= 1 the k-th
 * scatter */
static void path_uniforms(uint64_t seed, int64_t pixel, int sample, int k, double* a, double* b) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const uint32_t ctr[4] = {(uint32_t)pixel, (uint32_t)sample, (uint32_t)k, 0u};
  uint32_t x[4];
  kno_philox4x32_10(ctr, key, x);
  *a = u01(x[0]);
  *b = u01(x[1]);
}

/* orthonormal basis (b1, b2, n) of a unit normal (Duff, Burgess, Christensen,
 * Hery, Kensler, Liani, Villemin, "Building an Orthonormal Basis,
 * Revisited", JCGT 2017) */
void kno_onb(const double n[3], double b1[3], double b2[3]) {
  const double sign = n[2] >= 0.0 ? 1.0 : -1.0;
  const double a = -1.0 / (sign + n[2]);
  const double b = n[0] * n[1] * a;
  b1[0] = 1.0 + sign * n[0] * n[0] * a;
  b1[1] = sign * b;
  b1[2] = -sign * n[0];
  b2[0] = b;
  b2[1] = sign + n[1] * n[1] * a;
  b2[2] = -n[1];
}

/* cosine-weighted direction about n from (u1, u2) in [0,1)^2: local
 * (sqrt(u1) cos 2 pi u2, sqrt(u1) sin 2 pi u2, sqrt(1 - u1)) */
void kno_cosine_dir(const double n[3], double u1, double u2, double out[3]) {
  double b1[3], b2[3];
  kno_onb(n, b1, b2);
  const double r = sqrt(u1), phi = 2.0 * PI * u2;
  const double lx = r * cos(phi), ly = r * sin(phi), lz = sqrt(1.0 - u1);
  for (int a = 0; a < 3; ++a) out[a] = lx * b1[a] + ly * b2[a] + lz * n[a];
}

/* equirectangular environment: u = 1/2 + atan2(d_x, -d_z) / 2 pi,
 * v = acos(d_y) / pi (row 0 looks up +y); bilinear between texel centres,
 * wrapping in u, clamping in v */
void kno_env_lookup(const kno_env* e, const double d[3], double rgb[3]) {
  if (!e->rgb || e->w <= 0 || e->h <= 0) {
    rgb[0] = rgb[1] = rgb[2] = 0.0;
    return;
  }
  const double dy = d[1] < -1.0 ? -1.0 : (d[1] > 1.0 ? 1.0 : d[1]);
  const double u = 0.5 + atan2(d[0], -d[2]) / (2.0 * PI);
  const double v = acos(dy) / PI;
  const double x = u * e->w - 0.5, y = v * e->h - 0.5;
  const double fx0 = floor(x), fy0 = floor(y);
  const double fx = x - fx0, fy = y - fy0;
  int x0 = (int)fx0 % e->w;
  if (x0 < 0) x0 += e->w;
  const int x1 = (x0 + 1) % e->w;
  int y0 = (int)fy0, y1 = (int)fy0 + 1;
  y0 = y0 < 0 ? 0 : (y0 > e->h - 1 ? e->h - 1 : y0);
  y1 = y1 < 0 ? 0 : (y1 > e->h - 1 ? e->h - 1 : y1);
  for (int c = 0; c < 3; ++c) {
    const double t00 = e->rgb[((size_t)y0 * e->w + x0) * 3 + c], t01 = e->rgb[((size_t)y0 * e->w + x1) * 3 + c];
    const double t10 = e->rgb[((size_t)y1 * e->w + x0) * 3 + c], t11 = e->rgb[((size_t)y1 * e->w + x1) * 3 + c];
    rgb[c] = (1.0 - fy) * ((1.0 - fx) * t00 + fx * t01) + fy * ((1.0 - fx) * t10 + fx * t11);
  }
}

/* One path from the camera; returns its radiance.  `first` (may be NULL)
 * receives the primary segment's trace and shading for the auxiliary
 * outputs. */
static void trace_path(const kno_scene* s, const kno_camera* c, const kno_pt* pt, int64_t p, int sample,
                       double L[3], kno_trace_result* first, double* first_depth, double first_n[3]) {
  const int row = (int)(p / c->width), colm = (int)(p % c->width);
  double xi1 = 0.5, xi2 = 0.5;
  if (pt->spp > 1 || pt->jitter) path_uniforms(pt->seed, p, sample, 0, &xi1, &xi2);
  double o[3], d[3];
  kno_camera_ray(c, row, colm, xi1, xi2, o, d);
  double T[3] = {1.0, 1.0, 1.0};
  L[0] = L[1] = L[2] = 0.0;
  for (int k = 0;; ++k) {
    kno_trace_result r;
    kno_trace_mode(s, o, d, c->max_steps, c->eps, c->step_mode, &r);
    if (k == 0 && first) *first = r;
    if (r.status != KNO_HIT) {
      double env[3];
      kno_env_lookup(&pt->env, d, env);
      for (int a = 0; a < 3; ++a) L[a] += T[a] * env[a];
      return;
    }
    double dep, n[3], rgb[3], z[15];
    kno_shade(s, o, d, &r, &dep, n, rgb, z);
    if (k == 0 && first_depth) {
      *first_depth = dep;
      for (int a = 0; a < 3; ++a) first_n[a] = n[a];
    }
    if (k >= pt->bounces) return;
    for (int a = 0; a < 3; ++a) T[a] *= rgb[a];
    double u1, u2, nd[3];
    path_uniforms(pt->seed, p, sample, k + 1, &u1, &u2);
    kno_cosine_dir(n, u1, u2, nd);
    for (int a = 0; a < 3; ++a) {
      o[a] = o[a] + dep * d[a] + 1e-3 * n[a];
      d[a] = nd[a];
    }
  }
}

void kno_path_trace(const kno_scene* s, const kno_camera* c, const kno_pt* pt, const int64_t* pixels,
                    int64_t npix, double* rgb, double* depth, double* normal, uint8_t* hit, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
  for (int64_t q = 0; q < npix; ++q) {
    const int64_t p = pixels ? pixels[q] : q;
    double acc[3] = {0.0, 0.0, 0.0};
    kno_trace_result first;
    double dep = 0.0, n[3] = {0.0, 0.0, 0.0};
    for (int smp = 0; smp < pt->spp; ++smp) {
      double L[3];
      trace_path(s, c, pt, p, smp, L, smp == 0 ? &first : NULL, smp == 0 ? &dep : NULL,
                 smp == 0 ? n : NULL);
      for (int a = 0; a < 3; ++a) acc[a] += L[a];
    }
    const int h = first.status == KNO_HIT;
    for (int a = 0; a < 3; ++a) {
      if (rgb) rgb[q * 3 + a] = acc[a] / pt->spp;
      if (normal) normal[q * 3 + a] = h ? n[a] : 0.0;
    }
    if (depth) depth[q] = h ? dep : 0.0;
    if (hit) hit[q] = (uint8_t)h;
  }
}

/* ------------------------------------------------------------------------
 * Shared scenes (Sec. 3.4: the path tracer renders KiloNeuS objects next to
 * classic primitives; for each ray it finds the closest intersection with an
 * object's bounding volume, and inside a KiloNeuS object's box it
 * sphere-traces the neural surface).  Readings:
 *   - primitives are Lambertian spheres, axis-aligned boxes and triangles,
 *     two-sided: the shading normal faces the incoming ray;
 *   - a KiloNeuS instance is its scene placed by a uniform scale s > 0 and a
 *     translation T (world x = T + s x_local); its MLPs see local
 *     coordinates, so the local ray is ((o - T) / s, d) and a local
 *     parameter t' is the world distance s t'; instance boxes are disjoint;
 *   - a ray's next object is the nearest of: the closest primitive hit past
 *     t_prim_min, and the entry of each instance box that starts at or past
 *     t_inst_min (ties go to the primitive, then the lower index);
 *   - an instance is sphere-traced from its entry to min(box exit, the
 *     closest primitive hit); a march that leaves this interval continues
 *     the ray from the box exit (t_inst_min = the exit); running out of
 *     steps ends the ray as a miss, as for a single object.
 * ------------------------------------------------------------------------ */

static void face_ray(double n[3], const double d[3]) {
  if (n[0] * d[0] + n[1] * d[1] + n[2] * d[2] > 0.0)
    for (int a = 0; a < 3; ++a) n[a] = -n[a];
}

int kno_prim_hit(const kno_prim* p, const double o[3], const double d[3], double t_min, double* t,
                 double n[3]) {
  if (p->kind == KNO_PRIM_SPHERE) {
    const double oc[3] = {o[0] - p->p[0], o[1] - p->p[1], o[2] - p->p[2]};
    const double r = p->p[3];
    const double b = oc[0] * d[0] + oc[1] * d[1] + oc[2] * d[2];
    const double c = oc[0] * oc[0] + oc[1] * oc[1] + oc[2] * oc[2] - r * r;
    const double disc = b * b - c;
    if (disc < 0.0) return 0;
    const double sq = sqrt(disc);
    double th = -b - sq;
    if (!(th > t_min)) th = -b + sq;
    if (!(th > t_min)) return 0;
    *t = th;
    for (int a = 0; a < 3; ++a) n[a] = (o[a] + th * d[a] - p->p[a]) / r;
    face_ray(n, d);
    return 1;
  }
  if (p->kind == KNO_PRIM_BOX) {
    double tn = -INFINITY, tf = INFINITY;
    int an = -1, af = -1;
    for (int a = 0; a < 3; ++a) {
      if (d[a] == 0.0) {
        if (o[a] < p->p[a] || o[a] > p->p[3 + a]) return 0;
        continue;
      }
      double t1 = (p->p[a] - o[a]) / d[a], t2 = (p->p[3 + a] - o[a]) / d[a];
      if (t1 > t2) {
        const double x = t1;
        t1 = t2;
        t2 = x;
      }
      if (t1 > tn) {
        tn = t1;
        an = a;
      }
      if (t2 < tf) {
        tf = t2;
        af = a;
      }
    }
    if (tn > tf) return 0;
    int ax;
    if (tn > t_min) {
      *t = tn;
      ax = an;
    } else if (tf > t_min) {
      *t = tf;
      ax = af;
    } else {
      return 0;
    }
    if (ax < 0) return 0;
    n[0] = n[1] = n[2] = 0.0;
    n[ax] = d[ax] > 0.0 ? -1.0 : 1.0;
    return 1;
  }
  if (p->kind == KNO_PRIM_TRIANGLE) {
    /* Moller-Trumbore */
    const double* A = p->p;
    const double e1[3] = {p->p[3] - A[0], p->p[4] - A[1], p->p[5] - A[2]};
    const double e2[3] = {p->p[6] - A[0], p->p[7] - A[1], p->p[8] - A[2]};
    double pv[3], qv[3], tv[3] = {o[0] - A[0], o[1] - A[1], o[2] - A[2]};
    cross3(d, e2, pv);
    const double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
    if (fabs(det) < 1e-300) return 0;
    const double inv = 1.0 / det;
    const double u = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    cross3(tv, e1, qv);
    const double v = (d[0] * qv[0] + d[1] * qv[1] + d[2] * qv[2]) * inv;
    if (v < 0.0 || u + v > 1.0) return 0;
    const double th = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
    if (!(th > t_min)) return 0;
    *t = th;
    cross3(e1, e2, n);
    normalize3(n);
    face_ray(n, d);
    return 1;
  }
  return 0;
}

typedef struct {
  int32_t kind;     /* KNO_OBJ_* */
  int32_t index;
  double t;         /* primitive hit, or instance entry (world) */
  double t_exit;    /* instance box exit (world) */
  double t_prim;    /* closest primitive hit (INFINITY if none) */
  double n[3];      /* primitive: facing normal */
} world_next;

static void instance_ray(const kno_instance* in, const double o[3], double ol[3]) {
  for (int a = 0; a < 3; ++a) ol[a] = (o[a] - in->translate[a]) / in->scale;
}

/* the ray's next object past t_prim_min (primitives) and t_inst_min
 * (instance entries) */
static void world_step(const kno_world* w, const double o[3], const double d[3], double t_prim_min,
                       double t_inst_min, world_next* r) {
  r->kind = KNO_OBJ_NONE;
  r->index = -1;
  r->t = INFINITY;
  r->t_prim = INFINITY;
  int pi = -1;
  double pn[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < w->n_prim; ++i) {
    double t, n[3];
    if (kno_prim_hit(&w->prim[i], o, d, t_prim_min, &t, n) && t < r->t_prim) {
      r->t_prim = t;
      pi = i;
      memcpy(pn, n, sizeof(pn));
    }
  }
  int ii = -1;
  double te = INFINITY, tx = 0.0;
  for (int k = 0; k < w->n_inst; ++k) {
    const kno_instance* in = &w->inst[k];
    double ol[3], tn, tf;
    instance_ray(in, o, ol);
    if (!kno_slab(in->scene, ol, d, &tn, &tf)) continue;
    const double entry = in->scale * fmax(tn, 0.0);
    if (entry < t_inst_min) continue;
    if (entry < te) {
      te = entry;
      tx = in->scale * tf;
      ii = k;
    }
  }
  if (pi >= 0 && r->t_prim <= te) {
    r->kind = KNO_OBJ_PRIM;
    r->index = pi;
    r->t = r->t_prim;
    memcpy(r->n, pn, sizeof(pn));
  } else if (ii >= 0) {
    r->kind = KNO_OBJ_INST;
    r->index = ii;
    r->t = te;
    r->t_exit = tx;
  }
}

/* the surface a world ray meets: kind, world t, normal, albedo (KiloNeuS:
 * the color MLP); first_* of the KiloNeuS march for diagnostics */
typedef struct {
  int32_t kind;     /* KNO_OBJ_NONE: escaped (or ran out of steps) */
  int32_t index;
  double t, n[3], albedo[3];
} world_hit;

static void world_trace(const kno_world* w, const kno_camera* c, const double o[3], const double d[3],
                        world_hit* h) {
  double t_prim_min = 0.0, t_inst_min = 0.0;
  h->kind = KNO_OBJ_NONE;
  h->index = -1;
  for (int guard = 0; guard <= w->n_inst; ++guard) {
    world_next nx;
    world_step(w, o, d, t_prim_min, t_inst_min, &nx);
    if (nx.kind == KNO_OBJ_NONE) return;
    if (nx.kind == KNO_OBJ_PRIM) {
      h->kind = KNO_OBJ_PRIM;
      h->index = nx.index;
      h->t = nx.t;
      memcpy(h->n, nx.n, sizeof(h->n));
      memcpy(h->albedo, w->prim[nx.index].albedo, sizeof(h->albedo));
      return;
    }
    const kno_instance* in = &w->inst[nx.index];
    double ol[3];
    instance_ray(in, o, ol);
    const double tfar = fmin(nx.t_exit, nx.t_prim) / in->scale;
    kno_trace_result r;
    trace_interval(in->scene, ol, d, nx.t / in->scale, tfar, c->max_steps, c->eps, c->step_mode, &r);
    if (r.status == KNO_HIT) {
      double dep, z[15];
      kno_shade(in->scene, ol, d, &r, &dep, h->n, h->albedo, z);
      h->kind = KNO_OBJ_INST;
      h->index = nx.index;
      h->t = in->scale * dep;
      return;
    }
    if (r.status != KNO_EXIT_MISS) return;   /* out of steps: a miss */
    t_inst_min = nx.t_exit;                  /* on past this instance's box */
  }
}

void kno_world_render(const kno_world* w, const kno_camera* c, const int64_t* pixels, int64_t npix,
                      double* rgb, double* depth, double* normal, uint8_t* hit, int32_t* object,
                      int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t q = 0; q < npix; ++q) {
    const int64_t p = pixels ? pixels[q] : q;
    double o[3], d[3];
    kno_camera_ray(c, (int)(p / c->width), (int)(p % c->width), 0.5, 0.5, o, d);
    world_hit h;
    world_trace(w, c, o, d, &h);
    const int on = h.kind != KNO_OBJ_NONE;
    for (int a = 0; a < 3; ++a) {
      if (rgb) rgb[q * 3 + a] = on ? h.albedo[a] : c->background[a];
      if (normal) normal[q * 3 + a] = on ? h.n[a] : 0.0;
    }
    if (depth) depth[q] = on ? h.t : 0.0;
    if (hit) hit[q] = (uint8_t)on;
    /* object id: -1 none, instance k as k, primitive i as -(2 + i) */
    if (object) object[q] = h.kind == KNO_OBJ_INST ? h.index : (h.kind == KNO_OBJ_PRIM ? -(2 + h.index) : -1);
  }
}

void kno_world_path_trace(const kno_world* w, const kno_camera* c, const kno_pt* pt, const int64_t* pixels,
                          int64_t npix, double* rgb, double* depth, double* normal, uint8_t* hit,
                          int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
  for (int64_t q = 0; q < npix; ++q) {
    const int64_t p = pixels ? pixels[q] : q;
    const int row = (int)(p / c->width), colm = (int)(p % c->width);
    double acc[3] = {0.0, 0.0, 0.0}, dep0 = 0.0, n0[3] = {0.0, 0.0, 0.0};
    int h0 = 0;
    for (int smp = 0; smp < pt->spp; ++smp) {
      double xi1 = 0.5, xi2 = 0.5;
      if (pt->spp > 1 || pt->jitter) path_uniforms(pt->seed, p, smp, 0, &xi1, &xi2);
      double o[3], d[3], T[3] = {1.0, 1.0, 1.0}, L[3] = {0.0, 0.0, 0.0};
      kno_camera_ray(c, row, colm, xi1, xi2, o, d);
      for (int k = 0;; ++k) {
        world_hit h;
        world_trace(w, c, o, d, &h);
        if (k == 0 && smp == 0) {
          h0 = h.kind != KNO_OBJ_NONE;
          dep0 = h0 ? h.t : 0.0;
          for (int a = 0; a < 3; ++a) n0[a] = h0 ? h.n[a] : 0.0;
        }
        if (h.kind == KNO_OBJ_NONE) {
          double env[3];
          kno_env_lookup(&pt->env, d, env);
          for (int a = 0; a < 3; ++a) L[a] += T[a] * env[a];
          break;
        }
        if (k >= pt->bounces) break;
        for (int a = 0; a < 3; ++a) T[a] *= h.albedo[a];
        double u1, u2, nd[3];
        path_uniforms(pt->seed, p, smp, k + 1, &u1, &u2);
        kno_cosine_dir(h.n, u1, u2, nd);
        for (int a = 0; a < 3; ++a) {
          o[a] = o[a] + h.t * d[a] + 1e-3 * h.n[a];
          d[a] = nd[a];
        }
      }
      for (int a = 0; a < 3; ++a) acc[a] += L[a];
    }
    for (int a = 0; a < 3; ++a) {
      if (rgb) rgb[q * 3 + a] = acc[a] / pt->spp;
      if (normal) normal[q * 3 + a] = n0[a];
    }
    if (depth) depth[q] = dep0;
    if (hit) hit[q] = (uint8_t)h0;
  }
}

/* ------------------------------------------------------------------------
 * Point-query workloads built on the per-cell evaluation (Sec. 3.3: the
 * cell MLPs are evaluated on per-cell batches of points).
 * ------------------------------------------------------------------------ */

/* SDF value, world-space gradient and feature of the global, piecewise
 * KiloSDF at world point x: the MLP of the cell that contains x (cell map m
 * of Sec. 3.1: floor of the box-relative position over the cell side,
 * clamped to the grid), in that cell's local frame. */
static void sdf_at_point(const kno_scene* s, const double x[3], double* d, double grad[3], double z[15]) {
  int idx[3];
  for (int a = 0; a < 3; ++a) {
    int i = (int)floor((x[a] - s->bmin[a]) / cell_side(s, a));
    idx[a] = i < 0 ? 0 : (i > s->N - 1 ? s->N - 1 : i);
  }
  double xl[3], y[16], gl[3];
  local_coords(s, idx, x, xl);
  kno_sdf_eval(s, cell_index(s, idx), xl, y, grad ? gl : NULL);
  *d = y[0];
  if (grad)
    for (int a = 0; a < 3; ++a) grad[a] = gl[a] / (0.5 * cell_side(s, a));
  if (z)
    for (int i = 0; i < FEAT; ++i) z[i] = y[1 + i];
}

void kno_query(const kno_scene* s, const double* pts, int64_t n, double* d, double* grad, double* z,
               int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
  for (int64_t q = 0; q < n; ++q)
    sdf_at_point(s, pts + 3 * q, d + q, grad ? grad + 3 * q : NULL, z ? z + 15 * q : NULL);
}

/* Dense lattice sampling of the KiloSDF, the input of marching-cubes mesh
 * extraction (Sec. 4.1 extracts meshes at resolution 512).  Lattice point
 * (i, j, k), 0 <= i, j, k < R, lies at bmin + (bmax - bmin) (i, j, k) / (R - 1).
 * Its cell along an axis is floor(i N / (R - 1)) in integer arithmetic,
 * clamped to N - 1, so the last lattice plane (on the box face) belongs to
 * the last cell and a lattice point on an inner cell face to the cell above
 * it, as floor() of the exact position would give.  The point is evaluated
 * with that cell's MLP in the cell's local frame.  `lin` lists flattened
 * indices i + R (j + R k); outputs are per listed point. */
void kno_grid_sample(const kno_scene* s, int R, const int64_t* lin, int64_t n, double* d, double* grad,
                     double* z, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
  for (int64_t q = 0; q < n; ++q) {
    const int64_t l = lin[q];
    const int64_t ijk[3] = {l % R, (l / R) % R, l / ((int64_t)R * R)};
    int idx[3];
    double x[3];
    for (int a = 0; a < 3; ++a) {
      const int64_t c = ijk[a] * s->N / (R - 1);
      idx[a] = (int)(c > s->N - 1 ? s->N - 1 : c);
      x[a] = s->bmin[a] + (s->bmax[a] - s->bmin[a]) * (double)ijk[a] / (double)(R - 1);
    }
    double xl[3], y[16], gl[3];
    local_coords(s, idx, x, xl);
    kno_sdf_eval(s, cell_index(s, idx), xl, y, grad ? gl : NULL);
    d[q] = y[0];
    if (grad)
      for (int a = 0; a < 3; ++a) grad[3 * q + a] = gl[a] / (0.5 * cell_side(s, a));
    if (z)
      for (int i = 0; i < FEAT; ++i) z[15 * q + i] = y[1 + i];
  }
}

/* Eikonal term by central finite differences (Sec. 3.2, the eikonal loss;
 * Sec. 3.3 explains that the gradient is taken by finite differences of the
 * global piecewise SDF rather than by autodiff of single cell MLPs, which
 * is what couples neighbouring cells at their seams).  For each point x:
 * g_a = (d(x + delta e_a) - d(x - delta e_a)) / (2 delta), a = x, y, z, each
 * of the six stencil values taken with the MLP of the cell that contains the
 * stencil point; gnorm = |g|; the loss is the mean of (gnorm - 1)^2 over the
 * points.  stencil (may be NULL) receives the six values per point in the
 * order (+x, -x, +y, -y, +z, -z). */
void kno_eikonal_fd(const kno_scene* s, const double* pts, int64_t n, double delta, double* gnorm,
                    double* stencil, double* loss, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
  for (int64_t q = 0; q < n; ++q) {
    double g2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      double xp[3] = {pts[3 * q], pts[3 * q + 1], pts[3 * q + 2]};
      double xm[3] = {pts[3 * q], pts[3 * q + 1], pts[3 * q + 2]};
      xp[a] += delta;
      xm[a] -= delta;
      double dp, dm;
      sdf_at_point(s, xp, &dp, NULL, NULL);
      sdf_at_point(s, xm, &dm, NULL, NULL);
      if (stencil) {
        stencil[6 * q + 2 * a] = dp;
        stencil[6 * q + 2 * a + 1] = dm;
      }
      const double ga = (dp - dm) / (2.0 * delta);
      g2 += ga * ga;
    }
    gnorm[q] = sqrt(g2);
  }
  double acc = 0.0;
  for (int64_t q = 0; q < n; ++q) acc += (gnorm[q] - 1.0) * (gnorm[q] - 1.0);
  *loss = n > 0 ? acc / (double)n : 0.0;
}
