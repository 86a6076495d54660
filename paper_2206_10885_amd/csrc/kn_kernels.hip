// HIP kernels of the KiloNeuS rendering hot path for gfx950 (MI355X).
//
// Wavefront design (one frame):
//   k_raygen   pinhole rays, box clip (Sec. 3.4.1), entry cell, box misses
//   per round: k_scan    per-cell exclusive scan -> bin starts, work chunks
//              k_scatter counting sort of the round's rays by global cell
//                        (first round: per ray; later rounds: per chunk and
//                        exit face)
//              k_march   one work item per chunk (<= 256 rays) of a cell's
//                        bin: the cell's MLP weights (MFMA fragments) and the
//                        rays are staged in LDS; the waves step 16-ray tiles
//                        in passes over an LDS active list while rays stay in
//                        the cell; rays leaving for a neighbour cell are
//                        written to the chunk's own output range, grouped by
//                        exit face (no global list counter); hits are written
//                        to a list indexed by ray id
//   after the rounds: hits are binned by cell the same way, then k_shade
//              refines each hit with two Newton steps (value and the
//              directional derivative along the ray), takes the normalised
//              analytic gradient (value + 3 tangent columns per hit) and runs
//              the color MLP (Sec. 3.1 eq. 4).
#include "kn_device.h"
#include "kn_launch.h"

namespace kn {

constexpr uint32_t kInvalidKey = 0xFFFFFFFFu;  // record without a cell (box miss, no hit)

// ---------------------------------------------------------------------------
// wave-aggregated atomics
// ---------------------------------------------------------------------------
__device__ __forceinline__ void atomic_count_grouped(uint32_t* arr, uint32_t cs, uint32_t key, bool valid) {
  uint64_t todo = __ballot(valid);
  while (todo) {
    int leader = __ffsll((unsigned long long)todo) - 1;
    uint32_t lk = __shfl(key, leader);
    uint64_t grp = __ballot(valid && key == lk);
    if (lane_id() == leader) atomicAdd(&arr[(size_t)lk * cs], (uint32_t)__popcll(grp));
    todo &= ~grp;
  }
}

// Reserves a slot in arr[key * cs] for every valid lane.  The lanes are grouped by
// key first (ballots only); then each group's first lane adds the group's size
// with one atomic, all groups in the same instruction, so the wave waits for
// a single round trip however many keys it holds.
__device__ __forceinline__ uint32_t atomic_slot_grouped(uint32_t* arr, uint32_t cs, uint32_t key, bool valid) {
  const int lane = lane_id();
  uint64_t todo = __ballot(valid);
  int leader = lane;
  uint32_t rank = 0, size = 0;
  while (todo) {
    const int l = __ffsll((unsigned long long)todo) - 1;
    const uint32_t lk = __shfl(key, l);
    const bool mine = valid && key == lk;
    const uint64_t grp = __ballot(mine);
    if (mine) {
      leader = l;
      rank = lane_rank(grp);
    }
    if (lane == l) size = (uint32_t)__popcll(grp);
    todo &= ~grp;
  }
  uint32_t base = 0;
  if (valid && lane == leader) base = atomicAdd(&arr[(size_t)key * cs], size);
  base = (uint32_t)__shfl((int)base, leader);
  return base + rank;
}

// Adds the workgroup's count of `flag` to *counter with one global atomic
// (a single hot address must not take one atomic per wave).  Called by
// every thread of the workgroup.
__device__ __forceinline__ void wg_count(uint32_t* counter, bool flag, uint32_t* s_tmp) {
  if (threadIdx.x == 0) *s_tmp = 0u;
  __syncthreads();
  const uint64_t m = __ballot(flag);
  if (lane_id() == 0 && m) atomicAdd(s_tmp, (uint32_t)__popcll(m));
  __syncthreads();
  if (threadIdx.x == 0 && *s_tmp) atomicAdd(counter, *s_tmp);
}

__device__ __forceinline__ void write_miss(const OutPtrs& o, uint32_t pix, int steps, float t,
                                           float t_entry, int32_t cell, int32_t status, bool rgb = true) {
  if (rgb) {
    gmem(o.rgb)[3 * pix + 0] = o.bg[0];
    gmem(o.rgb)[3 * pix + 1] = o.bg[1];
    gmem(o.rgb)[3 * pix + 2] = o.bg[2];
  }
  if (o.depth) gmem(o.depth)[pix] = 0.0f;
  if (o.normal) {
    gmem(o.normal)[3 * pix + 0] = 0.0f;
    gmem(o.normal)[3 * pix + 1] = 0.0f;
    gmem(o.normal)[3 * pix + 2] = 0.0f;
  }
  if (o.hit) gmem(o.hit)[pix] = 0;
  if (o.steps) gmem(o.steps)[pix] = (uint16_t)steps;
  if (o.trace) {
    auto tr = gmem(o.trace + pix);
    tr->t_march = t;
    tr->t_entry = t_entry;
    tr->cell = cell;
    tr->status = status;
  }
}

// ---------------------------------------------------------------------------
// ray generation: one thread per pixel
// ---------------------------------------------------------------------------
// Pixel of position t (< W H) in tile order: bands of 16 rows, each cut into
// strips of 16 columns (the last band and strip narrower) taken row by row,
// so a workgroup's 256 positions cover a 16 x 16 tile and a wave's 64 a
// 16 x 4 one.  Rays binned together then enter the grid through few cells,
// so far fewer per-cell atomics of the count and of the first scatter meet
// at one address than with whole rows.
__device__ __forceinline__ uint32_t tile_order_pixel(uint32_t t, uint32_t W, uint32_t H) {
  const uint32_t band = t / (16u * W), row0 = 16u * band;
  const uint32_t hb = min(16u, H - row0);
  const uint32_t o = t - 16u * W * band;
  const uint32_t s = o / (16u * hb), col0 = 16u * s;
  const uint32_t ws = min(16u, W - col0);
  const uint32_t q = o - 16u * hb * s;
  return (row0 + q / ws) * W + col0 + q % ws;
}

// Primary rays: position t takes pixel tile_order_pixel(t); t is also the
// ray's place in U and, offset by rid_base, its id.
__global__ __launch_bounds__(256) void k_raygen(RaygenArgs a) {
  const uint32_t npix = (uint32_t)a.W * (uint32_t)a.Hh;
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  const bool valid = t < npix;
  const uint32_t pix = valid ? tile_order_pixel(t, (uint32_t)a.W, (uint32_t)a.Hh) : 0u;
  const SceneGeom& sg = a.sg;
  uint32_t cell = 0;
  bool inbox = false;
  float t0 = 0.0f, tf = 0.0f;
  float d[3] = {0, 0, 0};
  if (valid) {
    const int row = (int)(pix / (uint32_t)a.W), col = (int)(pix % (uint32_t)a.W);
    const uint32_t rid = a.rid_base + t;
    const float u = (2.0f * ((float)col + 0.5f) / (float)a.W - 1.0f) * a.tx;
    const float v = (1.0f - 2.0f * ((float)row + 0.5f) / (float)a.Hh) * a.ty;
    float n2 = 0.0f;
    for (int k = 0; k < 3; ++k) {
      d[k] = a.fwd[k] + u * a.right[k] + v * a.up[k];
      n2 += d[k] * d[k];
    }
    const float inv = 1.0f / sqrtf(n2);
    for (int k = 0; k < 3; ++k) d[k] *= inv;
    // slab test against the box
    float tn = -INFINITY;
    tf = INFINITY;
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
      if (d[k] != 0.0f) {
        float t1 = (sg.bmin[k] - a.eye[k]) / d[k], t2 = (sg.bmax[k] - a.eye[k]) / d[k];
        tn = fmaxf(tn, fminf(t1, t2));
        tf = fminf(tf, fmaxf(t1, t2));
      } else if (a.eye[k] < sg.bmin[k] || a.eye[k] > sg.bmax[k]) {
        ok = false;
      }
    }
    inbox = ok && tn <= tf && tf > 0.0f;
    if (inbox) {
      t0 = fmaxf(tn, 0.0f);
      int idx[3];
      for (int k = 0; k < 3; ++k) {
        int i = (int)floorf((a.eye[k] + t0 * d[k] - sg.bmin[k]) * sg.inv_side[k]);
        idx[k] = min(max(i, 0), sg.N - 1);
      }
      cell = sg.cell_base + (uint32_t)(idx[0] + sg.N * (idx[1] + sg.N * idx[2]));
      a.rs[rid] = RayStatic{a.eye[0], a.eye[1], a.eye[2], tf, d[0], d[1], d[2],
                            (a.slot << kPixBits) | pix};
      a.U[t] = RayRec{t0, t0, cell, rid};
    } else {
      a.U[t] = RayRec{0.0f, 0.0f, kInvalidKey, rid};
      write_miss(a.out, pix, 0, 0.0f, 0.0f, -1, kBoxMiss);
    }
  }
  atomic_count_grouped(a.counts, a.cs, cell, inbox);
  __shared__ uint32_t s_cnt;
  wg_count(&a.miss_done[a.slot], valid && !inbox, &s_cnt);
}

// Box clip of a ray (slab method); false when the ray misses the box.
__device__ __forceinline__ bool slab(const SceneGeom& sg, const float o[3], const float d[3], float* t0, float* t1) {
  float tn = -INFINITY, tf = INFINITY;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (d[k] != 0.0f) {
      const float a = (sg.bmin[k] - o[k]) / d[k], b = (sg.bmax[k] - o[k]) / d[k];
      tn = fmaxf(tn, fminf(a, b));
      tf = fminf(tf, fmaxf(a, b));
    } else if (o[k] < sg.bmin[k] || o[k] > sg.bmax[k]) {
      ok = false;
    }
  }
  *t0 = fmaxf(tn, 0.0f);
  *t1 = tf;
  return ok && tn <= tf && tf > 0.0f;
}

__device__ __forceinline__ uint32_t entry_cell(const SceneGeom& sg, const float o[3], const float d[3], float t) {
  int idx[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int i = (int)floorf((o[k] + t * d[k] - sg.bmin[k]) * sg.inv_side[k]);
    idx[k] = min(max(i, 0), sg.N - 1);
  }
  return sg.cell_base + (uint32_t)(idx[0] + sg.N * (idx[1] + sg.N * idx[2]));
}

// Path tracing: one thread per path (pixel, sample); pool ray id = path id.
// Samples other than the pixel centre are jittered by Philox event 0.
__global__ __launch_bounds__(256) void k_raygen_pt(RaygenPtArgs a) {
  const uint32_t npath = (uint32_t)a.W * (uint32_t)a.Hh * a.spp;
  const uint32_t id = blockIdx.x * 256u + threadIdx.x;
  const bool valid = id < npath;
  uint32_t cell = 0;
  bool inbox = false;
  if (valid) {
    const uint32_t pix = id / a.spp, smp = id % a.spp;
    const int row = (int)(pix / (uint32_t)a.W), col = (int)(pix % (uint32_t)a.W);
    float xi1 = 0.5f, xi2 = 0.5f;
    if (a.spp > 1 || a.jitter) path_uniforms(a.seed_lo, a.seed_hi, pix, a.sample_offset + smp, 0u, &xi1, &xi2);
    const float u = (2.0f * ((float)col + xi1) / (float)a.W - 1.0f) * a.tx;
    const float v = (1.0f - 2.0f * ((float)row + xi2) / (float)a.Hh) * a.ty;
    float d[3], n2 = 0.0f;
    for (int k = 0; k < 3; ++k) {
      d[k] = a.fwd[k] + u * a.right[k] + v * a.up[k];
      n2 += d[k] * d[k];
    }
    const float inv = 1.0f / sqrtf(n2);
    for (int k = 0; k < 3; ++k) d[k] *= inv;
    float t0, tf;
    inbox = slab(a.sg, a.eye, d, &t0, &tf);
    PathRec pr{{1.0f, 1.0f, 1.0f}, {0.0f, 0.0f, 0.0f}, 0u, 0u};
    if (a.out.seg) {
      SegRec* sr = a.out.seg + (size_t)id * (a.bounces + 1u);
      for (uint32_t k = 0; k <= a.bounces; ++k)
        sr[k] = SegRec{{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}, 0.0f, 0.0f, 0.0f, {0.0f, 0.0f, 0.0f},
                       {0.0f, 0.0f, 0.0f}, -1, -1, 0u, {0u, 0u}};
      sr[0].o[0] = a.eye[0]; sr[0].o[1] = a.eye[1]; sr[0].o[2] = a.eye[2];
      sr[0].d[0] = d[0]; sr[0].d[1] = d[1]; sr[0].d[2] = d[2];
      if (!inbox) sr[0].status = kBoxMiss;
    }
    if (inbox) {
      cell = entry_cell(a.sg, a.eye, d, t0);
      a.rs[id] = RayStatic{a.eye[0], a.eye[1], a.eye[2], tf, d[0], d[1], d[2], (a.slot << kPixBits) | pix};
      a.U[id] = RayRec{t0, t0, cell, id};
    } else {
      a.U[id] = RayRec{0.0f, 0.0f, kInvalidKey, id};
      env_lookup(a.env, a.env_w, a.env_h, d, pr.L);
      if (smp == 0) write_miss(a.out, pix, 0, 0.0f, 0.0f, -1, kBoxMiss, false);
    }
    a.path[id] = pr;
  }
  atomic_count_grouped(a.counts, a.cs, cell, inbox);
  __shared__ uint32_t s_cnt;
  wg_count(&a.miss_done[a.slot], valid && !inbox, &s_cnt);
}

// ---------------------------------------------------------------------------
// Shared scenes (Sec. 3.4): Lambertian primitives and KiloNeuS instances.
// A world ray goes to its nearest object: the closest primitive hit past
// tpm, or the nearest instance box entered at or past tim (ties to the
// primitive, then the lower index).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void face_ray(float n[3], const float d[3]) {
  if (n[0] * d[0] + n[1] * d[1] + n[2] * d[2] > 0.0f)
    for (int k = 0; k < 3; ++k) n[k] = -n[k];
}

// closest hit of primitive p past t_min: t and the normal facing the ray
__device__ bool prim_hit(const PrimDev& p, const float o[3], const float d[3], float t_min, float* t,
                         float n[3]) {
  if (p.kind == 1u) {   // sphere
    // roots of t^2 + 2 b t + c (unit d).  In float32, b^2 - c cancels near
    // the silhouette; r^2 - |oc - b d|^2 is the same discriminant without
    // that cancellation.  The root of larger magnitude is q = -(b + sign(b)
    // sqrt(disc)), the other c / q (their product is c).
    const float oc[3] = {o[0] - p.p[0], o[1] - p.p[1], o[2] - p.p[2]};
    const float r = p.p[3];
    const float b = oc[0] * d[0] + oc[1] * d[1] + oc[2] * d[2];
    const float l[3] = {oc[0] - b * d[0], oc[1] - b * d[1], oc[2] - b * d[2]};
    const float disc = r * r - (l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
    if (disc < 0.0f) return false;
    const float c = oc[0] * oc[0] + oc[1] * oc[1] + oc[2] * oc[2] - r * r;
    const float q = -(b + copysignf(sqrtf(disc), b));
    const float t2 = q != 0.0f ? c / q : q;
    float th = fminf(q, t2);
    if (!(th > t_min)) th = fmaxf(q, t2);
    if (!(th > t_min)) return false;
    *t = th;
    for (int k = 0; k < 3; ++k) n[k] = (o[k] + th * d[k] - p.p[k]) / r;
    face_ray(n, d);
    return true;
  }
  if (p.kind == 2u) {   // axis-aligned box
    float tn = -INFINITY, tf = INFINITY;
    int an = -1, af = -1;
    for (int k = 0; k < 3; ++k) {
      if (d[k] == 0.0f) {
        if (o[k] < p.p[k] || o[k] > p.p[3 + k]) return false;
        continue;
      }
      float t1 = (p.p[k] - o[k]) / d[k], t2 = (p.p[3 + k] - o[k]) / d[k];
      if (t1 > t2) {
        const float x = t1;
        t1 = t2;
        t2 = x;
      }
      if (t1 > tn) {
        tn = t1;
        an = k;
      }
      if (t2 < tf) {
        tf = t2;
        af = k;
      }
    }
    if (tn > tf) return false;
    int ax;
    if (tn > t_min) {
      *t = tn;
      ax = an;
    } else if (tf > t_min) {
      *t = tf;
      ax = af;
    } else {
      return false;
    }
    if (ax < 0) return false;
    n[0] = n[1] = n[2] = 0.0f;
    n[ax] = d[ax] > 0.0f ? -1.0f : 1.0f;
    return true;
  }
  if (p.kind == 3u) {   // triangle (Moller-Trumbore)
    const float e1[3] = {p.p[3] - p.p[0], p.p[4] - p.p[1], p.p[5] - p.p[2]};
    const float e2[3] = {p.p[6] - p.p[0], p.p[7] - p.p[1], p.p[8] - p.p[2]};
    const float tv[3] = {o[0] - p.p[0], o[1] - p.p[1], o[2] - p.p[2]};
    const float pv[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    const float det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
    if (det == 0.0f) return false;
    const float inv = 1.0f / det;
    const float u = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
    if (u < 0.0f || u > 1.0f) return false;
    const float qv[3] = {tv[1] * e1[2] - tv[2] * e1[1], tv[2] * e1[0] - tv[0] * e1[2], tv[0] * e1[1] - tv[1] * e1[0]};
    const float v = (d[0] * qv[0] + d[1] * qv[1] + d[2] * qv[2]) * inv;
    if (v < 0.0f || u + v > 1.0f) return false;
    const float th = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
    if (!(th > t_min)) return false;
    *t = th;
    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const float nl = 1.0f / sqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int k = 0; k < 3; ++k) n[k] *= nl;
    face_ray(n, d);
    return true;
  }
  return false;
}

// camera rays of a world render (one per path) into the first world list
__global__ __launch_bounds__(256) void k_world_raygen(WorldRaygenArgs a, uint32_t npath) {
  const uint32_t id = blockIdx.x * 256u + threadIdx.x;
  if (id >= npath) return;
  const uint32_t pix = id / a.spp, smp = id % a.spp;
  const int row = (int)(pix / (uint32_t)a.W), col = (int)(pix % (uint32_t)a.W);
  float xi1 = 0.5f, xi2 = 0.5f;
  if (a.pt && (a.spp > 1 || a.jitter)) path_uniforms(a.seed_lo, a.seed_hi, pix, a.sample_offset + smp, 0u, &xi1, &xi2);
  const float u = (2.0f * ((float)col + xi1) / (float)a.W - 1.0f) * a.tx;
  const float v = (1.0f - 2.0f * ((float)row + xi2) / (float)a.Hh) * a.ty;
  float d[3], n2 = 0.0f;
  for (int k = 0; k < 3; ++k) {
    d[k] = a.fwd[k] + u * a.right[k] + v * a.up[k];
    n2 += d[k] * d[k];
  }
  const float inv = 1.0f / sqrtf(n2);
  WorldRec w;
  for (int k = 0; k < 3; ++k) {
    w.o[k] = a.eye[k];
    w.d[k] = d[k] * inv;
  }
  w.tpm = 0.0f;
  w.tim = 0.0f;
  w.rid = id;
  w.pad[0] = w.pad[1] = w.pad[2] = 0u;
  a.out[id] = w;
  if (a.pt) a.path[id] = PathRec{{1.0f, 1.0f, 1.0f}, {0.0f, 0.0f, 0.0f}, 0u, 0u};
}

// Each record: its next object.  A primitive hit is shaded here (primary:
// the outputs; path tracing: albedo, scatter, and the loop goes on in this
// thread); an escape ends the path (environment); an instance entry becomes
// a march record of the next round, in the instance's local frame, marched
// from the box entry to the nearer of the box exit and the primitive hit.
__global__ __launch_bounds__(256) void k_world_step(WorldStepArgs a) {
  __shared__ uint32_t s_cnt;
  const uint32_t n = a.n_dev ? *a.n_dev : a.n;
  const int lane = lane_id();
  const ReqEnt& qr = a.tabs.reqs[0];   // world renders are one request (slot 0)
  for (uint32_t base = blockIdx.x * 256u; base < n; base += gridDim.x * 256u) {
    const uint32_t i = base + threadIdx.x;
    bool spawn = false, finished = false;
    uint32_t ncell = 0;
    RayRec nrec{0, 0, 0, 0};
    if (i < n) {
      const ReqEnt q = qr;
      WorldRec w = a.in[i];
      const uint32_t rid = w.rid, pix = q.pt ? rid / q.spp : rid, smp = q.pt ? rid % q.spp : 0u;
      PathRec pr;
      if (q.pt) pr = a.tabs.path[rid];
      for (;;) {
        // the nearest primitive hit and instance entry
        float tp = INFINITY, pn[3] = {0.0f, 0.0f, 0.0f};
        int pi = -1;
        for (uint32_t k = 0; k < a.n_prims; ++k) {
          float th, nn[3];
          if (prim_hit(a.prims[k], w.o, w.d, w.tpm, &th, nn) && th < tp) {
            tp = th;
            pi = (int)k;
            pn[0] = nn[0];
            pn[1] = nn[1];
            pn[2] = nn[2];
          }
        }
        float te = INFINITY, tx = 0.0f, ol[3] = {0.0f, 0.0f, 0.0f};
        int ii = -1;
        for (uint32_t k = 0; k < a.tabs.n_scenes; ++k) {
          const SceneEnt& se = a.tabs.scenes[k];
          float l[3], tn, tf;
          for (int c = 0; c < 3; ++c) l[c] = (w.o[c] - se.wt[c]) / se.ws;
          if (!slab(se.sg, l, w.d, &tn, &tf)) continue;
          const float entry = se.ws * fmaxf(tn, 0.0f);
          if (entry < w.tim || !(entry < te)) continue;
          te = entry;
          tx = se.ws * tf;
          ii = (int)k;
          ol[0] = l[0];
          ol[1] = l[1];
          ol[2] = l[2];
        }
        const bool first = !q.pt || (pr.bounce == 0 && smp == 0);
        if (ii >= 0 && !(pi >= 0 && tp <= te)) {
          // into instance ii: a march record for the next round
          const SceneEnt& se = a.tabs.scenes[ii];
          const float t0 = te / se.ws, tfar = fminf(tx, tp) / se.ws;
          ncell = entry_cell(se.sg, ol, w.d, t0);
          a.rs[rid] = RayStatic{ol[0], ol[1], ol[2], tfar, w.d[0], w.d[1], w.d[2], pix};
          a.ws[rid] = WState{{w.o[0], w.o[1], w.o[2]}, w.tpm};
          nrec = RayRec{t0, t0, ncell, rid};
          spawn = true;
          break;
        }
        if (pi < 0) {
          // the ray escapes
          if (q.pt) {
            float e[3];
            env_lookup(q.env, q.env_w, q.env_h, w.d, e);
            for (int c = 0; c < 3; ++c) pr.L[c] += pr.T[c] * e[c];
          }
          if (first) write_miss(q.out, pix, 0, 0.0f, 0.0f, -1, kBoxMiss, !q.pt);
          finished = true;
          break;
        }
        // a primitive hit
        const PrimDev& pm = a.prims[pi];
        if (first) {
          const OutPtrs& out = q.out;
          if (!q.pt) {
            gmem(out.rgb)[3 * pix + 0] = pm.albedo[0];
            gmem(out.rgb)[3 * pix + 1] = pm.albedo[1];
            gmem(out.rgb)[3 * pix + 2] = pm.albedo[2];
          }
          if (out.depth) gmem(out.depth)[pix] = tp;
          if (out.normal) {
            gmem(out.normal)[3 * pix + 0] = pn[0];
            gmem(out.normal)[3 * pix + 1] = pn[1];
            gmem(out.normal)[3 * pix + 2] = pn[2];
          }
          if (out.hit) gmem(out.hit)[pix] = 1;
          if (out.steps) gmem(out.steps)[pix] = 0;
          if (out.trace) {
            auto tr = gmem(out.trace + pix);
            tr->t_march = tp;
            tr->t_entry = tp;
            tr->cell = -(2 + pi);
            tr->status = kHit;
          }
        }
        if (!q.pt || pr.bounce >= q.bounces) {
          finished = true;
          break;
        }
        // scatter off the primitive and go on from 1e-3 off its surface
        for (int c = 0; c < 3; ++c) pr.T[c] *= pm.albedo[c];
        float u1, u2, nd[3];
        path_uniforms(q.seed_lo, q.seed_hi, pix, q.sample_offset + smp, pr.bounce + 1u, &u1, &u2);
        cosine_dir(pn, u1, u2, nd);
        for (int c = 0; c < 3; ++c) {
          w.o[c] = w.o[c] + tp * w.d[c] + 1e-3f * pn[c];
          w.d[c] = nd[c];
        }
        w.tpm = 0.0f;
        w.tim = 0.0f;
        ++pr.bounce;
      }
      if (q.pt) a.tabs.path[rid] = pr;
    }
    // one reservation per wave of exactly its spawns (the list holds at most
    // one record per ray)
    const uint64_t sm = __ballot(spawn);
    const uint32_t ns = (uint32_t)__popcll(sm);
    if (ns) {
      uint32_t b = 0;
      if (lane == 0) b = atomicAdd(a.n_spawn, ns);
      b = __shfl(b, 0);
      if (spawn) a.spawn[b + lane_rank(sm)] = nrec;
    }
    atomic_count_grouped(a.counts_next, a.cs, ncell, spawn);
    wg_count(&a.tabs.miss_done[0], finished, &s_cnt);
  }
}

// Path tracing: pixel = mean radiance of its samples, in sample order.
__global__ __launch_bounds__(256) void k_resolve(ResolveArgs a) {
  const uint32_t pix = blockIdx.x * 256u + threadIdx.x;
  if (pix >= a.npix) return;
  float L[3] = {0.0f, 0.0f, 0.0f};
  if (a.accum && a.sample_offset)
    for (int c = 0; c < 3; ++c) L[c] = a.accum[3 * pix + c];
  for (uint32_t s = 0; s < a.spp; ++s) {
    const PathRec& pr = a.path[(size_t)pix * a.spp + s];
    for (int c = 0; c < 3; ++c) L[c] += pr.L[c];
  }
  if (a.accum)
    for (int c = 0; c < 3; ++c) a.accum[3 * pix + c] = L[c];
  // progressive accumulation: the running sum over the calls so far
  const float inv = 1.0f / (float)((a.accum ? a.sample_offset : 0u) + a.spp);
  for (int c = 0; c < 3; ++c) a.rgb[3 * pix + c] = L[c] * inv;
}

// ---------------------------------------------------------------------------
// per-round scan: bin starts, scatter cursors, work chunks
// ---------------------------------------------------------------------------
// Inclusive prefix sum over the 64 lanes of a wave on DPP: four row shifts
// build the sums inside each row of 16 lanes, then the last lane of row 0 is
// broadcast into row 1 (and of row 2 into row 3), and the last lane of row 1
// into rows 2 and 3.  Lanes whose source lies outside the row read 0.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

__device__ __forceinline__ uint32_t lane63(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, 63); }

// The scan runs as kScanTiles workgroups of 4 waves; workgroup g owns the
// cell tile [g*TS, (g+1)*TS) and wave w of it the strip of SW cells at w*SW
// (TS, SW multiples of 64).  A wave walks its strip 64 cells at a time, one
// cell per lane, so that every load and store covers consecutive words.
//  1. each wave sums its strip; the 4 sums are scanned into wave offsets and
//     the tile's sums;
//  2. the tile publishes its sums (tagged with the launch's epoch) and adds
//     up those of the tiles before it as they appear (decoupled look-back).
//     Tiles are numbered by a ticket taken at start, so a tile only waits for
//     tiles that started before it and never wait themselves: every wait
//     ends.  The last tile writes the totals and the work cursors;
//  3. each wave scans every step of 64 cells across the lanes, carrying the
//     step total, and writes the bin starts and the chunks of its cells.
// Cells are visited in increasing order, so bins and chunks are laid out in
// cell order.  A cell's count is its new records (counts) plus, when runs is
// given, the rays the previous round's chunks hand on to it; those come first
// in the bin, at offsets their chunks reserved.  Empty cells are not written:
// their cursor is never read and their counts are already zero.  T is a power
// of two.
__global__ __launch_bounds__(256) void k_scan(ScanArgs a) {
  __shared__ uint32_t s_tile, s_wr[4], s_wk[4], s_base[2];
  const uint32_t tid = threadIdx.x, lane = (uint32_t)lane_id();
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid >> 6));
  if (tid == 0) s_tile = atomicAdd(a.ticket, 1u);
  __syncthreads();
  const uint32_t ticket = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_tile);
  const uint32_t g = ticket % kScanTiles;
  const unsigned long long epoch = (unsigned long long)(ticket / kScanTiles + 1u) << 32;
  const uint32_t tm = a.T - 1u, ts = (uint32_t)__builtin_ctz(a.T);
  const uint32_t TS = ((a.C + 64u * kScanTiles - 1u) / (64u * kScanTiles)) * 64u;
  const uint32_t SW = ((TS / 64u + 3u) / 4u) * 64u;
  const uint32_t t0 = min(a.C, g * TS), t1 = min(a.C, t0 + TS);
  const uint32_t s0 = min(t1, t0 + wave * SW), s1 = min(t1, s0 + SW);
  const uint32_t nst = (s1 - s0 + 63u) >> 6;   // steps of 64 cells in this strip
  const uint32_t* counts = a.counts;
  const uint32_t* runs = a.runs;
  const size_t cs = a.cs;
  uint32_t sr = 0, sk = 0;
  for (uint32_t q = 0; q < nst; q += 8u) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t c = s0 + 64u * (q + (uint32_t)u) + lane;
      v[u] = c < s1 ? counts[(size_t)c * cs] + (runs ? runs[(size_t)c * cs] : 0u) : 0u;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sr += v[u];
      sk += (v[u] + tm) >> ts;
    }
  }
  const uint32_t wr = lane63(wave_incl_scan(sr)), wk = lane63(wave_incl_scan(sk));
  if (lane == 0) {
    s_wr[wave] = wr;
    s_wk[wave] = wk;
  }
  __syncthreads();
  if (wave == 0) {
    const uint32_t vr = lane < 4u ? s_wr[lane] : 0u, vk = lane < 4u ? s_wk[lane] : 0u;
    const uint32_t ir = wave_incl_scan(vr), ik = wave_incl_scan(vk);
    if (lane < 4u) {
      s_wr[lane] = ir - vr;
      s_wk[lane] = ik - vk;
    }
    const uint32_t tr = lane63(ir), tk = lane63(ik);
    if (lane == 0) {
      __hip_atomic_store(&a.flags[2 * g], epoch | tr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&a.flags[2 * g + 1], epoch | tk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // look back: lane j < g waits for tile j's sums
    uint32_t pr = 0, pk = 0;
    if (lane < g) {
      for (uint32_t it = 0;; ++it) {
        const unsigned long long fr =
            __hip_atomic_load(&a.flags[2 * lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long fk =
            __hip_atomic_load(&a.flags[2 * lane + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((fr & ~0xFFFFFFFFull) == epoch && (fk & ~0xFFFFFFFFull) == epoch) {
          pr = (uint32_t)fr;
          pk = (uint32_t)fk;
          break;
        }
        if (it == (1u << 22)) {   // bound on the wait (never reached)
          atomicOr(a.err, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    const uint32_t br = lane63(wave_incl_scan(pr)), bk = lane63(wave_incl_scan(pk));
    if (lane == 0) {
      s_base[0] = br;
      s_base[1] = bk;
    }
    if (g == kScanTiles - 1u) {
      const uint32_t nch = bk + tk;
      if (lane == 0) {
        *a.n_chunks = nch;
        if (a.host_ring)
          __hip_atomic_store(a.host_ring + a.ring_tag % kRoundRing,
                             ((unsigned long long)a.ring_tag << 32) | (unsigned long long)nch, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_SYSTEM);
        if (a.zero_word) *a.zero_word = 0u;
        if (a.zero_word2) *a.zero_word2 = 0u;
        if (a.total) *a.total += br + tr;
      }
      if (lane < (uint32_t)kGroups) {
        const uint32_t g0 = (uint32_t)(((uint64_t)nch * lane) / kGroups);
        a.grab[lane * kGroupStride] = g0;
        a.grab0[lane * kGroupStride] = g0;
      }
    }
  }
  __syncthreads();
  uint32_t R = s_base[0] + s_wr[wave], K = s_base[1] + s_wk[wave];
  // the bin of cell c: the runs handed on to it first (at base[c]), then the
  // new records (cursor[c] = base[c] + runs[c])
  uint32_t c = s0 + lane;
  uint32_t m1 = c < s1 ? counts[c * cs] : 0u, m2 = c + 64u < s1 ? counts[(c + 64u) * cs] : 0u;
  uint32_t h1 = c < s1 && runs ? runs[c * cs] : 0u, h2 = c + 64u < s1 && runs ? runs[(c + 64u) * cs] : 0u;
  for (uint32_t q = 0; q < nst; ++q, c += 64u) {
    const uint32_t nm = m1, nh = h1;
    m1 = m2;
    h1 = h2;
    m2 = c + 128u < s1 ? counts[(c + 128u) * cs] : 0u;
    h2 = c + 128u < s1 && runs ? runs[(c + 128u) * cs] : 0u;
    const uint32_t n = nm + nh;
    const uint32_t k = (n + tm) >> ts;
    const uint32_t ir = wave_incl_scan(n), ik = wave_incl_scan(k);
    if (n) {
      const uint32_t r = R + ir - n;
      uint32_t j = K + ik - k;
      a.cursor[c * cs] = r + nh;
      if (a.base) a.base[c] = r;
      for (uint32_t i = 0; i < n; i += a.T) a.chunks[j++] = make_uint2(c | (min(a.T, n - i) << kCellBits), r + i);
      if (a.zero_counts) {
        if (nm) a.counts[c * cs] = 0u;
        if (nh) a.runs[c * cs] = 0u;
      }
    }
    R += lane63(ir);
    K += lane63(ik);
  }
}

// ---------------------------------------------------------------------------
// Work distribution without one hot counter: the n items of a kernel are
// split into kGroups contiguous ranges, each with its own cursor on its own
// cache line; a workgroup takes `batch` consecutive items from the range of
// its group (blockIdx % kGroups, which follows the round-robin placement of
// workgroups on the XCDs) and steals from the other ranges once its own is
// used up.  Returns false when every range is exhausted.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool grab_batch(uint32_t* grab, uint32_t n, uint32_t batch, uint32_t& first,
                                           uint32_t& last) {
  const uint32_t home = blockIdx.x % (uint32_t)kGroups;
  for (uint32_t k = 0; k < (uint32_t)kGroups; ++k) {
    const uint32_t x = (home + k) % (uint32_t)kGroups;
    const uint32_t end = (uint32_t)(((uint64_t)n * (x + 1)) / kGroups);
    if (__hip_atomic_load(&grab[x * kGroupStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= end)
      continue;  // early-out; the atomic decides
    const uint32_t j = atomicAdd(&grab[x * kGroupStride], batch);
    if (j < end) {
      first = j;
      last = min(j + batch, end);
      return true;
    }
  }
  return false;
}

// thread 0 of the shading and query kernels: next chunk into s[0..3]
// (cell, start, count, valid), batch cursor in s[4], s[5]
__device__ __forceinline__ void next_item(uint32_t* grab, uint32_t n, const uint2* chunks, uint32_t* s) {
  if (s[4] >= s[5]) {
    uint32_t first, last;
    if (!grab_batch(grab, n, 2u, first, last)) {
      s[3] = 0u;
      return;
    }
    s[4] = first;
    s[5] = last;
  }
  const uint2 c = chunks[s[4]++];
  s[0] = c.x & kCellMask;
  s[1] = c.y;
  s[2] = c.x >> kCellBits;
  s[3] = 1u;
}

// ---------------------------------------------------------------------------
// counting-sort scatter of a record list by cell
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scatter(ScatterArgs a) {
  const uint32_t n = a.n_dev ? *a.n_dev : a.n;
  for (uint32_t base = blockIdx.x * 256u; base < n; base += gridDim.x * 256u) {
    const uint32_t i = base + threadIdx.x;
    RayRec r = i < n ? a.in[i] : RayRec{0, 0, kInvalidKey, 0};
    const bool valid = r.key != kInvalidKey;
    const uint32_t cell = r.key & kCellMask;
    const uint32_t pos = atomic_slot_grouped(a.cursor, a.cs, cell, valid);
    if (valid) {
      a.out[pos] = r;
      if (a.clear_in) a.in[i].key = kInvalidKey;
    }
  }
}

// Index of the pool scene that owns global cell `cell`.
__device__ __forceinline__ uint32_t scene_index(const SceneEnt* scn, uint32_t n_scenes, uint32_t cell) {
  uint32_t k = 0;
  while (k + 1u < n_scenes && cell >= scn[k].cell_end) ++k;
  return k;
}
__device__ __forceinline__ uint32_t scene_of(const PoolTabs& t, uint32_t cell) {
  return scene_index(t.scenes, t.n_scenes, cell);
}

// Neighbour of `cell` through face f = 2 * axis + (positive side); f = 6 is
// the cell itself (rays that used their step quota in this round).
__device__ __forceinline__ uint32_t neighbor_cell(const SceneGeom& sg, uint32_t cell, int face) {
  if (face == 6) return cell;
  const uint32_t N = (uint32_t)sg.N, lc = cell - sg.cell_base;
  int idx[3] = {(int)(lc % N), (int)((lc / N) % N), (int)(lc / (N * N))};
  idx[face >> 1] += (face & 1) ? 1 : -1;
  return sg.cell_base + (uint32_t)(idx[0] + (int)N * (idx[1] + (int)N * idx[2]));
}

// a value that is the same in every lane, as a scalar
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// destination of record i of a chunk's runs: the base of the run that holds
// it (o_f = offset of run f, d_f = destination of run f minus o_f), plus i
__device__ __forceinline__ uint32_t run_dest(uint32_t i, uint32_t o1, uint32_t o2, uint32_t o3, uint32_t o4,
                                             uint32_t o5, uint32_t o6, uint32_t d0, uint32_t d1, uint32_t d2,
                                             uint32_t d3, uint32_t d4, uint32_t d5, uint32_t d6) {
  uint32_t d = d0;
  d = i >= o1 ? d1 : d;
  d = i >= o2 ? d2 : d;
  d = i >= o3 ? d3 : d;
  d = i >= o4 ? d4 : d;
  d = i >= o5 ? d5 : d;
  d = i >= o6 ? d6 : d;
  return d + i;
}

// Rounds >= 1: each chunk of the previous round left its next-round rays in
// its own range of U, grouped by exit face (and a seventh group that stays
// in the cell), and reserved each run's place in its destination bin when it
// counted it; one wave moves the chunk's runs there (bin start + reserved
// offset: no atomics).  The records and the bin starts are loaded together
// and copied in one flat pass: a record's run follows from the seven run
// offsets.  The next chunk's descriptors are fetched ahead.
__global__ __launch_bounds__(256) void k_scatter_chunks(ScatterChunksArgs a) {
  const uint32_t nch = *a.n_chunks;
  const uint32_t lane = (uint32_t)lane_id();
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
  uint2 c = make_uint2(0u, 0u);
  uint4 fa = make_uint4(0u, 0u, 0u, 0u), fb = fa, oa = fa, ob = fa;
  if (wave < nch) {
    c = a.chunks[wave];
    fa = a.chunk_out[4 * wave];
    fb = a.chunk_out[4 * wave + 1];
    oa = a.chunk_out[4 * wave + 2];
    ob = a.chunk_out[4 * wave + 3];
  }
  uint4* out = reinterpret_cast<uint4*>(a.S);
  for (uint32_t j = wave; j < nch; j += nwaves) {
    // the chunk is the same in every lane
    const uint32_t cell = uniform(c.x) & kCellMask, start = uniform(c.y);
    // run sizes by exit face (x-, x+, y-, y+, z-, z+, stay) and their offsets
    const uint32_t n0 = uniform(fa.x), n1 = uniform(fa.y), n2 = uniform(fa.z), n3 = uniform(fa.w);
    const uint32_t n4 = uniform(fb.x), n5 = uniform(fb.y), n6 = uniform(fb.z);
    const uint32_t o1 = n0, o2 = o1 + n1, o3 = o2 + n2, o4 = o3 + n3, o5 = o4 + n4, o6 = o5 + n5;
    const uint32_t total = o6 + n6;
    // lane f < 7: run f's reserved offset in its destination bin
    const uint32_t roff = lane == 0u ? oa.x : lane == 1u ? oa.y : lane == 2u ? oa.z : lane == 3u ? oa.w
                        : lane == 4u ? ob.x : lane == 5u ? ob.y : lane == 6u ? ob.z : 0u;
    const uint32_t jn = j + nwaves;
    if (jn < nch) {
      c = a.chunks[jn];
      fa = a.chunk_out[4 * jn];
      fb = a.chunk_out[4 * jn + 1];
      oa = a.chunk_out[4 * jn + 2];
      ob = a.chunk_out[4 * jn + 3];
    }
    if (total == 0u) continue;
    // indexes past the chunk's records are clamped to its last one (and not
    // stored)
    const uint4* src = reinterpret_cast<const uint4*>(a.U) + start;
    const uint32_t last = total - 1u;
    uint4 v0 = src[min(lane, last)], v1 = src[min(lane + 64u, last)];
    uint4 v2 = src[min(lane + 128u, last)], v3 = src[min(lane + 192u, last)];
    // lanes 0..6: the seven runs' destinations
    const uint32_t mine = lane == 0u ? n0 : lane == 1u ? n1 : lane == 2u ? n2 : lane == 3u ? n3
                        : lane == 4u ? n4 : lane == 5u ? n5 : lane == 6u ? n6 : 0u;
    uint32_t dst = 0;
    if (mine) dst = a.base[neighbor_cell(a.tabs.scenes[scene_of(a.tabs, cell)].sg, cell, (int)lane)] + roff;
    // destination of record i: its run's base minus the run's offset, plus i
    const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)dst, 0);
    const uint32_t d1 = (uint32_t)__builtin_amdgcn_readlane((int)dst, 1) - o1;
    const uint32_t d2 = (uint32_t)__builtin_amdgcn_readlane((int)dst, 2) - o2;
    const uint32_t d3 = (uint32_t)__builtin_amdgcn_readlane((int)dst, 3) - o3;
    const uint32_t d4 = (uint32_t)__builtin_amdgcn_readlane((int)dst, 4) - o4;
    const uint32_t d5 = (uint32_t)__builtin_amdgcn_readlane((int)dst, 5) - o5;
    const uint32_t d6 = (uint32_t)__builtin_amdgcn_readlane((int)dst, 6) - o6;
    for (uint32_t b0 = 0;;) {
      const uint32_t i0 = b0 + lane, i1 = i0 + 64u, i2 = i0 + 128u, i3 = i0 + 192u;
      const uint32_t e0 = run_dest(i0, o1, o2, o3, o4, o5, o6, d0, d1, d2, d3, d4, d5, d6);
      const uint32_t e1 = run_dest(i1, o1, o2, o3, o4, o5, o6, d0, d1, d2, d3, d4, d5, d6);
      const uint32_t e2 = run_dest(i2, o1, o2, o3, o4, o5, o6, d0, d1, d2, d3, d4, d5, d6);
      const uint32_t e3 = run_dest(i3, o1, o2, o3, o4, o5, o6, d0, d1, d2, d3, d4, d5, d6);
      if (i0 < total) out[e0] = v0;
      if (i1 < total) out[e1] = v1;
      if (i2 < total) out[e2] = v2;
      if (i3 < total) out[e3] = v3;
      b0 += 256u;
      if (b0 >= total) break;
      v0 = src[min(b0 + lane, last)];
      v1 = src[min(b0 + lane + 64u, last)];
      v2 = src[min(b0 + lane + 128u, last)];
      v3 = src[min(b0 + lane + 192u, last)];
    }
  }
}

// ---------------------------------------------------------------------------
// SDF MLP of one cell on a 16-point MFMA tile, weights in registers.
// Lane (g, p) supplies encoding slots j of point p and receives hidden units
// 16b + 4g + r of point p.  Returns the SDF value d for the lane's point
// (identical in the 4 lanes of the point).
// ---------------------------------------------------------------------------
// float32: A fragments from the LDS block ([slot/4][lane][slot%4] floats)
template <int H>
__device__ __forceinline__ float march_eval_f32(const float* blk, int lane, int g,
                                                const float (&v)[kPeSlots], SoftplusK k) {
  constexpr int NB = H / 16, S1 = NB * kPeSlots, S2 = NB * (H / 4), SF = S1 + S2;
  const f32x4* fr = reinterpret_cast<const f32x4*>(blk);
  const float* vec = blk + 64 * SF;
  f32x4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = *reinterpret_cast<const f32x4*>(vec + 16 * b + 4 * g);
  {
    float w[S1];
#pragma unroll
    for (int s4 = 0; s4 < S1 / 4; ++s4) {
      const f32x4 t = fr[s4 * 64 + lane];
      w[4 * s4 + 0] = t[0]; w[4 * s4 + 1] = t[1]; w[4 * s4 + 2] = t[2]; w[4 * s4 + 3] = t[3];
    }
#pragma unroll
    for (int q = 0; q < kPeSlots; ++q)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = mfma_f32(w[b * kPeSlots + q], v[q], acc[b]);
  }
  float a1[NB][4];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) a1[b][r] = softplus_x2(acc[b][r], k);
  f32x4 acc2[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc2[b] = *reinterpret_cast<const f32x4*>(vec + H + 16 * b + 4 * g);
  {
    float w[S2];
#pragma unroll
    for (int s4 = 0; s4 < S2 / 4; ++s4) {
      const f32x4 t = fr[(S1 / 4 + s4) * 64 + lane];
      w[4 * s4 + 0] = t[0]; w[4 * s4 + 1] = t[1]; w[4 * s4 + 2] = t[2]; w[4 * s4 + 3] = t[3];
    }
#pragma unroll
    for (int q = 0; q < H / 4; ++q)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc2[b] = mfma_f32(w[b * (H / 4) + q], a1[q / 4][q % 4], acc2[b]);
  }
  float f = 0.0f;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const f32x4 w3 = *reinterpret_cast<const f32x4*>(vec + 2 * H + 16 * b + 4 * g);
#pragma unroll
    for (int r = 0; r < 4; ++r) f = fmaf(w3[r], softplus_x2(acc2[b][r], k), f);
  }
  f += __shfl_xor(f, 16);
  f += __shfl_xor(f, 32);
  return f + vec[3 * H];
}

// bfloat16: A fragments ([frag][lane] x 8 bf16) from the LDS block; every
// layer input rounded to bfloat16, float32 accumulation, bias and softplus;
// the hidden layers' pre-activations come out scaled by beta log2(e)
template <int H>
__device__ __forceinline__ float march_eval_bf16(const float* blk, int lane, int g, const float (&v)[kPeSlots],
                                                 SoftplusK k) {
  constexpr int NB = H / 16, F1 = NB * 2, F2 = F1 + NB * (H / 32), NF = F2 + H / 32;
  const uint4* fr = reinterpret_cast<const uint4*>(blk);
  const float* vec = blk + 64 * 4 * NF;
  bf16x8 e0, e1;
#pragma unroll
  for (int i = 0; i < 8; ++i) e0[i] = (__bf16)v[i];
  e1[0] = (__bf16)v[8];
  e1[1] = (__bf16)v[9];
#pragma unroll
  for (int i = 2; i < 8; ++i) e1[i] = (__bf16)0.0f;
  f32x4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = *reinterpret_cast<const f32x4*>(vec + 16 * b + 4 * g);
  {
    uint4 wf[2 * NB];   // the layer's fragments are read together, ahead of its MFMAs
#pragma unroll
    for (int i = 0; i < 2 * NB; ++i) wf[i] = fr[i * 64 + lane];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      acc[b] = mfma_bf16(__builtin_bit_cast(bf16x8, wf[2 * b]), e0, acc[b]);
      acc[b] = mfma_bf16(__builtin_bit_cast(bf16x8, wf[2 * b + 1]), e1, acc[b]);
    }
  }
  bf16x8 x[H / 32];
#pragma unroll
  for (int c = 0; c < H / 32; ++c)
#pragma unroll
    for (int i = 0; i < 8; ++i) x[c][i] = (__bf16)softplus_x2k(acc[2 * c + i / 4][i % 4]);
  f32x4 acc2[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc2[b] = *reinterpret_cast<const f32x4*>(vec + H + 16 * b + 4 * g);
#pragma unroll
  for (int c = 0; c < H / 32; ++c) {
    uint4 wf[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) wf[b] = fr[(F1 + b * (H / 32) + c) * 64 + lane];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc2[b] = mfma_bf16(__builtin_bit_cast(bf16x8, wf[b]), x[c], acc2[b]);
  }
  // SDF output row on MFMA: rows 0 (bfloat16 weights) and 1 (their
  // remainders) of the product, in lane group 0
  f32x4 y = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < H / 32; ++c) {
    bf16x8 x2;
#pragma unroll
    for (int i = 0; i < 8; ++i) x2[i] = (__bf16)softplus_x2k(acc2[2 * c + i / 4][i % 4]);
    y = mfma_bf16(__builtin_bit_cast(bf16x8, fr[(F2 + c) * 64 + lane]), x2, y);
  }
  return (y[0] + y[1]) + vec[3 * H];   // output row: hi (row 0) + lo (row 1)
}

// fp8: one tile through the two-tile evaluator (used by the point query)
template <int H>
__device__ __forceinline__ float march_eval_fp8(const float* blk, int lane, int g, const float (&v)[kPeSlots],
                                                SoftplusK k);

template <int H, int P>
__device__ __forceinline__ float march_eval(const float* blk, int lane, int g, const float (&v)[kPeSlots],
                                            SoftplusK k) {
  if constexpr (P == kPrecBf16) return march_eval_bf16<H>(blk, lane, g, v, k);
  else if constexpr (P == kPrecFp8) return march_eval_fp8<H>(blk, lane, g, v, k);
  else return march_eval_f32<H>(blk, lane, g, v, k);
}

// Two 16-point tiles at once: every weight fragment read from LDS feeds two
// MFMAs, and the two independent chains hide each other's latency.
template <int H>
__device__ __forceinline__ void march_eval2_f32(const float* blk, int lane, int g, const float (&v0)[kPeSlots],
                                                const float (&v1)[kPeSlots], SoftplusK k, float& f0, float& f1) {
  constexpr int NB = H / 16, S1 = NB * kPeSlots, S2 = NB * (H / 4), SF = S1 + S2;
  const f32x4* fr = reinterpret_cast<const f32x4*>(blk);
  const float* vec = blk + 64 * SF;
  f32x4 acc0[NB], acc1[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc1[b] = acc0[b] = *reinterpret_cast<const f32x4*>(vec + 16 * b + 4 * g);
#pragma unroll
  for (int s4 = 0; s4 < S1 / 4; ++s4) {
    const f32x4 t = fr[s4 * 64 + lane];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int sl = 4 * s4 + c, b = sl / kPeSlots, q = sl % kPeSlots;
      acc0[b] = mfma_f32(t[c], v0[q], acc0[b]);
      acc1[b] = mfma_f32(t[c], v1[q], acc1[b]);
    }
  }
  float a0[NB][4], a1[NB][4];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a0[b][r] = softplus_x2(acc0[b][r], k);
      a1[b][r] = softplus_x2(acc1[b][r], k);
    }
#pragma unroll
  for (int b = 0; b < NB; ++b) acc1[b] = acc0[b] = *reinterpret_cast<const f32x4*>(vec + H + 16 * b + 4 * g);
#pragma unroll
  for (int s4 = 0; s4 < S2 / 4; ++s4) {
    const f32x4 t = fr[(S1 / 4 + s4) * 64 + lane];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int sl = 4 * s4 + c, b = sl / (H / 4), q = sl % (H / 4);
      acc0[b] = mfma_f32(t[c], a0[q / 4][q % 4], acc0[b]);
      acc1[b] = mfma_f32(t[c], a1[q / 4][q % 4], acc1[b]);
    }
  }
  float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const f32x4 w3 = *reinterpret_cast<const f32x4*>(vec + 2 * H + 16 * b + 4 * g);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      s0 = fmaf(w3[r], softplus_x2(acc0[b][r], k), s0);
      s1 = fmaf(w3[r], softplus_x2(acc1[b][r], k), s1);
    }
  }
  s0 += __shfl_xor(s0, 16);
  s1 += __shfl_xor(s1, 16);
  s0 += __shfl_xor(s0, 32);
  s1 += __shfl_xor(s1, 32);
  f0 = s0 + vec[3 * H];
  f1 = s1 + vec[3 * H];
}

template <int H>
__device__ __forceinline__ void march_eval2_bf16(const float* blk, int lane, int g, const float (&v0)[kPeSlots],
                                                 const float (&v1)[kPeSlots], SoftplusK k, float& f0, float& f1) {
  constexpr int NB = H / 16, F1 = NB * 2, F2 = F1 + NB * (H / 32), NF = F2 + H / 32;
  const uint4* fr = reinterpret_cast<const uint4*>(blk);
  const float* vec = blk + 64 * 4 * NF;
  bf16x8 e0[2], e1[2];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    e0[0][i] = (__bf16)v0[i];
    e1[0][i] = (__bf16)v1[i];
  }
  e0[1][0] = (__bf16)v0[8];
  e0[1][1] = (__bf16)v0[9];
  e1[1][0] = (__bf16)v1[8];
  e1[1][1] = (__bf16)v1[9];
#pragma unroll
  for (int i = 2; i < 8; ++i) e0[1][i] = e1[1][i] = (__bf16)0.0f;
  f32x4 acc0[NB], acc1[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc1[b] = acc0[b] = *reinterpret_cast<const f32x4*>(vec + 16 * b + 4 * g);
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const bf16x8 w = __builtin_bit_cast(bf16x8, fr[(2 * b + c) * 64 + lane]);
      acc0[b] = mfma_bf16(w, e0[c], acc0[b]);
      acc1[b] = mfma_bf16(w, e1[c], acc1[b]);
    }
  bf16x8 x0[H / 32], x1[H / 32];
#pragma unroll
  for (int c = 0; c < H / 32; ++c)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      x0[c][i] = (__bf16)softplus_x2k(acc0[2 * c + i / 4][i % 4]);
      x1[c][i] = (__bf16)softplus_x2k(acc1[2 * c + i / 4][i % 4]);
    }
#pragma unroll
  for (int b = 0; b < NB; ++b) acc1[b] = acc0[b] = *reinterpret_cast<const f32x4*>(vec + H + 16 * b + 4 * g);
#pragma unroll
  for (int c = 0; c < H / 32; ++c)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const bf16x8 w = __builtin_bit_cast(bf16x8, fr[(F1 + b * (H / 32) + c) * 64 + lane]);
      acc0[b] = mfma_bf16(w, x0[c], acc0[b]);
      acc1[b] = mfma_bf16(w, x1[c], acc1[b]);
    }
  f32x4 y0 = f32x4{0.0f, 0.0f, 0.0f, 0.0f}, y1 = y0;
#pragma unroll
  for (int c = 0; c < H / 32; ++c) {
    bf16x8 z0, z1;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      z0[i] = (__bf16)softplus_x2k(acc0[2 * c + i / 4][i % 4]);
      z1[i] = (__bf16)softplus_x2k(acc1[2 * c + i / 4][i % 4]);
    }
    const bf16x8 w = __builtin_bit_cast(bf16x8, fr[(F2 + c) * 64 + lane]);
    y0 = mfma_bf16(w, z0, y0);
    y1 = mfma_bf16(w, z1, y1);
  }
  f0 = (y0[0] + y0[1]) + vec[3 * H];   // output row: hi (row 0) + lo (row 1)
  f1 = (y1[0] + y1[1]) + vec[3 * H];
}

// fp8 e4m3: A fragments ([frag][lane] x 8 bytes); layer inputs quantised
// with power-of-two scales (encoding: 1; a1: vec[3H+3] applied to 2k a1),
// the products accumulated in float32, then u = acc * scale + bias (for
// layer 1 both stored times k = beta log2(e), as the bfloat16 block's);
// softplus in float32; the SDF output row on bfloat16 MFMA.
template <int H>
__device__ __forceinline__ void march_eval2_fp8(const float* blk, int lane, int g, const float (&v0)[kPeSlots],
                                                const float (&v1)[kPeSlots], SoftplusK k, float& f0, float& f1) {
  constexpr int NB = H / 16, F1 = NB * 2, NF = F1 + NB * (H / 32);
  const uint2* fr = reinterpret_cast<const uint2*>(blk);
  const uint4* f3 = reinterpret_cast<const uint4*>(blk + 2 * 64 * NF);
  const float* vec = blk + 2 * 64 * NF + 4 * 64 * (H / 32);
  const float s1 = vec[3 * H + 1], s2 = vec[3 * H + 2], ia = vec[3 * H + 3];
  const long e0[2] = {fp8x8(v0[0], v0[1], v0[2], v0[3], v0[4], v0[5], v0[6], v0[7]),
                      fp8x8(v0[8], v0[9], 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f)};
  const long e1[2] = {fp8x8(v1[0], v1[1], v1[2], v1[3], v1[4], v1[5], v1[6], v1[7]),
                      fp8x8(v1[8], v1[9], 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f)};
  f32x4 acc0[NB], acc1[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc1[b] = acc0[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const long w = __builtin_bit_cast(long, fr[(2 * b + c) * 64 + lane]);
      acc0[b] = mfma_fp8(w, e0[c], acc0[b]);
      acc1[b] = mfma_fp8(w, e1[c], acc1[b]);
    }
  long x0[H / 32], x1[H / 32];
#pragma unroll
  for (int c = 0; c < H / 32; ++c) {
    float q0[8], q1[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int b = 2 * c + i / 4, r = i % 4;
      const float bias = vec[16 * b + 4 * g + r];
      q0[i] = fminf(softplus_x2k(fmaf(acc0[b][r], s1, bias)) * ia, kE4m3MaxF);
      q1[i] = fminf(softplus_x2k(fmaf(acc1[b][r], s1, bias)) * ia, kE4m3MaxF);
    }
    x0[c] = fp8x8(q0[0], q0[1], q0[2], q0[3], q0[4], q0[5], q0[6], q0[7]);
    x1[c] = fp8x8(q1[0], q1[1], q1[2], q1[3], q1[4], q1[5], q1[6], q1[7]);
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) acc1[b] = acc0[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < H / 32; ++c)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const long w = __builtin_bit_cast(long, fr[(F1 + b * (H / 32) + c) * 64 + lane]);
      acc0[b] = mfma_fp8(w, x0[c], acc0[b]);
      acc1[b] = mfma_fp8(w, x1[c], acc1[b]);
    }
  f32x4 y0 = f32x4{0.0f, 0.0f, 0.0f, 0.0f}, y1 = y0;
#pragma unroll
  for (int c = 0; c < H / 32; ++c) {
    bf16x8 z0, z1;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int b = 2 * c + i / 4, r = i % 4;
      const float bias = vec[H + 16 * b + 4 * g + r];
      z0[i] = (__bf16)softplus_x2(fmaf(acc0[b][r], s2, bias), k);
      z1[i] = (__bf16)softplus_x2(fmaf(acc1[b][r], s2, bias), k);
    }
    const bf16x8 w = __builtin_bit_cast(bf16x8, f3[c * 64 + lane]);
    y0 = mfma_bf16(w, z0, y0);
    y1 = mfma_bf16(w, z1, y1);
  }
  f0 = (y0[0] + y0[1]) + vec[3 * H];   // output row: hi (row 0) + lo (row 1)
  f1 = (y1[0] + y1[1]) + vec[3 * H];
}

template <int H>
__device__ __forceinline__ float march_eval_fp8(const float* blk, int lane, int g, const float (&v)[kPeSlots],
                                                SoftplusK k) {
  constexpr int NB = H / 16, F1 = NB * 2, NF = F1 + NB * (H / 32);
  const uint2* fr = reinterpret_cast<const uint2*>(blk);
  const uint4* f3 = reinterpret_cast<const uint4*>(blk + 2 * 64 * NF);
  const float* vec = blk + 2 * 64 * NF + 4 * 64 * (H / 32);
  const float s1 = vec[3 * H + 1], s2 = vec[3 * H + 2], ia = vec[3 * H + 3];
  const long e[2] = {fp8x8(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]),
                     fp8x8(v[8], v[9], 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f)};
  f32x4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  {
    uint2 wf[2 * NB];   // the layer's fragments are read together, ahead of its MFMAs
#pragma unroll
    for (int i = 0; i < 2 * NB; ++i) wf[i] = fr[i * 64 + lane];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[b] = mfma_fp8(__builtin_bit_cast(long, wf[2 * b + c]), e[c], acc[b]);
  }
  long x[H / 32];
#pragma unroll
  for (int c = 0; c < H / 32; ++c) {
    float q[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int b = 2 * c + i / 4, r = i % 4;
      q[i] = fminf(softplus_x2k(fmaf(acc[b][r], s1, vec[16 * b + 4 * g + r])) * ia, kE4m3MaxF);
    }
    x[c] = fp8x8(q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7]);
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < H / 32; ++c) {
    uint2 wf[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) wf[b] = fr[(F1 + b * (H / 32) + c) * 64 + lane];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = mfma_fp8(__builtin_bit_cast(long, wf[b]), x[c], acc[b]);
  }
  f32x4 y = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < H / 32; ++c) {
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int b = 2 * c + i / 4, r = i % 4;
      z[i] = (__bf16)softplus_x2(fmaf(acc[b][r], s2, vec[H + 16 * b + 4 * g + r]), k);
    }
    y = mfma_bf16(__builtin_bit_cast(bf16x8, f3[c * 64 + lane]), z, y);
  }
  return (y[0] + y[1]) + vec[3 * H];   // output row: hi (row 0) + lo (row 1)
}

template <int H, int P>
__device__ __forceinline__ void march_eval2(const float* blk, int lane, int g, const float (&v0)[kPeSlots],
                                            const float (&v1)[kPeSlots], SoftplusK k, float& f0, float& f1) {
  if constexpr (P == kPrecBf16) march_eval2_bf16<H>(blk, lane, g, v0, v1, k, f0, f1);
  else if constexpr (P == kPrecFp8) march_eval2_fp8<H>(blk, lane, g, v0, v1, k, f0, f1);
  else march_eval2_f32<H>(blk, lane, g, v0, v1, k, f0, f1);
}

// Copies one packed per-cell block (words % 4 == 0, 16-byte aligned at both
// ends) into LDS with direct global-to-LDS loads: 16 bytes per lane, so one
// wave instruction fills 1 KB, and all of a thread's loads are in flight at
// once without passing through registers.  stage_wait() must precede the
// barrier after which the block is read.
__device__ __forceinline__ void stage_block(float* lds, const float* src, uint32_t words) {
  const uint32_t n4 = words / 4u, lane = threadIdx.x & 63u;
  const uint32_t nw = blockDim.x >> 6;
  for (uint32_t c = threadIdx.x >> 6; c * 64u < n4; c += nw) {
    const uint32_t i = c * 64u + lane;
    if (i < n4)
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)(src + 4u * i),
          (__attribute__((address_space(3))) void*)(lds + 256u * c), 16, 0, 0);
  }
}

// the wave's direct-to-LDS loads have landed: vmcnt(0) (expcnt and lgkmcnt
// left at their maxima), as a builtin so that the compiler's own wait
// tracking knows every vector memory operation before it is complete
__device__ __forceinline__ void stage_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Workgroup barrier for data in LDS only: waits for this wave's own LDS
// operations, not for vector memory, so direct global-to-LDS loads (weight
// staging for the next work item) stay in flight across it.  A
// __syncthreads() here would wait for them (its release fence covers every
// LDS write, the pending direct loads included).  The signal fences keep the
// compiler from moving memory operations across the barrier.  Only for
// exchanges through LDS whose writers are ordinary LDS stores.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt and expcnt left at their maxima
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

struct CellBox {
  int ix, iy, iz;
  float c[3];
  float cs[3];   // -(c / h): local coordinate x_l = fma(x, 1/h, cs)
};

__device__ __forceinline__ CellBox cell_box(const SceneGeom& sg, uint32_t lc) {
  CellBox b;
  const uint32_t N = (uint32_t)sg.N;
  b.ix = (int)(lc % N);
  b.iy = (int)((lc / N) % N);
  b.iz = (int)(lc / (N * N));
  b.c[0] = sg.bmin[0] + ((float)b.ix + 0.5f) * sg.side[0];
  b.c[1] = sg.bmin[1] + ((float)b.iy + 0.5f) * sg.side[1];
  b.c[2] = sg.bmin[2] + ((float)b.iz + 0.5f) * sg.side[2];
  // c / h = bmin / h + 2 i + 1: exact integers for the [-1,1]^3 box
  b.cs[0] = -fmaf(sg.bmin[0], sg.inv_half[0], (float)(2 * b.ix + 1));
  b.cs[1] = -fmaf(sg.bmin[1], sg.inv_half[1], (float)(2 * b.iy + 1));
  b.cs[2] = -fmaf(sg.bmin[2], sg.inv_half[2], (float)(2 * b.iz + 1));
  return b;
}

// Nearest exit plane of cell (ix,iy,iz) along the ray; *axis gets its axis
// (ties to the lowest axis).  RCP: the distance to each plane is taken
// through the hardware reciprocal of the direction (within 2 ulp of the
// quotient) instead of a correctly rounded division; the low-precision
// marches use it, as the exit only bounds their steps and the next cell
// starts from the same value.
template <bool RCP = false>
__device__ __forceinline__ float cell_exit(const SceneGeom& sg, const CellBox& cb, const float o[3],
                                           const float d[3], int* axis) {
  const int idx[3] = {cb.ix, cb.iy, cb.iz};
  float best = INFINITY;
  int ba = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (d[k] != 0.0f) {
      float plane = sg.bmin[k] + (float)(idx[k] + (d[k] > 0.0f ? 1 : 0)) * sg.side[k];
      float tk = RCP ? (plane - o[k]) * __builtin_amdgcn_rcpf(d[k]) : (plane - o[k]) / d[k];
      if (tk < best) {
        best = tk;
        ba = k;
      }
    }
  }
  *axis = ba;
  return best;
}

// in-cell status of a staged ray
// (kOutJump: an unclamped step left the cell; the ray goes on in the cell
// that contains its new point)
enum : uint32_t { kStay = 0, kOutHit = 1, kOutNext = 2, kOutExit = 3, kOutBudget = 4, kOutJump = 5 };
// the staged ray word: steps (bits 0-9), exit axis (10-11), status (12-14),
// the slot's step budget (16-25) and unclamped-step flag (26)
constexpr uint32_t kStUnclamped = 1u << 26;

// ---------------------------------------------------------------------------
// the march: one workgroup (4 waves) per chunk of <= kChunk rays of one cell
// ---------------------------------------------------------------------------
struct Job {
  uint32_t cell, start, count, id, scene;
  bool valid;
};

// (plain LDS reads: the workgroup barrier before every call orders them)
// (the fields are uniform: taken into scalar registers, so that the work
// derived from them stays on the scalar unit)
__device__ __forceinline__ Job read_job(const uint32_t* s) {
  auto u = [](uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); };
  return Job{u(s[0]), u(s[1]), u(s[2]), u(s[3]), u(s[5]), u(s[4]) != 0u};
}

// Thread 0's source of march work items.  Items are taken one at a time from
// the workgroup's home range, and the atomic for the following item is issued
// when one is taken, so its round trip overlaps the item in progress (the
// workgroup holds at most two items; increments past the end of the range
// are harmless).  Once the home range is used up the other ranges are visited
// synchronously.
// The cursor is advanced with an atomic increment (bound 2^32 - 1, so it
// never wraps), which the compiler leaves alone, so the result is waited for
// only where it is used.
__device__ __forceinline__ uint32_t cursor_take(uint32_t* c) {
  return __builtin_amdgcn_atomic_inc32(c, 0xFFFFFFFFu, __ATOMIC_RELAXED, "agent");
}

struct Grabber {
  uint32_t n;        // work items in this launch
  uint32_t end;      // end of the home range
  uint32_t pend;     // result of the atomic issued ahead on the home range
  uint32_t* cursor;  // the home range's cursor
};

__device__ __forceinline__ Grabber grab_init(uint32_t* grab, uint32_t n) {
  const uint32_t home = blockIdx.x % (uint32_t)kGroups;
  Grabber G;
  G.n = n;
  G.end = (uint32_t)(((uint64_t)n * (home + 1)) / kGroups);
  G.cursor = grab + home * kGroupStride;
  G.pend = cursor_take(G.cursor);
  return G;
}

__device__ __forceinline__ bool grab_next(uint32_t* grab, Grabber& G, uint32_t& j) {
  // taken into a scalar first, so the new atomic can reuse the register
  j = (uint32_t)__builtin_amdgcn_readfirstlane((int)G.pend);
  G.pend = cursor_take(G.cursor);
  if (j < G.end) return true;
  uint32_t last;
  return grab_batch(grab, G.n, 1u, j, last);
}

// work item j (its descriptor c) into s[0..5] (cell, start, count, id,
// valid, scene)
__device__ __forceinline__ void put_job(const SceneEnt* scn, uint32_t n_scenes, uint32_t* s, uint2 c, uint32_t j) {
  s[0] = c.x & kCellMask;
  s[1] = c.y;
  s[2] = c.x >> kCellBits;
  s[3] = j;
  s[5] = scene_index(scn, n_scenes, s[0]);
  s[4] = 1u;
}

// Both MLP widths in one kernel when HM = 0 (pools mixing scenes of H = 32
// and H = 64); the branch is uniform over the workgroup.
template <int HM, int P>
__device__ __forceinline__ void march_eval2_h(int H, const float* blk, int lane, int g,
                                              const float (&v0)[kPeSlots], const float (&v1)[kPeSlots],
                                              SoftplusK k, float& f0, float& f1) {
  if constexpr (HM != 0) {
    march_eval2<HM, P>(blk, lane, g, v0, v1, k, f0, f1);
  } else {
    if (H == 64) march_eval2<64, P>(blk, lane, g, v0, v1, k, f0, f1);
    else march_eval2<32, P>(blk, lane, g, v0, v1, k, f0, f1);
  }
}

template <int HM, int P>
__device__ __forceinline__ float march_eval_h(int H, const float* blk, int lane, int g, const float (&v)[kPeSlots],
                                              SoftplusK k) {
  if constexpr (HM != 0) return march_eval<HM, P>(blk, lane, g, v, k);
  else return H == 64 ? march_eval<64, P>(blk, lane, g, v, k) : march_eval<32, P>(blk, lane, g, v, k);
}

// s_st word of a staged ray: steps | exit axis << 10 | status << 12 | step budget << 16
// PAIR: each wave evaluates two 16-ray tiles per step (shared weight reads,
// two independent chains); otherwise one tile with more waves per SIMD (WPE).
// UNC: a variant for requests with unclamped steps (the default kernel has
// no code for them)
template <int HM, int P, bool PAIR, int WPE, bool UNC>
__global__ __launch_bounds__(256, WPE) void k_march(MarchArgs a) {
  extern __shared__ __align__(16) float s_dyn[];
  float* s_t = s_dyn;
  float* s_te = s_t + kChunk;
  float* s_o = s_te + kChunk;        // [3][kChunk]
  float* s_d = s_o + 3 * kChunk;     // [3][kChunk]
  float* s_tf = s_d + 3 * kChunk;
  float* s_ce = s_tf + kChunk;
  float* s_eps = s_ce + kChunk;
  uint32_t* s_rid = reinterpret_cast<uint32_t*>(s_eps + kChunk);
  uint32_t* s_pix = s_rid + kChunk;
  uint32_t* s_st = s_pix + kChunk;
  uint16_t* s_act = reinterpret_cast<uint16_t*>(s_st + kChunk);  // [2][kChunk]
  float* s_w = reinterpret_cast<float*>(s_act + 2 * kChunk);      // weight block (16-byte aligned)
  __shared__ uint32_t s_job[6], s_jn[6];   // current / next work item: cell, start, count, id, valid, scene
  // per pass p: survivors counted in s_nact[(p + 1) % 3] (three slots, so
  // that thread 0 can clear the next pass's one during a pass: a slot's last
  // reader is always behind an earlier barrier)
  __shared__ uint32_t s_nact[3];
  // The output phase runs while the next item's weight block is being
  // staged by direct global-to-LDS loads, and the compiler makes every LDS
  // atomic wait for those loads to land (it cannot tell the block from the
  // counters).  So the phase counts with wave ballots and plain LDS stores
  // instead: per wave, the rays of each class (exit faces 0-5, staying 6,
  // jumping 7, hits 8), and per wave and request slot the misses.
  constexpr int kCls = 9;
  __shared__ uint32_t s_wcnt[4][kCls];
  __shared__ uint32_t s_foff[7], s_jbase;
  __shared__ uint32_t s_wmiss[4][kMaxSlots];   // misses per wave and request slot
  __shared__ unsigned long long s_wtot[4][2];  // evaluations and tiles per wave
  // the pool's scene table and each request slot's eps and step budget,
  // copied once: every work item reads them
  __shared__ SceneEnt s_scn[kMaxScenes];
  __shared__ float s_qeps[kMaxSlots];
  __shared__ uint32_t s_qmst[kMaxSlots];
  // a round without work items (the last rounds a frame enqueues ahead of
  // knowing that it is done) returns before staging anything
  if (*a.n_chunks == 0u) return;
  const int tid = threadIdx.x, lane = lane_id(), g = lane >> 4, p = lane & 15, wave = tid >> 6;
  const PeLane pl = make_pe_lane(g);
  unsigned long long wv_evals = 0, wv_tiles = 0, wg_chunks = 0;  // lane 0's / thread 0's tallies
  uint32_t loaded = 0xFFFFFFFFu;
  // this chunk's ray record and static data, loaded ahead during the
  // previous chunk when possible
  RayRec pf_rec = {0, 0, 0, 0};
  RayStatic pf_st = {0, 0, 0, 0, 0, 0, 1, 0};
  bool pf_rec_ok = false, pf_st_ok = false;
  if (tid < kMaxSlots) {
    for (int w = 0; w < 4; ++w) s_wmiss[w][tid] = 0u;
    s_qeps[tid] = a.tabs.reqs[tid].eps;
    s_qmst[tid] = a.tabs.reqs[tid].max_steps | (a.tabs.reqs[tid].unclamped ? (kStUnclamped >> 16) : 0u);
  }
  {
    static_assert(sizeof(SceneEnt) % 4 == 0, "scene entries are copied as words");
    const uint32_t words = a.tabs.n_scenes * (uint32_t)(sizeof(SceneEnt) / 4);
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.tabs.scenes);
    uint32_t* dst = reinterpret_cast<uint32_t*>(s_scn);
    for (uint32_t i = (uint32_t)tid; i < words; i += 256u) dst[i] = src[i];
  }
  __syncthreads();
  Grabber G{0u, 0u, 0u, nullptr};   // thread 0's
  // threads 1..7: the last work item's run reservation, stored one item later
  constexpr uint32_t kNoJob = 0xFFFFFFFFu;
  uint32_t pend_job = kNoJob, pend_off = 0u;
  // thread 0: a work item's counters start at zero
  auto clear_item = [&]() {
    s_nact[1] = 0u;
    s_jn[4] = 0u;
  };
  if (tid == 0) {
    G = grab_init(a.grab, *a.n_chunks);
    uint32_t j;
    if (grab_next(a.grab, G, j)) put_job(s_scn, a.tabs.n_scenes, s_job, a.chunks[j], j);
    else s_job[4] = 0u;
    clear_item();
  }
  __syncthreads();
  for (;;) {
    const Job jb = read_job(s_job);
    if (!jb.valid) break;
    const uint32_t cell = jb.cell, start = jb.start, count = jb.count, job = jb.id;
    // thread 0 takes the next work item's index now and starts loading its
    // descriptor; both round trips overlap the staging below
    uint2 cn = make_uint2(0u, 0u);
    uint32_t jn = 0;
    bool jn_ok = false;
    if (tid == 0) {
      jn_ok = grab_next(a.grab, G, jn);
      if (jn_ok) cn = a.chunks[jn];
    }
    const SceneEnt* se = s_scn + __builtin_amdgcn_readfirstlane(jb.scene);
    const SceneGeom sg = se->sg;
    const SoftplusK spk = se->spk;
    const int H = HM ? HM : sg.H;
    const int N = sg.N;
    const uint32_t lc = cell - sg.cell_base;
    const CellBox cb = cell_box(sg, lc);
    if (cell != loaded) {
      stage_block(s_w, se->march + (size_t)lc * se->march_words, se->march_words);
      loaded = cell;
    }
    if ((uint32_t)tid < count) {
      const RayRec r = pf_rec_ok ? pf_rec : a.S[start + tid];
      const RayStatic st = pf_st_ok ? pf_st : a.rs[r.rid];
      const uint32_t qs = st.pix >> kPixBits;
      const float o[3] = {st.ox, st.oy, st.oz}, d[3] = {st.dx, st.dy, st.dz};
      int eax;
      const float ce = cell_exit<P != kPrecF32>(sg, cb, o, d, &eax);
      s_t[tid] = r.t;
      s_te[tid] = r.t_entry;
      for (int k = 0; k < 3; ++k) {
        s_o[k * kChunk + tid] = o[k];
        s_d[k * kChunk + tid] = d[k];
      }
      s_tf[tid] = st.t_far;
      s_ce[tid] = ce;
      s_eps[tid] = s_qeps[qs];
      s_rid[tid] = r.rid;
      s_pix[tid] = st.pix;
      s_st[tid] = (r.key >> kCellBits) | ((uint32_t)eax << 10) | (s_qmst[qs] << 16);
      s_act[tid] = (uint16_t)tid;
    }
    pf_rec_ok = pf_st_ok = false;
    stage_wait();
    if (tid >= 1 && tid <= 7 && pend_job != kNoJob) {
      reinterpret_cast<uint32_t*>(a.chunk_out)[16u * pend_job + 8u + (uint32_t)tid - 1u] = pend_off;
      pend_job = kNoJob;
    }
    // the next work item's descriptor is in (the staging wait covered it)
    if (tid == 0 && jn_ok) put_job(s_scn, a.tabs.n_scenes, s_jn, cn, jn);
    __syncthreads();
    // start loading the next work item's rays (their static data one pass
    // later, once the record is in)
    {
      const Job nx = read_job(s_jn);
      if (nx.valid && (uint32_t)tid < nx.count) {
        pf_rec = a.S[nx.start + tid];
        pf_rec_ok = true;
      }
    }

    // passes over the rays still inside the cell; after max_passes the rest
    // go on in the next round (same cell), so a few slow rays near the
    // surface do not hold the workgroup
    uint32_t nact = count, wave_evals = 0, wave_tiles = 0;
    int cur = 0;
    for (int pass = 0; nact && pass < a.max_passes; ++pass) {
      const uint32_t ntiles = (nact + 15u) >> 4;
      const uint16_t* act_in = s_act + cur * kChunk;
      uint16_t* act_out = s_act + (cur ^ 1) * kChunk;
      const int i1 = (pass + 1) % 3, i2 = (pass + 2) % 3;
      if (tid == 0) s_nact[i2] = 0u;   // the next pass's counter (last used two passes ago)
      // tiles dealt round-robin to the workgroup's waves: every tile costs
      // one evaluation, so a fixed deal balances as well as a shared counter
      // would, without its two LDS round trips per tile
      constexpr uint32_t kTileStep = (PAIR ? 2u : 1u) * (256u / 64u);
      for (uint32_t tile = (PAIR ? 2u : 1u) * (uint32_t)wave; tile < ntiles; tile += kTileStep) {
        uint32_t ri[2];
        bool valid[2];
        float t[2], o[2][3], d[2][3], v[2][kPeSlots];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const uint32_t idx = (PAIR || u == 0) ? (tile + (uint32_t)u) * 16u + (uint32_t)p : 0xFFFFFFFFu;
          valid[u] = idx < nact;
          ri[u] = valid[u] ? act_in[idx] : 0u;
          t[u] = s_t[ri[u]];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            o[u][k] = s_o[k * kChunk + ri[u]];
            d[u][k] = s_d[k * kChunk + ri[u]];
          }
          float xl[3];
#pragma unroll
          for (int k = 0; k < 3; ++k)
            xl[k] = valid[u] ? fmaf(fmaf(t[u], d[u][k], o[u][k]), sg.inv_half[k], cb.cs[k]) : 0.0f;
          pe_values<P != kPrecF32>(pl, xl[0], xl[1], xl[2], v[u]);
        }
        float f[2];
        if constexpr (PAIR) {
          march_eval2_h<HM, P>(H, s_w, lane, g, v[0], v[1], spk, f[0], f[1]);
        } else {
          f[0] = march_eval_h<HM, P>(H, s_w, lane, g, v[0], spk);
          f[1] = 0.0f;
        }
        ++wave_tiles;
        bool stay[2] = {false, false};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          wave_evals += (uint32_t)__popcll(__ballot(valid[u]) & 0xFFFFull);
          if (valid[u] && g == 0) {
            const uint32_t r_ = ri[u];
            const uint32_t stw = s_st[r_];
            const uint32_t steps = (stw & 1023u) + 1u, eax = (stw >> 10) & 3u;
            uint32_t status = kStay;
            float tt = t[u];
            if (f[u] < s_eps[r_]) {
              status = kOutHit;
            } else {
              const float te = fmaxf(tt, s_ce[r_]);
              if (tt + f[u] < te) {
                // an in-cell step can pass t_far only when the interval ends
                // inside the box (a world ray cut short by a primitive)
                tt = tt + f[u];
                if (tt > s_tf[r_]) status = kOutExit;
              } else if (UNC && (stw & kStUnclamped)) {
                // Hart's full step: the ray goes on in the cell of its new point
                tt = tt + f[u];
                status = tt > s_tf[r_] ? kOutExit : kOutJump;
              } else {
                tt = te;
                const int sgn = d[u][eax] > 0.0f ? 1 : -1;
                const int ni = (eax == 0 ? cb.ix : (eax == 1 ? cb.iy : cb.iz)) + sgn;
                status = (ni < 0 || ni >= N || tt > s_tf[r_]) ? kOutExit : kOutNext;
              }
              // (the unclamped flag above the budget is set only for the
              // UNC kernel's requests)
              if ((status == kStay || status == kOutNext || (UNC && status == kOutJump)) &&
                  steps >= (UNC ? ((stw >> 16) & 1023u) : (stw >> 16)))
                status = kOutBudget;
            }
            s_t[r_] = tt;
            s_st[r_] = steps | (eax << 10) | (status << 12) | (stw & 0xFFFF0000u);
            stay[u] = status == kStay;
          }
        }
        const uint64_t sm0 = __ballot(stay[0]), sm1 = __ballot(stay[1]);
        if (sm0 | sm1) {
          const uint32_t n0 = (uint32_t)__popcll(sm0);
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(&s_nact[i1], n0 + (uint32_t)__popcll(sm1));
          base = __builtin_amdgcn_readfirstlane(base);   // every lane is active here
          if (stay[0]) act_out[base + lane_rank(sm0)] = (uint16_t)ri[0];
          if (stay[1]) act_out[base + n0 + lane_rank(sm1)] = (uint16_t)ri[1];
        }
      }
      __syncthreads();
      nact = s_nact[i1];
      // the next work item's ray records (loaded before pass 0) are in: its
      // static ray data follows
      if (pass == 0 && pf_rec_ok) {
        // the record's ray id is taken here, not before the passes: the
        // compiler would otherwise form the address ahead of the loop and
        // wait there for the record to arrive
        uint32_t rid = pf_rec.rid;
        asm volatile("" : "+v"(rid));
        pf_st = a.rs[rid];
        pf_st_ok = true;
      }
      cur ^= 1;
    }
    // the weights are not read again for this work item: the next one's
    // block starts loading now, behind the output phase (the staging wait
    // of the next item covers it); so does the next item's static ray data
    // when this item ended after one pass
    if (pf_rec_ok && !pf_st_ok) {
      pf_st = a.rs[pf_rec.rid];
      pf_st_ok = true;
    }
    {
      const Job nx = read_job(s_jn);
      if (nx.valid && nx.cell != loaded) {
        const SceneEnt* sn = s_scn + __builtin_amdgcn_readfirstlane(nx.scene);
        stage_block(s_w, sn->march + (size_t)(nx.cell - sn->sg.cell_base) * sn->march_words, sn->march_words);
        loaded = nx.cell;
      }
    }
    wv_evals += wave_evals;
    wv_tiles += wave_tiles;

    // results: misses written out, hits appended to the hit list, rays for
    // the next round into this chunk's range of U, grouped by exit face
    // (face 6: still in this cell after max_passes)
    uint32_t status = kOutHit, steps = 0, face = 0, slot = 0, dest = 0, cls = kCls;
    bool miss = false;
    float t = 0.0f, t_entry = 0.0f;
    if ((uint32_t)tid < count) {
      const uint32_t stw = s_st[tid];
      status = (stw >> 12) & 7u;
      steps = stw & 1023u;
      t = s_t[tid];
      t_entry = s_te[tid];
      if (UNC && status == kOutJump) {
        // the cell containing the new point (cell map of Sec. 3.1, clamped)
        int idx[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const float x = fmaf(t, s_d[k * kChunk + tid], s_o[k * kChunk + tid]);
          idx[k] = min(max((int)floorf((x - sg.bmin[k]) * sg.inv_side[k]), 0), N - 1);
        }
        dest = sg.cell_base + (uint32_t)(idx[0] + N * (idx[1] + N * idx[2]));
        t_entry = t;
        cls = 7u;
      } else if (status == kOutNext || status == kStay) {
        const uint32_t eax = (stw >> 10) & 3u;
        face = status == kStay ? 6u : 2u * eax + (s_d[eax * kChunk + tid] > 0.0f ? 1u : 0u);
        if (status == kOutNext) t_entry = t;
        cls = face;
      } else if (status == kOutHit) {
        a.hits[s_rid[tid]] = RayRec{t, t_entry, cell | (steps << kCellBits), s_rid[tid]};
        cls = 8u;
      } else {
        const uint32_t px = s_pix[tid];
        slot = px >> kPixBits;
        miss = true;
        const ReqEnt q = a.tabs.reqs[slot];   // copied before the first store
        const int32_t mst = status == kOutExit ? kExitMiss : kBudgetMiss;
        if (q.world && status == kOutExit) {
          // a world ray that reached the end of its interval goes on past
          // this instance's box
          const uint32_t rid = s_rid[tid];
          const float ol[3] = {s_o[tid], s_o[kChunk + tid], s_o[2 * kChunk + tid]};
          const float d[3] = {s_d[tid], s_d[kChunk + tid], s_d[2 * kChunk + tid]};
          float tn, tf;
          (void)slab(sg, ol, d, &tn, &tf);
          const WState w = a.ws[rid];
          WorldRec wr;
          for (int c = 0; c < 3; ++c) {
            wr.o[c] = w.o[c];
            wr.d[c] = d[c];
          }
          wr.tpm = w.tpm;
          wr.tim = se->ws * tf;
          wr.rid = rid;
          wr.pad[0] = wr.pad[1] = wr.pad[2] = 0u;
          a.wlist[atomicAdd(a.n_w, 1u)] = wr;   // world renders only
          miss = false;
        } else if (q.pt) {
          // the path escapes: radiance += throughput x environment
          const uint32_t rid = s_rid[tid];
          PathRec& pr = a.tabs.path[rid];
          const float d[3] = {s_d[tid], s_d[kChunk + tid], s_d[2 * kChunk + tid]};
          float e[3];
          env_lookup(q.env, q.env_w, q.env_h, d, e);
          for (int c = 0; c < 3; ++c) pr.L[c] += pr.T[c] * e[c];
          if (pr.bounce == 0 && rid % q.spp == 0)
            write_miss(q.out, px & kPixMask, (int)steps, t, t_entry, (int32_t)cell, mst, false);
          if (q.out.seg) {
            auto& sr = *gmem(q.out.seg + (size_t)rid * (q.bounces + 1u) + pr.bounce);
            sr.t_march = t;
            sr.t_entry = t_entry;
            sr.cell = (int32_t)cell;
            sr.status = mst;
            sr.steps = steps;
          }
        } else {
          write_miss(q.out, px & kPixMask, (int)steps, t, t_entry, (int32_t)cell, mst);
        }
      }
    }
    // this wave's count of each class and each lane's rank in its class
    // (hits need no rank, and only the unclamped kernel has jumped rays)
    uint32_t rank = 0;
#pragma unroll
    for (uint32_t c = 0; c < (uint32_t)kCls; ++c) {
      if (!UNC && c == 7u) {
        if (lane == 0) s_wcnt[wave][c] = 0u;
        continue;
      }
      const uint64_t m = __ballot(cls == c);
      if (c != 8u) {
        const uint32_t r = lane_rank(m);
        if (cls == c) rank = r;
      }
      if (lane == 0) s_wcnt[wave][c] = (uint32_t)__popcll(m);
    }
    // misses per request slot: one lane per slot group adds to the wave's row
    for (uint64_t todo = __ballot(miss); todo;) {
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const uint32_t sl = (uint32_t)__builtin_amdgcn_readlane((int)slot, leader);
      const uint64_t grp = __ballot(miss && slot == sl);
      if (lane == leader) s_wmiss[wave][sl] += (uint32_t)__popcll(grp);
      todo &= ~grp;
    }
    // jumped rays are counted in their new cells for the next round
    if constexpr (UNC) atomic_count_grouped(a.counts_next, a.cs, dest, status == kOutJump && (uint32_t)tid < count);
    lds_barrier();
    if (tid == 0) {
      uint32_t tot[kCls];
#pragma unroll
      for (int c = 0; c < kCls; ++c) tot[c] = s_wcnt[0][c] + s_wcnt[1][c] + s_wcnt[2][c] + s_wcnt[3][c];
      if (UNC && tot[7]) s_jbase = atomicAdd(a.n_jump, tot[7]);
      uint32_t off = 0;
      for (int f = 0; f < 7; ++f) {
        s_foff[f] = off;
        off += tot[f];
      }
      a.chunk_out[4 * job] = make_uint4(tot[0], tot[1], tot[2], tot[3]);
      a.chunk_out[4 * job + 1] = make_uint4(tot[4], tot[5], tot[6], tot[8]);
      if (tot[8]) atomicAdd(&a.hit_count[(size_t)cell * a.cs], tot[8]);
      ++wg_chunks;
    } else if (tid <= 7) {
      // run f = tid - 1 reserves its place in the destination cell's next bin
      // (an empty run adds 0 to this cell); the offset is stored during the
      // next work item, after a wait that staging makes anyway, so the
      // atomic's round trip is never waited for on its own
      const uint32_t f = (uint32_t)tid - 1u, n = s_wcnt[0][f] + s_wcnt[1][f] + s_wcnt[2][f] + s_wcnt[3][f];
      pend_off = atomicAdd(&a.runs_next[(size_t)(n ? neighbor_cell(sg, cell, (int)f) : cell) * a.cs], n);
      pend_job = job;
    }
    lds_barrier();
    if (cls < 8u) {
      // rank among the item's rays of this class: the waves before this one first
      for (int w = 0; w < wave; ++w) rank += s_wcnt[w][cls];
      if (cls < 7u)
        a.U[start + s_foff[face] + rank] =
            RayRec{t, t_entry, neighbor_cell(sg, cell, (int)face) | (steps << kCellBits), s_rid[tid]};
      else if (UNC)
        a.jump[s_jbase + rank] = RayRec{t, t_entry, dest | (steps << kCellBits), s_rid[tid]};
    }
    if (tid == 0) {   // the next work item, and its counters cleared
      for (int i = 0; i < 6; ++i) s_job[i] = s_jn[i];
      clear_item();
    }
    lds_barrier();
  }
  if (tid >= 1 && tid <= 7 && pend_job != kNoJob)
    reinterpret_cast<uint32_t*>(a.chunk_out)[16u * pend_job + 8u + (uint32_t)tid - 1u] = pend_off;
  if (lane == 0) {
    s_wtot[wave][0] = wv_evals;
    s_wtot[wave][1] = wv_tiles;
  }
  __syncthreads();
  if (tid < kMaxSlots) {
    const uint32_t m = s_wmiss[0][tid] + s_wmiss[1][tid] + s_wmiss[2][tid] + s_wmiss[3][tid];
    if (m) atomicAdd(&a.tabs.miss_done[tid], m);
  }
  if (tid == 0 && wg_chunks) {   // this workgroup's line of the tallies
    unsigned long long* ev = a.evals + (size_t)(blockIdx.x % kTallyLines) * 16u;
    atomicAdd(&ev[0], s_wtot[0][0] + s_wtot[1][0] + s_wtot[2][0] + s_wtot[3][0]);
    atomicAdd(&ev[1], s_wtot[0][1] + s_wtot[1][1] + s_wtot[2][1] + s_wtot[3][1]);
    atomicAdd(&ev[2], wg_chunks);
  }
}

// ---------------------------------------------------------------------------
// Full float32 SDF MLP on a tile of 4 points x 4 columns (value and the three
// world-axis tangents, forward mode): returns the output rows 4g..4g+3 of
// this lane's column.  Weights are read from the LDS block as MFMA fragments.
// ---------------------------------------------------------------------------
template <int H, int C = 4>
__device__ __forceinline__ f32x4 sdf_full(const float* blk, int lane, int g, bool value_col,
                                          const float (&v)[kPeSlots], SoftplusK k) {
  constexpr int NB = H / 16, S1 = NB * kPeSlots, S2 = S1 + NB * (H / 4);
  const float* vec = blk + 64 * shade_frag_slots(H);
  f32x4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
    acc[b] = value_col ? *reinterpret_cast<const f32x4*>(vec + 16 * b + 4 * g) : f32x4{0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < kPeSlots; ++q)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = mfma_f32(blk[(b * kPeSlots + q) * 64 + lane], v[q], acc[b]);
  float a1[NB][4];
#pragma unroll
  for (int b = 0; b < NB; ++b) act_forward<C>(acc[b], lane & (C - 1), value_col, k, a1[b]);
  f32x4 acc2[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
    acc2[b] = value_col ? *reinterpret_cast<const f32x4*>(vec + H + 16 * b + 4 * g) : f32x4{0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < H / 4; ++q)
#pragma unroll
    for (int b = 0; b < NB; ++b)
      acc2[b] = mfma_f32(blk[(S1 + b * (H / 4) + q) * 64 + lane], a1[q / 4][q % 4], acc2[b]);
  float a2[NB][4];
#pragma unroll
  for (int b = 0; b < NB; ++b) act_forward<C>(acc2[b], lane & (C - 1), value_col, k, a2[b]);
  f32x4 y = value_col ? *reinterpret_cast<const f32x4*>(vec + 2 * H + 4 * g) : f32x4{0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < H / 4; ++q) y = mfma_f32(blk[(S2 + q) * 64 + lane], a2[q / 4][q % 4], y);
  return y;
}

// ---------------------------------------------------------------------------
// The same SDF MLP (value and tangent columns) on bfloat16 MFMA with split
// operands: every weight w is hi + lo with hi = bf16(w), lo = bf16(w - hi)
// (packed on the host), every layer input x likewise (split here), and each
// product is wh*xh + wh*xl + wl*xh, accumulated in float32; the dropped wl*xl
// term and the rounding of the lo parts leave a relative error of about 2^-16
// per product.  Fragment layout of the bf16 march (units in unit_bf16 order),
// biases and activations as in sdf_full.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void split_bf16x8(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const __bf16 h = (__bf16)x[i];
    hi[i] = h;
    lo[i] = (__bf16)(x[i] - (float)h);
  }
}

__device__ __forceinline__ f32x4 mfma_split(uint4 wh, uint4 wl, bf16x8 xh, bf16x8 xl, f32x4 c) {
  c = mfma_bf16(__builtin_bit_cast(bf16x8, wl), xh, c);
  c = mfma_bf16(__builtin_bit_cast(bf16x8, wh), xl, c);
  return mfma_bf16(__builtin_bit_cast(bf16x8, wh), xh, c);
}

template <int H, int C = 4>
__device__ __forceinline__ f32x4 sdf_full3(const float* blk, int lane, int g, bool value_col,
                                           const float (&v)[kPeSlots], SoftplusK k) {
  constexpr int NB = H / 16, F1 = NB * 2, F2 = F1 + NB * (H / 32), NF = shade3_frags(H);
  const uint4* fh = reinterpret_cast<const uint4*>(blk);
  const uint4* fl = fh + NF * 64;
  const float* vec = blk + 2 * 256 * NF + 64 * 32;
  bf16x8 eh[2], el[2];
  {
    float x0[8], x1[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      x0[i] = v[i];
      x1[i] = i < kPeSlots - 8 ? v[8 + i] : 0.0f;
    }
    split_bf16x8(x0, eh[0], el[0]);
    split_bf16x8(x1, eh[1], el[1]);
  }
  f32x4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    acc[b] = value_col ? *reinterpret_cast<const f32x4*>(vec + 16 * b + 4 * g) : f32x4{0, 0, 0, 0};
    const uint4 h0 = fh[(2 * b) * 64 + lane], h1 = fh[(2 * b + 1) * 64 + lane];
    const uint4 l0 = fl[(2 * b) * 64 + lane], l1 = fl[(2 * b + 1) * 64 + lane];
    acc[b] = mfma_split(h0, l0, eh[0], el[0], acc[b]);
    acc[b] = mfma_split(h1, l1, eh[1], el[1], acc[b]);
  }
  float a1[NB][4];
#pragma unroll
  for (int b = 0; b < NB; ++b) act_forward<C>(acc[b], lane & (C - 1), value_col, k, a1[b]);
  f32x4 acc2[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
    acc2[b] = value_col ? *reinterpret_cast<const f32x4*>(vec + H + 16 * b + 4 * g) : f32x4{0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < H / 32; ++c) {
    float x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = a1[2 * c + i / 4][i % 4];
    bf16x8 xh, xl;
    split_bf16x8(x, xh, xl);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int f = F1 + b * (H / 32) + c;
      acc2[b] = mfma_split(fh[f * 64 + lane], fl[f * 64 + lane], xh, xl, acc2[b]);
    }
  }
  float a2[NB][4];
#pragma unroll
  for (int b = 0; b < NB; ++b) act_forward<C>(acc2[b], lane & (C - 1), value_col, k, a2[b]);
  f32x4 y = value_col ? *reinterpret_cast<const f32x4*>(vec + 2 * H + 4 * g) : f32x4{0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < H / 32; ++c) {
    float x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = a2[2 * c + i / 4][i % 4];
    bf16x8 xh, xl;
    split_bf16x8(x, xh, xl);
    y = mfma_split(fh[(F2 + c) * 64 + lane], fl[(F2 + c) * 64 + lane], xh, xl, y);
  }
  return y;
}

// Encoding slot e (0..32) of the color input [x_l(3), gamma_4(v)(27), n(3)].
__device__ __forceinline__ float color_in_slot(int e, const float xl[3], const float v[3],
                                               const float n[3]) {
  if (e < 3) return xl[e];
  if (e < 30) {
    const int i = e - 3;
    if (i < 3) return v[i];
    const int a = (i - 3) / 8, k = ((i - 3) % 8) / 2;
    const float r = v[a] * ldexpf(1.0f, k - 1);
    return ((i - 3) & 1) ? cos_rev(r) : sin_rev(r);
  }
  return n[e - 30];
}

// ---------------------------------------------------------------------------
// shading: per chunk of a cell's hits; each wave shades 4 hits per tile
// ---------------------------------------------------------------------------
template <int HM, int C = 4, bool B3 = false>
__device__ __forceinline__ f32x4 sdf_full_h(int H, const float* blk, int lane, int g, bool value_col,
                                            const float (&v)[kPeSlots], SoftplusK k) {
  if constexpr (B3) {
    if constexpr (HM != 0) {
      return sdf_full3<HM, C>(blk, lane, g, value_col, v, k);
    } else {
      if (H == 64) return sdf_full3<64, C>(blk, lane, g, value_col, v, k);
      return sdf_full3<32, C>(blk, lane, g, value_col, v, k);
    }
  } else if constexpr (HM != 0) {
    return sdf_full<HM, C>(blk, lane, g, value_col, v, k);
  } else {
    if (H == 64) return sdf_full<64, C>(blk, lane, g, value_col, v, k);
    return sdf_full<32, C>(blk, lane, g, value_col, v, k);
  }
}

// PT: path tracing; the hit scatters (Lambertian, albedo = color MLP) or
// ends its path; otherwise the color is the pixel's rgb.  B3: the SDF MLP
// from the split-bfloat16 block (pools marching in bf16 or fp8), else from
// the float32 block.
// 3 waves per SIMD: the shading chain (MFMA -> softplus -> MFMA) is
// latency-bound, and 3 waves fit in the register file without spills
template <int HM, bool PT, bool B3>
__global__ __launch_bounds__(256, 3) void k_shade(ShadeArgs a) {
  extern __shared__ __align__(16) float s_mem[];
  float* s_stage = s_mem;                 // 4 waves x 4 hits x 48
  float* s_block = s_mem + 4 * 4 * kColIn;
  __shared__ uint32_t s_job[7];   // cell, start, count, valid, batch cursor, batch end, scene
  __shared__ uint32_t s_done[kMaxSlots];   // paths / rays finished here, per request slot
  const int lane = lane_id(), g = lane >> 4, col = lane & 15, h = col >> 2, s = col & 3;
  const int wave = threadIdx.x >> 6;
  const bool value_col = s == 0;
  const PeLane pl = make_pe_lane(g);
  uint32_t loaded = 0xFFFFFFFFu;
  // this wave's block of the spawn list [sp_cur, sp_end) (path tracing)
  uint32_t sp_cur = 0, sp_end = 0;
  if (threadIdx.x < kMaxSlots) s_done[threadIdx.x] = 0u;
  if (threadIdx.x == 0) s_job[4] = s_job[5] = 0u;
  for (;;) {
    if (threadIdx.x == 0) {
      next_item(a.grab, *a.n_chunks, a.chunks, s_job);
      if (s_job[3]) s_job[6] = scene_of(a.tabs, s_job[0]);
    }
    __syncthreads();
    if (!s_job[3]) break;
    const uint32_t cell = s_job[0], start = s_job[1], count = s_job[2];
    const SceneEnt* se = a.tabs.scenes + __builtin_amdgcn_readfirstlane(s_job[6]);
    const SceneGeom sg = se->sg;
    const SoftplusK spk = se->spk;
    const int H = HM ? HM : sg.H;
    const uint32_t lc = cell - sg.cell_base;
    if (cell != loaded) {
      stage_block(s_block, se->shade + (size_t)lc * se->shade_words, se->shade_words);
      stage_wait();
      __syncthreads();
      loaded = cell;
    }
    // colour fragments (one float per lane) and the bias vector
    const float* cfr = B3 ? s_block + 2 * 256 * shade3_frags(H)
                          : s_block + 64 * ((H / 16) * kPeSlots + (H / 16) * (H / 4) + H / 4);
    const float* vec = cfr + 64 * 32;
    const CellBox cb = cell_box(sg, lc);
    float* stage = s_stage + wave * 4 * kColIn;
    // each wave takes 8 hits: two 2-column passes (value and derivative
    // along the ray) give the two Newton steps of all 8, then a 4-column pass
    // per 4 hits (value and world gradient) at the refined point gives the
    // normal, the feature and the color
    const int hA = col >> 1, sA = col & 1;
    for (uint32_t base = (uint32_t)wave * 8u; base < count; base += 32u) {
      float tA;
      RayRec rA;
      RayStatic sA_;
      {
        const uint32_t idx = base + (uint32_t)hA;
        const bool valid = idx < count;
        rA = valid ? a.S[start + idx] : RayRec{0, 0, cell, 0};
        sA_ = valid ? a.rs[rA.rid] : RayStatic{0, 0, 0, 0, 0, 0, 1, 0};
        const RayRec& r = rA;
        const RayStatic& st = sA_;
        const float o[3] = {st.ox, st.oy, st.oz}, d[3] = {st.dx, st.dy, st.dz};
        int eax;
        const float ce = cell_exit(sg, cb, o, d, &eax);
        tA = r.t;
#pragma unroll 1
        for (int it = 0; it < 2; ++it) {
          asm volatile("" ::: "memory");
          float xl[3];
#pragma unroll
          for (int k = 0; k < 3; ++k) xl[k] = valid ? fmaf(fmaf(tA, d[k], o[k]), sg.inv_half[k], cb.cs[k]) : 0.0f;
          float v[kPeSlots];
          pe_values_dir(pl, sA == 0, d[0] * sg.inv_half[0], d[1] * sg.inv_half[1], d[2] * sg.inv_half[2],
                        xl[0], xl[1], xl[2], v);
          const f32x4 y = sdf_full_h<HM, 2, B3>(H, s_block, lane, g, sA == 0, v, spk);
          const float f0 = __shfl(y[0], 2 * hA), gd = __shfl(y[0], 2 * hA + 1);
          if (gd < -1e-3f) tA = fminf(fmaxf(tA - f0 / gd, r.t_entry), ce);
        }
      }
#pragma unroll 1
      for (int half = 0; half < 2; ++half) {
      const uint32_t hh = 4u * (uint32_t)half + (uint32_t)h;   // hit of this half
      const uint32_t idx = base + hh;
      const bool valid = idx < count;
      // this hit's records, from the lanes that held it in the Newton passes
      const int src = 2 * (int)hh;
      const float t = __shfl(tA, src);
      const RayRec r{__shfl(rA.t, src), __shfl(rA.t_entry, src), (uint32_t)__shfl((int)rA.key, src),
                     (uint32_t)__shfl((int)rA.rid, src)};
      const RayStatic st{__shfl(sA_.ox, src), __shfl(sA_.oy, src), __shfl(sA_.oz, src), __shfl(sA_.t_far, src),
                         __shfl(sA_.dx, src), __shfl(sA_.dy, src), __shfl(sA_.dz, src),
                         (uint32_t)__shfl((int)sA_.pix, src)};
      const float o[3] = {st.ox, st.oy, st.oz}, d[3] = {st.dx, st.dy, st.dz};
      float xl[3], gr[3];
      f32x4 y;
      {
        asm volatile("" ::: "memory");
#pragma unroll
        for (int k = 0; k < 3; ++k) xl[k] = valid ? fmaf(fmaf(t, d[k], o[k]), sg.inv_half[k], cb.cs[k]) : 0.0f;
        float v[kPeSlots];
        const float ih = s == 1 ? sg.inv_half[0] : s == 2 ? sg.inv_half[1] : s == 3 ? sg.inv_half[2] : 0.0f;
        pe_values_tangent(pl, s, ih, xl[0], xl[1], xl[2], v);
        y = sdf_full_h<HM, 4, B3>(H, s_block, lane, g, value_col, v, spk);
        const int src = 4 * h;
        gr[0] = __shfl(y[0], src + 1);
        gr[1] = __shfl(y[0], src + 2);
        gr[2] = __shfl(y[0], src + 3);
      }
      const float gn2 = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
      float n[3];
      if (!(gn2 > 1e-38f)) {
        n[0] = -d[0]; n[1] = -d[1]; n[2] = -d[2];
      } else {
        const float inv = 1.0f / sqrtf(gn2);
        n[0] = gr[0] * inv; n[1] = gr[1] * inv; n[2] = gr[2] * inv;
      }
      // stage the color input of the 4 hits of this tile
      wave_lds_sync();
      {
        const int kk = 4 * g + s;  // 0..15 within the hit
        stage[h * kColIn + kk] = color_in_slot(kk, xl, d, n);
        if (kk + 16 < 33) stage[h * kColIn + kk + 16] = color_in_slot(kk + 16, xl, d, n);
        if (kk == 15) stage[h * kColIn + 32] = color_in_slot(32, xl, d, n);
        if (value_col) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int orow = 4 * g + rr;
            if (orow >= 1) stage[h * kColIn + 33 + orow - 1] = y[rr];
          }
        }
      }
      wave_lds_sync();
      const float* vc = vec + 2 * H + 16;   // bc1[32], bc2[4]
      f32x4 c1[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) c1[b] = *reinterpret_cast<const f32x4*>(vc + 16 * b + 4 * g);
#pragma unroll
      for (int q = 0; q < 12; ++q) {
        const float bq = stage[h * kColIn + 4 * q + g];
#pragma unroll
        for (int b = 0; b < 2; ++b) c1[b] = mfma_f32(cfr[(b * 12 + q) * 64 + lane], bq, c1[b]);
      }
      f32x4 c2 = g == 0 ? *reinterpret_cast<const f32x4*>(vc + 32) : f32x4{0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < 8; ++q)
        c2 = mfma_f32(cfr[(24 + q) * 64 + lane], fmaxf(c1[q / 4][q % 4], 0.0f), c2);
      const bool writer = valid && g == 0 && value_col;
      const uint32_t slot = st.pix >> kPixBits;
      bool done = writer, spawn = false, wgo = false;
      uint32_t ncell = 0;
      RayRec nrec{0, 0, 0, 0};
      if (writer) {
        // copied before the first store, so all its fields load together
        // (a store through an output pointer could otherwise alias the table)
        ReqEnt q = a.tabs.reqs[slot];
        const OutPtrs& out = q.out;
        const uint32_t px = st.pix & kPixMask;
        const float rgb[3] = {sigmoid(c2[0]), sigmoid(c2[1]), sigmoid(c2[2])};
        bool aux = true;
        PathRec pr;
        uint32_t smp = 0;
        if constexpr (PT) {
          pr = a.tabs.path[r.rid];
          smp = r.rid % q.spp;
          aux = pr.bounce == 0 && smp == 0;
          if (q.world) q.out.seg = nullptr;   // no segment records in worlds
        } else {
          gmem(out.rgb)[3 * px + 0] = rgb[0];
          gmem(out.rgb)[3 * px + 1] = rgb[1];
          gmem(out.rgb)[3 * px + 2] = rgb[2];
        }
        if (aux) {
          if (out.depth) gmem(out.depth)[px] = se->ws * t;   // world distance (ws = 1 outside worlds)
          if (out.normal) {
            gmem(out.normal)[3 * px + 0] = n[0];
            gmem(out.normal)[3 * px + 1] = n[1];
            gmem(out.normal)[3 * px + 2] = n[2];
          }
          if (out.hit) gmem(out.hit)[px] = 1;
          if (out.steps) gmem(out.steps)[px] = (uint16_t)(r.key >> kCellBits);
          if (out.trace) {
            auto tr = gmem(out.trace + px);
            tr->t_march = r.t;
            tr->t_entry = r.t_entry;
            tr->cell = (int32_t)cell;
            tr->status = kHit;
          }
        }
        if constexpr (PT) {
          if (out.seg) {
            auto& sr = *gmem(out.seg + (size_t)r.rid * (q.bounces + 1u) + pr.bounce);
            sr.t_march = r.t;
            sr.t_entry = r.t_entry;
            sr.t = t;
            for (int c = 0; c < 3; ++c) {
              sr.n[c] = n[c];
              sr.albedo[c] = rgb[c];
            }
            sr.cell = (int32_t)cell;
            sr.status = kHit;
            sr.steps = r.key >> kCellBits;
          }
          if (pr.bounce < q.bounces) {
            // scatter: cosine-weighted about n, throughput x albedo, the new
            // segment starts 1e-3 off the surface
            for (int c = 0; c < 3; ++c) pr.T[c] *= rgb[c];
            float u1, u2, nd[3], no[3];
            path_uniforms(q.seed_lo, q.seed_hi, px, q.sample_offset + smp, pr.bounce + 1u, &u1, &u2);
            cosine_dir(n, u1, u2, nd);
            ++pr.bounce;
            if (q.world) {
              // the path goes on in the world from 1e-3 (world units) off the surface
              WorldRec wr;
              for (int c = 0; c < 3; ++c) {
                wr.o[c] = se->wt[c] + se->ws * (o[c] + t * d[c]) + 1e-3f * n[c];
                wr.d[c] = nd[c];
              }
              wr.tpm = 0.0f;
              wr.tim = 0.0f;
              wr.rid = r.rid;
              wr.pad[0] = wr.pad[1] = wr.pad[2] = 0u;
              a.wlist[atomicAdd(a.n_w, 1u)] = wr;   // world renders only
              wgo = true;
              done = false;
            }
            for (int c = 0; c < 3; ++c) no[c] = o[c] + t * d[c] + 1e-3f * n[c];
            if (out.seg) {
              auto& sn = *gmem(out.seg + (size_t)r.rid * (q.bounces + 1u) + pr.bounce);
              for (int c = 0; c < 3; ++c) {
                sn.o[c] = no[c];
                sn.d[c] = nd[c];
              }
            }
            float t0, tf;
            if (wgo) {
            } else if (slab(sg, no, nd, &t0, &tf)) {
              ncell = entry_cell(sg, no, nd, t0);
              a.rs[r.rid] = RayStatic{no[0], no[1], no[2], tf, nd[0], nd[1], nd[2], st.pix};
              nrec = RayRec{t0, t0, ncell, r.rid};
              spawn = true;
              done = false;
            } else {
              float e[3];
              env_lookup(q.env, q.env_w, q.env_h, nd, e);
              for (int c = 0; c < 3; ++c) pr.L[c] += pr.T[c] * e[c];
              if (out.seg) gmem(out.seg + (size_t)r.rid * (q.bounces + 1u) + pr.bounce)->status = kBoxMiss;
            }
          }
          a.tabs.path[r.rid] = pr;
        }
      }
      if constexpr (PT) {
        const uint64_t sm = __ballot(spawn);
        const uint32_t ns = (uint32_t)__popcll(sm);
        if (ns) {
          if (sp_cur + ns > sp_end) {
            // close the block (fill its rest with invalid records), take a new one
            for (uint32_t i = sp_cur + (uint32_t)lane; i < sp_end; i += 64u) a.spawn[i] = RayRec{0, 0, kInvalidKey, 0};
            uint32_t b = 0;
            if (lane == 0) b = atomicAdd(a.n_spawn, kSpawnBlock);
            sp_cur = __shfl(b, 0);
            sp_end = sp_cur + kSpawnBlock;
          }
          if (spawn) a.spawn[sp_cur + lane_rank(sm)] = nrec;
          sp_cur += ns;
        }
        atomic_count_grouped(a.counts_next, a.cs, ncell, spawn);
      }
      if (done) atomicAdd(&s_done[slot], 1u);
      }
    }
    __syncthreads();
  }
  if constexpr (PT) {
    for (uint32_t i = sp_cur + (uint32_t)lane; i < sp_end; i += 64u) a.spawn[i] = RayRec{0, 0, kInvalidKey, 0};
  }
  if (threadIdx.x < kMaxSlots && s_done[threadIdx.x]) atomicAdd(&a.tabs.hit_done[threadIdx.x], s_done[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// batched point query: bin points by cell, then evaluate
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_query_bin(QueryBinArgs a) {
  const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  const bool valid = i < a.n;
  uint32_t cell = 0;
  if (valid) {
    int idx[3];
    for (int k = 0; k < 3; ++k) {
      int c = (int)floorf((a.pts[3 * i + k] - a.sg.bmin[k]) * a.sg.inv_side[k]);
      idx[k] = min(max(c, 0), a.sg.N - 1);
    }
    cell = a.sg.cell_base + (uint32_t)(idx[0] + a.sg.N * (idx[1] + a.sg.N * idx[2]));
    a.U[i] = RayRec{0.0f, 0.0f, cell, (uint32_t)i};
  }
  atomic_count_grouped(a.counts, a.cs, cell, valid);
}

template <int H, int P>
__global__ __launch_bounds__(256) void k_query_d(QueryArgs a) {
  extern __shared__ __align__(16) float s_block[];
  __shared__ uint32_t s_job[6];   // cell, start, count, valid, batch cursor, batch end
  const int lane = lane_id(), g = lane >> 4, p = lane & 15, wave = threadIdx.x >> 6;
  const PeLane pl = make_pe_lane(g);
  const SceneGeom& sg = a.sg;
  uint32_t loaded = 0xFFFFFFFFu;
  if (threadIdx.x == 0) s_job[4] = s_job[5] = 0u;
  for (;;) {
    if (threadIdx.x == 0) next_item(a.grab, *a.n_chunks, a.chunks, s_job);
    __syncthreads();
    if (!s_job[3]) break;
    const uint32_t cell = s_job[0], start = s_job[1], count = s_job[2];
    const uint32_t lc = cell - sg.cell_base;
    if (cell != loaded) {
      stage_block(s_block, a.blocks + (size_t)lc * a.block_words, a.block_words);
      stage_wait();
      __syncthreads();
      loaded = cell;
    }
    const CellBox cb = cell_box(sg, lc);
    for (uint32_t base = (uint32_t)wave * 16u; base < count; base += 64u) {
      const uint32_t idx = base + (uint32_t)p;
      const bool valid = idx < count;
      const uint32_t pi = valid ? a.S[start + idx].rid : 0u;
      float xl[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) xl[k] = valid ? fmaf(a.pts[3 * (size_t)pi + k], sg.inv_half[k], cb.cs[k]) : 0.0f;
      float v[kPeSlots];
      pe_values<false>(pl, xl[0], xl[1], xl[2], v);
      const float f = march_eval<H, P>(s_block, lane, g, v, a.spk);
      if (valid && g == 0) a.d_out[pi] = f;
    }
    __syncthreads();
  }
}

template <int H>
__global__ __launch_bounds__(256) void k_query_full(QueryArgs a) {
  extern __shared__ __align__(16) float s_block[];
  __shared__ uint32_t s_job[6];   // cell, start, count, valid, batch cursor, batch end
  const int lane = lane_id(), g = lane >> 4, col = lane & 15, h = col >> 2, s = col & 3;
  const int wave = threadIdx.x >> 6;
  const PeLane pl = make_pe_lane(g);
  const SceneGeom& sg = a.sg;
  uint32_t loaded = 0xFFFFFFFFu;
  if (threadIdx.x == 0) s_job[4] = s_job[5] = 0u;
  for (;;) {
    if (threadIdx.x == 0) next_item(a.grab, *a.n_chunks, a.chunks, s_job);
    __syncthreads();
    if (!s_job[3]) break;
    const uint32_t cell = s_job[0], start = s_job[1], count = s_job[2];
    const uint32_t lc = cell - sg.cell_base;
    if (cell != loaded) {
      stage_block(s_block, a.blocks + (size_t)lc * a.block_words, a.block_words);
      stage_wait();
      __syncthreads();
      loaded = cell;
    }
    const CellBox cb = cell_box(sg, lc);
    for (uint32_t base = (uint32_t)wave * 4u; base < count; base += 16u) {
      const uint32_t idx = base + (uint32_t)h;
      const bool valid = idx < count;
      const uint32_t pi = valid ? a.S[start + idx].rid : 0u;
      float xl[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) xl[k] = valid ? fmaf(a.pts[3 * (size_t)pi + k], sg.inv_half[k], cb.cs[k]) : 0.0f;
      float v[kPeSlots];
      pe_values_tangent(pl, s, s ? sg.inv_half[s - 1] : 0.0f, xl[0], xl[1], xl[2], v);
      const f32x4 y = sdf_full<H>(s_block, lane, g, s == 0, v, a.spk);
      if (valid) {
        if (g == 0 && s == 0 && a.d_out) a.d_out[pi] = y[0];
        if (g == 0 && s > 0 && a.grad_out) a.grad_out[3 * (size_t)pi + s - 1] = y[0];
        if (s == 0 && a.z_out) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int orow = 4 * g + rr;
            if (orow >= 1) a.z_out[15 * (size_t)pi + orow - 1] = y[rr];
          }
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// dense lattice sampling (mesh-extraction input, Sec. 4.1): the R^3 lattice
// spanning the box is already grouped by cell, so it needs no binning.  A
// work item is (cell, a 256-point part of the cell's lattice points); each
// persistent workgroup takes a contiguous range of items, so it stages a
// cell's weights once for all of that cell's items in its range.
// ---------------------------------------------------------------------------
// first lattice index along an axis whose cell floor(i N / (R - 1)) is c
__device__ __forceinline__ uint32_t grid_lo(uint32_t c, uint32_t N, uint32_t R) {
  return (c * (R - 1u) + N - 1u) / N;
}
// one past the last (the last cell also takes the lattice plane on the box face)
__device__ __forceinline__ uint32_t grid_hi(uint32_t c, uint32_t N, uint32_t R) {
  return c + 1u >= N ? R : grid_lo(c + 1u, N, R);
}

struct GridItem {
  uint32_t lc, q0, cnt, nx, nxy;
  uint32_t lo[3];
};

__device__ __forceinline__ GridItem grid_item(const GridArgs& a, uint64_t it, const CellBox& cb, uint32_t lc) {
  GridItem gi;
  const uint32_t N = (uint32_t)a.sg.N;
  const uint32_t idx[3] = {(uint32_t)cb.ix, (uint32_t)cb.iy, (uint32_t)cb.iz};
  uint32_t n[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gi.lo[k] = grid_lo(idx[k], N, a.R);
    n[k] = grid_hi(idx[k], N, a.R) - gi.lo[k];
  }
  gi.lc = lc;
  gi.q0 = (uint32_t)(it % a.K) * 256u;
  gi.nx = n[0];
  gi.nxy = n[0] * n[1];
  gi.cnt = gi.nxy * n[2];
  return gi;
}

// lattice point q of the item's cell: its flat output index and local
// coordinates x_l = (2 N i - (2 c + 1)(R - 1)) / (R - 1) per axis (the box
// cancels); the numerator is an exact integer, so x_l is rounded once
__device__ __forceinline__ uint64_t grid_point(const GridArgs& a, const GridItem& gi, const CellBox& cb, uint32_t q,
                                               float xl[3]) {
  const uint32_t c = q / gi.nxy, r = q - c * gi.nxy, b = r / gi.nx, i = r - b * gi.nx;
  const uint32_t ijk[3] = {gi.lo[0] + i, gi.lo[1] + b, gi.lo[2] + c};
  const int idx[3] = {cb.ix, cb.iy, cb.iz};
  const int N = a.sg.N, rm1 = (int)a.R - 1;
#pragma unroll
  for (int k = 0; k < 3; ++k) xl[k] = (float)(2 * N * (int)ijk[k] - (2 * idx[k] + 1) * rm1) / a.rm1;
  return (uint64_t)ijk[0] + (uint64_t)a.R * ((uint64_t)ijk[1] + (uint64_t)a.R * (uint64_t)ijk[2]);
}

template <int H, int P>
__global__ __launch_bounds__(256) void k_grid_d(GridArgs a) {
  extern __shared__ __align__(16) float s_block[];
  const int lane = lane_id(), g = lane >> 4, p = lane & 15, wave = threadIdx.x >> 6;
  const PeLane pl = make_pe_lane(g);
  const uint32_t N = (uint32_t)a.sg.N;
  const uint64_t T = (uint64_t)N * N * N * a.K;
  const uint64_t it0 = T * blockIdx.x / gridDim.x, it1 = T * (blockIdx.x + 1u) / gridDim.x;
  uint32_t loaded = 0xFFFFFFFFu;
  for (uint64_t it = it0; it < it1; ++it) {
    const uint32_t lc = (uint32_t)(it / a.K);
    const CellBox cb = cell_box(a.sg, lc);
    const GridItem gi = grid_item(a, it, cb, lc);
    if (gi.q0 >= gi.cnt) continue;   // the cell has fewer parts (uniform)
    if (lc != loaded) {
      __syncthreads();   // every wave is done with the previous cell's block
      stage_block(s_block, a.blocks + (size_t)lc * a.block_words, a.block_words);
      stage_wait();
      __syncthreads();
      loaded = lc;
    }
    for (uint32_t t = (uint32_t)wave; t < 16u; t += 4u) {
      const uint32_t q = gi.q0 + 16u * t + (uint32_t)p;
      const bool valid = q < gi.cnt;
      float xl[3] = {0.0f, 0.0f, 0.0f};
      uint64_t o = 0;
      if (valid) o = grid_point(a, gi, cb, q, xl);
      float v[kPeSlots];
      pe_values<false>(pl, xl[0], xl[1], xl[2], v);
      const float f = march_eval<H, P>(s_block, lane, g, v, a.spk);
      if (valid && g == 0) a.d_out[o] = f;
    }
  }
}

// value and world gradient (float32 shading block, forward mode: 4 points x
// 4 columns per tile)
template <int H>
__global__ __launch_bounds__(256) void k_grid_full(GridArgs a) {
  extern __shared__ __align__(16) float s_block[];
  const int lane = lane_id(), g = lane >> 4, col = lane & 15, h = col >> 2, s = col & 3;
  const int wave = threadIdx.x >> 6;
  const PeLane pl = make_pe_lane(g);
  const uint32_t N = (uint32_t)a.sg.N;
  const uint64_t T = (uint64_t)N * N * N * a.K;
  const uint64_t it0 = T * blockIdx.x / gridDim.x, it1 = T * (blockIdx.x + 1u) / gridDim.x;
  uint32_t loaded = 0xFFFFFFFFu;
  for (uint64_t it = it0; it < it1; ++it) {
    const uint32_t lc = (uint32_t)(it / a.K);
    const CellBox cb = cell_box(a.sg, lc);
    const GridItem gi = grid_item(a, it, cb, lc);
    if (gi.q0 >= gi.cnt) continue;
    if (lc != loaded) {
      __syncthreads();
      stage_block(s_block, a.blocks + (size_t)lc * a.block_words, a.block_words);
      stage_wait();
      __syncthreads();
      loaded = lc;
    }
    for (uint32_t t = (uint32_t)wave; t < 64u; t += 4u) {
      const uint32_t q = gi.q0 + 4u * t + (uint32_t)h;
      const bool valid = q < gi.cnt;
      float xl[3] = {0.0f, 0.0f, 0.0f};
      uint64_t o = 0;
      if (valid) o = grid_point(a, gi, cb, q, xl);
      float v[kPeSlots];
      pe_values_tangent(pl, s, s ? a.sg.inv_half[s - 1] : 0.0f, xl[0], xl[1], xl[2], v);
      const f32x4 y = sdf_full<H>(s_block, lane, g, s == 0, v, a.spk);
      if (valid && g == 0) {
        if (s == 0) a.d_out[o] = y[0];
        else if (a.grad_out) a.grad_out[3u * o + (uint32_t)(s - 1)] = y[0];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// eikonal term by central differences (Sec. 3.2, Sec. 3.3): the six stencil
// points of each point, then (after a point query of the stencil) the
// gradient norms and the mean squared residual
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_eik_points(EikArgs a) {
  const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (i >= 6u * a.n) return;
  const uint64_t q = i / 6u;
  const uint32_t s = (uint32_t)(i - 6u * q), ax = s >> 1;
  float x[3] = {a.pts[3u * q], a.pts[3u * q + 1u], a.pts[3u * q + 2u]};
  x[ax] = (s & 1u) ? x[ax] - a.delta : x[ax] + a.delta;   // order +x, -x, +y, -y, +z, -z
#pragma unroll
  for (int k = 0; k < 3; ++k) a.stencil_pts[3u * i + k] = x[k];
}

__global__ __launch_bounds__(256) void k_eik_combine(EikArgs a) {
  __shared__ double s_sum[256];
  const uint64_t q = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  double r = 0.0;
  if (q < a.n) {
    float g2 = 0.0f;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const float ga = (a.stencil[6u * q + 2u * ax] - a.stencil[6u * q + 2u * ax + 1u]) / (2.0f * a.delta);
      g2 = fmaf(ga, ga, g2);
    }
    const float gn = sqrtf(g2);
    a.gnorm[q] = gn;
    r = (double)(gn - 1.0f) * (double)(gn - 1.0f);
  }
  s_sum[threadIdx.x] = r;
  __syncthreads();
  for (uint32_t w = 128u; w; w >>= 1) {
    if (threadIdx.x < w) s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[blockIdx.x] = s_sum[0];
}

// one workgroup: the partial sums in a fixed order, so the loss is the same
// on every run
__global__ __launch_bounds__(256) void k_eik_loss(EikArgs a, uint32_t nparts) {
  __shared__ double s_sum[256];
  double acc = 0.0;
  for (uint32_t i = threadIdx.x; i < nparts; i += 256u) acc += a.partial[i];
  s_sum[threadIdx.x] = acc;
  __syncthreads();
  for (uint32_t w = 128u; w; w >>= 1) {
    if (threadIdx.x < w) s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && a.loss) a.loss[0] = s_sum[0] / (double)a.n;
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_raygen(const RaygenArgs& a, hipStream_t st) {
  if (a.cs == 0) return hipErrorInvalidValue;   // counter stride unset
  const uint32_t npix = (uint32_t)a.W * (uint32_t)a.Hh;
  hipLaunchKernelGGL(k_raygen, dim3((npix + 255u) / 256u), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_scan(const ScanArgs& a, hipStream_t st) {
  if (a.cs == 0) return hipErrorInvalidValue;   // counter stride unset
  if (a.T == 0 || a.T > 512 || (a.T & (a.T - 1u)) != 0) return hipErrorInvalidValue;
  if (!a.ticket || !a.flags || !a.err) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scan, dim3(kScanTiles), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_scatter(const ScatterArgs& a, uint32_t grid, hipStream_t st) {
  if (a.cs == 0) return hipErrorInvalidValue;   // counter stride unset
  hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_scatter_chunks(const ScatterChunksArgs& a, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_chunks, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

size_t march_lds_bytes(uint32_t block_words) {
  return (size_t)block_words * 4u + (size_t)kChunk * (14u * 4u + 2u * 2u);  // 14 words + 2 list slots per ray
}

size_t shade_lds_bytes(uint32_t block_words) { return ((size_t)block_words + 4u * 4u * kColIn) * 4u; }

template <int HM, int P, bool PAIR, int WPE>
static hipError_t march_t(const MarchArgs& a, uint32_t block_words, uint32_t grid, hipStream_t st) {
  const size_t lds = march_lds_bytes(block_words);
  if (!a.jump) {
    hipLaunchKernelGGL((k_march<HM, P, PAIR, WPE, false>), dim3(grid), dim3(256), lds, st, a);
  } else {
    // unclamped steps: kn_render only (one request, H 32 or 64)
    if constexpr (HM == 0) return hipErrorInvalidValue;
    else hipLaunchKernelGGL((k_march<HM, P, PAIR, WPE, true>), dim3(grid), dim3(256), lds, st, a);
  }
  return hipGetLastError();
}

// Per precision: tile pairing and waves per SIMD (measured on 1080p frames of
// a 16^3, H=64 scene; the chosen forms compile without register spills).
template <int HM>
static hipError_t march_p(const MarchArgs& a, int prec, uint32_t block_words, uint32_t grid, hipStream_t st) {
  if (prec == kPrecF32) return march_t<HM, kPrecF32, true, 1>(a, block_words, grid, st);
  if (prec == kPrecBf16) return march_t<HM, kPrecBf16, false, 3>(a, block_words, grid, st);
  if (prec == kPrecFp8) return march_t<HM, kPrecFp8, false, 3>(a, block_words, grid, st);
  return hipErrorInvalidValue;
}

hipError_t launch_march(const MarchArgs& a, int H, int prec, uint32_t block_words, uint32_t grid,
                        hipStream_t st) {
  if (a.cs == 0) return hipErrorInvalidValue;   // counter stride unset
  if (H == 32) return march_p<32>(a, prec, block_words, grid, st);
  if (H == 64) return march_p<64>(a, prec, block_words, grid, st);
  if (H == 0) return march_p<0>(a, prec, block_words, grid, st);
  return hipErrorInvalidValue;
}

template <bool PT, bool B3>
static hipError_t shade_t(const ShadeArgs& a, int H, size_t lds, uint32_t grid, hipStream_t st) {
  if (H == 32) hipLaunchKernelGGL((k_shade<32, PT, B3>), dim3(grid), dim3(256), lds, st, a);
  else if (H == 64) hipLaunchKernelGGL((k_shade<64, PT, B3>), dim3(grid), dim3(256), lds, st, a);
  else if (H == 0) hipLaunchKernelGGL((k_shade<0, PT, B3>), dim3(grid), dim3(256), lds, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_shade(const ShadeArgs& a, int H, int prec, bool pt, uint32_t block_words, uint32_t grid,
                        hipStream_t st) {
  if (a.cs == 0) return hipErrorInvalidValue;   // counter stride unset
  const size_t lds = shade_lds_bytes(block_words);
  const bool b3 = prec != kPrecF32;
  if (pt) return b3 ? shade_t<true, true>(a, H, lds, grid, st) : shade_t<true, false>(a, H, lds, grid, st);
  return b3 ? shade_t<false, true>(a, H, lds, grid, st) : shade_t<false, false>(a, H, lds, grid, st);
}

hipError_t launch_raygen_pt(const RaygenPtArgs& a, hipStream_t st) {
  if (a.cs == 0) return hipErrorInvalidValue;   // counter stride unset
  const uint32_t n = (uint32_t)a.W * (uint32_t)a.Hh * a.spp;
  hipLaunchKernelGGL(k_raygen_pt, dim3((n + 255u) / 256u), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_resolve(const ResolveArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_resolve, dim3((a.npix + 255u) / 256u), dim3(256), 0, st, a);
  return hipGetLastError();
}

// word fill and copy (clearing and restoring counters without memset or
// memcpy nodes, for callers that record the work into graphs)
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, uint32_t n, uint32_t v) {
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) p[i] = v;
}

__global__ __launch_bounds__(256) void k_copy_u32(uint32_t* dst, const uint32_t* src, uint32_t n) {
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) dst[i] = src[i];
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (!p || n > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const uint32_t grid = (uint32_t)std::min<size_t>((n + 255u) / 256u, 1024u);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, st, p, (uint32_t)n, v);
  return hipGetLastError();
}

hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (!dst || !src || n > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const uint32_t grid = (uint32_t)std::min<size_t>((n + 255u) / 256u, 1024u);
  hipLaunchKernelGGL(k_copy_u32, dim3(grid), dim3(256), 0, st, dst, src, (uint32_t)n);
  return hipGetLastError();
}

hipError_t launch_query_bin(const QueryBinArgs& a, hipStream_t st) {
  if (a.cs == 0) return hipErrorInvalidValue;   // counter stride unset
  hipLaunchKernelGGL(k_query_bin, dim3((uint32_t)((a.n + 255u) / 256u)), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int H>
static hipError_t query_d_h(const QueryArgs& a, int prec, size_t lds, uint32_t grid, hipStream_t st) {
  if (prec == kPrecF32) hipLaunchKernelGGL((k_query_d<H, kPrecF32>), dim3(grid), dim3(256), lds, st, a);
  else if (prec == kPrecBf16) hipLaunchKernelGGL((k_query_d<H, kPrecBf16>), dim3(grid), dim3(256), lds, st, a);
  else if (prec == kPrecFp8) hipLaunchKernelGGL((k_query_d<H, kPrecFp8>), dim3(grid), dim3(256), lds, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_query_d(const QueryArgs& a, int H, int prec, uint32_t grid, hipStream_t st) {
  const size_t lds = (size_t)a.block_words * 4u;
  if (H == 32) return query_d_h<32>(a, prec, lds, grid, st);
  if (H == 64) return query_d_h<64>(a, prec, lds, grid, st);
  return hipErrorInvalidValue;
}

hipError_t launch_query_full(const QueryArgs& a, int H, uint32_t grid, hipStream_t st) {
  const size_t lds = (size_t)a.block_words * 4u;
  if (H == 32) hipLaunchKernelGGL(k_query_full<32>, dim3(grid), dim3(256), lds, st, a);
  else if (H == 64) hipLaunchKernelGGL(k_query_full<64>, dim3(grid), dim3(256), lds, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int H>
static hipError_t grid_d_h(const GridArgs& a, int prec, size_t lds, uint32_t grid, hipStream_t st) {
  if (prec == kPrecF32) hipLaunchKernelGGL((k_grid_d<H, kPrecF32>), dim3(grid), dim3(256), lds, st, a);
  else if (prec == kPrecBf16) hipLaunchKernelGGL((k_grid_d<H, kPrecBf16>), dim3(grid), dim3(256), lds, st, a);
  else if (prec == kPrecFp8) hipLaunchKernelGGL((k_grid_d<H, kPrecFp8>), dim3(grid), dim3(256), lds, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_grid_d(const GridArgs& a, int H, int prec, uint32_t grid, hipStream_t st) {
  if (a.R < 2 || a.K == 0) return hipErrorInvalidValue;
  const size_t lds = (size_t)a.block_words * 4u;
  if (H == 32) return grid_d_h<32>(a, prec, lds, grid, st);
  if (H == 64) return grid_d_h<64>(a, prec, lds, grid, st);
  return hipErrorInvalidValue;
}

hipError_t launch_grid_full(const GridArgs& a, int H, uint32_t grid, hipStream_t st) {
  if (a.R < 2 || a.K == 0) return hipErrorInvalidValue;
  const size_t lds = (size_t)a.block_words * 4u;
  if (H == 32) hipLaunchKernelGGL(k_grid_full<32>, dim3(grid), dim3(256), lds, st, a);
  else if (H == 64) hipLaunchKernelGGL(k_grid_full<64>, dim3(grid), dim3(256), lds, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_eik_points(const EikArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_eik_points, dim3((uint32_t)((6u * a.n + 255u) / 256u)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_eik_combine(const EikArgs& a, hipStream_t st) {
  const uint32_t nb = (uint32_t)((a.n + 255u) / 256u);
  hipLaunchKernelGGL(k_eik_combine, dim3(nb), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_eik_loss, dim3(1), dim3(256), 0, st, a, nb);
  return hipGetLastError();
}

hipError_t launch_world_raygen(const WorldRaygenArgs& a, uint32_t npath, hipStream_t st) {
  hipLaunchKernelGGL(k_world_raygen, dim3((npath + 255u) / 256u), dim3(256), 0, st, a, npath);
  return hipGetLastError();
}

hipError_t launch_world_step(const WorldStepArgs& a, uint32_t grid, hipStream_t st) {
  if (a.cs == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_world_step, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace kn
