// HIP kernels of the KiloNeuS rendering hot path for gfx950 (MI355X).
//
// Wavefront design (one frame):
//   k_raygen   pinhole rays, box clip (Sec. 3.4.1), entry cell, box misses
//   per round: k_scan    per-cell exclusive scan -> bin starts, work chunks
//              k_scatter counting-sort of the round's rays by global cell
//              k_march   one workgroup per chunk of a cell's bin: the cell's
//                        SDF MLP weights are staged once in LDS then held in
//                        registers as MFMA fragments; 16-ray tiles step the
//                        sphere tracer while rays stay in the cell, empty
//                        tile slots are refilled from the chunk; rays that
//                        cross into a neighbour cell are compacted (wave
//                        ballot + one atomic per wave) into the next round
//   after the rounds: hits are binned by cell the same way, then k_shade
//              refines each hit with two Newton steps, takes the normalised
//              analytic gradient (forward-mode: value + 3 tangent columns per
//              hit in one MFMA tile) and runs the color MLP (Sec. 3.1 eq. 4).
#include "kn_device.h"
#include "kn_launch.h"

namespace kn {

// ---------------------------------------------------------------------------
// wave-aggregated atomics
// ---------------------------------------------------------------------------
__device__ __forceinline__ void atomic_count_grouped(uint32_t* arr, uint32_t key, bool valid) {
  uint64_t todo = __ballot(valid);
  while (todo) {
    int leader = __ffsll((unsigned long long)todo) - 1;
    uint32_t lk = __shfl(key, leader);
    uint64_t grp = __ballot(valid && key == lk);
    if (lane_id() == leader) atomicAdd(&arr[lk], (uint32_t)__popcll(grp));
    todo &= ~grp;
  }
}

__device__ __forceinline__ uint32_t atomic_slot_grouped(uint32_t* arr, uint32_t key, bool valid) {
  uint64_t todo = __ballot(valid);
  uint32_t pos = 0;
  while (todo) {
    int leader = __ffsll((unsigned long long)todo) - 1;
    uint32_t lk = __shfl(key, leader);
    bool mine = valid && key == lk;
    uint64_t grp = __ballot(mine);
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(&arr[lk], (uint32_t)__popcll(grp));
    base = __shfl(base, leader);
    if (mine) pos = base + (uint32_t)__popcll(grp & lanemask_lt());
    todo &= ~grp;
  }
  return pos;
}

// one atomic per wave on a list counter; returns this lane's slot (valid lanes)
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool valid) {
  uint64_t m = __ballot(valid);
  uint32_t base = 0;
  if (m) {
    if (lane_id() == __ffsll((unsigned long long)m) - 1) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, __ffsll((unsigned long long)m) - 1);
  }
  return base + (uint32_t)__popcll(m & lanemask_lt());
}

__device__ __forceinline__ void write_miss(const OutPtrs& o, uint32_t pix, int steps, float t,
                                           float t_entry, int32_t cell, int32_t status) {
  o.rgb[3 * pix + 0] = o.bg[0];
  o.rgb[3 * pix + 1] = o.bg[1];
  o.rgb[3 * pix + 2] = o.bg[2];
  if (o.depth) o.depth[pix] = 0.0f;
  if (o.normal) {
    o.normal[3 * pix + 0] = 0.0f;
    o.normal[3 * pix + 1] = 0.0f;
    o.normal[3 * pix + 2] = 0.0f;
  }
  if (o.hit) o.hit[pix] = 0;
  if (o.steps) o.steps[pix] = (uint16_t)steps;
  if (o.trace) o.trace[pix] = TraceRec{t, t_entry, cell, status};
}

// ---------------------------------------------------------------------------
// ray generation: one thread per pixel
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_raygen(RaygenArgs a) {
  const uint32_t npix = (uint32_t)a.W * (uint32_t)a.Hh;
  const uint32_t pix = blockIdx.x * 256u + threadIdx.x;
  const bool valid = pix < npix;
  const SceneGeom& sg = a.sg;
  uint32_t cell = 0;
  bool inbox = false;
  float t0 = 0.0f, tf = 0.0f;
  float d[3] = {0, 0, 0};
  if (valid) {
    const int row = (int)(pix / (uint32_t)a.W), col = (int)(pix % (uint32_t)a.W);
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
      a.rs[pix] = RayStatic{a.eye[0], a.eye[1], a.eye[2], tf, d[0], d[1], d[2], pix};
    } else {
      write_miss(a.out, pix, 0, 0.0f, 0.0f, -1, kBoxMiss);
    }
  }
  const uint32_t pos = wave_append(&a.ctrl->n_list[0], inbox);
  if (inbox) a.U[pos] = RayRec{t0, t0, cell, pix};
  atomic_count_grouped(a.counts, cell, inbox);
}

// ---------------------------------------------------------------------------
// per-round scan (one workgroup): bin starts, scatter cursors, work chunks
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_scan(ScanArgs a) {
  __shared__ uint32_t s_r[1024], s_k[1024];
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (a.C + 1023u) / 1024u;
  const uint32_t c0 = min(a.C, tid * per), c1 = min(a.C, c0 + per);
  uint32_t sr = 0, sk = 0;
  for (uint32_t c = c0; c < c1; ++c) {
    uint32_t n = a.counts[c];
    sr += n;
    sk += (n + a.T - 1u) / a.T;
  }
  s_r[tid] = sr;
  s_k[tid] = sk;
  __syncthreads();
  for (uint32_t off = 1; off < 1024u; off <<= 1) {
    uint32_t vr = tid >= off ? s_r[tid - off] : 0u;
    uint32_t vk = tid >= off ? s_k[tid - off] : 0u;
    __syncthreads();
    s_r[tid] += vr;
    s_k[tid] += vk;
    __syncthreads();
  }
  uint32_t R = s_r[tid] - sr, K = s_k[tid] - sk;
  for (uint32_t c = c0; c < c1; ++c) {
    uint32_t n = a.counts[c];
    a.cursor[c] = R;
    for (uint32_t i = 0; i < n; i += a.T) {
      uint32_t m = min(a.T, n - i);
      a.chunks[K++] = make_uint2(c | (m << kCellBits), R + i);
    }
    R += n;
    if (a.zero_counts) a.counts[c] = 0u;
  }
  if (tid == 1023u) {
    *a.n_chunks = s_k[1023];
    *a.chunk_next = 0u;
    if (a.zero_word) *a.zero_word = 0u;
  }
}

// ---------------------------------------------------------------------------
// counting-sort scatter of a record list by cell
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scatter(ScatterArgs a) {
  const uint32_t n = *a.n_in;
  for (uint32_t base = blockIdx.x * 256u; base < n; base += gridDim.x * 256u) {
    const uint32_t i = base + threadIdx.x;
    const bool valid = i < n;
    RayRec r = valid ? a.in[i] : RayRec{0, 0, 0, 0};
    const uint32_t cell = r.key & kCellMask;
    const uint32_t pos = atomic_slot_grouped(a.cursor, cell, valid);
    if (valid) a.out[pos] = r;
  }
}

// ---------------------------------------------------------------------------
// SDF MLP of one cell on a 16-point MFMA tile, weights in registers.
// Lane (g, p) supplies encoding slots j of point p and receives hidden units
// 16b + 4g + r of point p.  Returns the SDF value d for the lane's point
// (identical in the 4 lanes of the point).
// ---------------------------------------------------------------------------
template <int H, bool BF>
struct MarchW;

template <int H>
struct MarchW<H, false> {
  static constexpr int NB = H / 16, S1 = NB * kPeSlots, SF = S1 + NB * (H / 4);
  float fr[SF];
  float b1[NB][4], b2[NB][4], w3[NB][4];
  float b3;

  __device__ __forceinline__ void load(const float* blk, int lane, int g) {
    const f32x4* p = reinterpret_cast<const f32x4*>(blk);
#pragma unroll
    for (int s4 = 0; s4 < SF / 4; ++s4) {
      f32x4 v = p[s4 * 64 + lane];
      fr[4 * s4 + 0] = v[0];
      fr[4 * s4 + 1] = v[1];
      fr[4 * s4 + 2] = v[2];
      fr[4 * s4 + 3] = v[3];
    }
    const float* vec = blk + 64 * SF;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        b1[b][r] = vec[16 * b + 4 * g + r];
        b2[b][r] = vec[H + 16 * b + 4 * g + r];
        w3[b][r] = vec[2 * H + 16 * b + 4 * g + r];
      }
    }
    b3 = vec[3 * H];
  }

  __device__ __forceinline__ float eval(const float (&v)[kPeSlots], SoftplusK k) const {
    f32x4 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = f32x4{b1[b][0], b1[b][1], b1[b][2], b1[b][3]};
#pragma unroll
    for (int q = 0; q < kPeSlots; ++q) {
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = mfma_f32(fr[b * kPeSlots + q], v[q], acc[b]);
    }
    float a1[NB][4];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) a1[b][r] = softplus(acc[b][r], k);
    f32x4 acc2[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc2[b] = f32x4{b2[b][0], b2[b][1], b2[b][2], b2[b][3]};
#pragma unroll
    for (int q = 0; q < H / 4; ++q) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
        acc2[b] = mfma_f32(fr[S1 + b * (H / 4) + q], a1[q / 4][q % 4], acc2[b]);
    }
    float f = 0.0f;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) f = fmaf(w3[b][r], softplus(acc2[b][r], k), f);
    f += __shfl_xor(f, 16);
    f += __shfl_xor(f, 32);
    return f + b3;
  }
};

template <int H>
struct MarchW<H, true> {
  static constexpr int NB = H / 16, F1 = NB * 2, NF = F1 + NB * (H / 32);
  bf16x8 fr[NF];
  float b1[NB][4], b2[NB][4], w3[NB][4];
  float b3;

  __device__ __forceinline__ void load(const float* blk, int lane, int g) {
    const uint4* p = reinterpret_cast<const uint4*>(blk);
#pragma unroll
    for (int f = 0; f < NF; ++f) fr[f] = __builtin_bit_cast(bf16x8, p[f * 64 + lane]);
    const float* vec = blk + 64 * 4 * NF;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        b1[b][r] = vec[16 * b + 4 * g + r];
        b2[b][r] = vec[H + 16 * b + 4 * g + r];
        w3[b][r] = vec[2 * H + 16 * b + 4 * g + r];
      }
    }
    b3 = vec[3 * H];
  }

  __device__ __forceinline__ float eval(const float (&v)[kPeSlots], SoftplusK k) const {
    bf16x8 e0, e1;
#pragma unroll
    for (int i = 0; i < 8; ++i) e0[i] = (__bf16)v[i];
    e1[0] = (__bf16)v[8];
    e1[1] = (__bf16)v[9];
#pragma unroll
    for (int i = 2; i < 8; ++i) e1[i] = (__bf16)0.0f;
    f32x4 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = f32x4{b1[b][0], b1[b][1], b1[b][2], b1[b][3]};
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = mfma_bf16(fr[2 * b + 0], e0, acc[b]);
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = mfma_bf16(fr[2 * b + 1], e1, acc[b]);
    bf16x8 x[H / 32];
#pragma unroll
    for (int c = 0; c < H / 32; ++c)
#pragma unroll
      for (int i = 0; i < 8; ++i) x[c][i] = (__bf16)softplus(acc[2 * c + i / 4][i % 4], k);
    f32x4 acc2[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc2[b] = f32x4{b2[b][0], b2[b][1], b2[b][2], b2[b][3]};
#pragma unroll
    for (int c = 0; c < H / 32; ++c) {
#pragma unroll
      for (int b = 0; b < NB; ++b) acc2[b] = mfma_bf16(fr[F1 + b * (H / 32) + c], x[c], acc2[b]);
    }
    float f = 0.0f;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) f = fmaf(w3[b][r], bf16_round(softplus(acc2[b][r], k)), f);
    f += __shfl_xor(f, 16);
    f += __shfl_xor(f, 32);
    return f + b3;
  }
};

// copies one packed per-cell block (words % 4 == 0) into LDS
__device__ __forceinline__ void stage_block(float* lds, const float* src, uint32_t words) {
  const f32x4* s = reinterpret_cast<const f32x4*>(src);
  f32x4* d = reinterpret_cast<f32x4*>(lds);
  for (uint32_t i = threadIdx.x; i < words / 4u; i += blockDim.x) d[i] = s[i];
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
// (ties to the lowest axis).
__device__ __forceinline__ float cell_exit(const SceneGeom& sg, const CellBox& cb, const float o[3],
                                           const float d[3], int* axis) {
  const int idx[3] = {cb.ix, cb.iy, cb.iz};
  float best = INFINITY;
  int ba = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (d[k] != 0.0f) {
      float plane = sg.bmin[k] + (float)(idx[k] + (d[k] > 0.0f ? 1 : 0)) * sg.side[k];
      float tk = (plane - o[k]) / d[k];
      if (tk < best) {
        best = tk;
        ba = k;
      }
    }
  }
  *axis = ba;
  return best;
}

enum : int { kStay = 0, kOutHit = 1, kOutNext = 2, kOutExit = 3, kOutBudget = 4 };

// ---------------------------------------------------------------------------
// the march: one workgroup (4 waves) per chunk of a cell's bin
// ---------------------------------------------------------------------------
template <int H, bool BF>
__global__ __launch_bounds__(256) void k_march(MarchArgs a) {
  using W = MarchW<H, BF>;
  extern __shared__ float s_block[];
  __shared__ uint32_t s_job[4];
  __shared__ uint32_t s_cursor, s_nhit, s_evals;
  __shared__ uint32_t s_face[6];
  const int lane = lane_id(), g = lane >> 4, p = lane & 15;
  const bool rep = g == 0;  // lanes 0..15 write the results of their point
  const PeLane pl = make_pe_lane(g);
  const SceneGeom& sg = a.sg;
  const int N = sg.N;
  W w;
  uint32_t loaded = 0xFFFFFFFFu;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t j = atomicAdd(a.chunk_next, 1u);
      const uint32_t nch = *a.n_chunks;
      if (j < nch) {
        const uint2 c = a.chunks[j];
        s_job[0] = c.x & kCellMask;
        s_job[1] = c.y;
        s_job[2] = c.x >> kCellBits;
        s_job[3] = 1u;
      } else {
        s_job[3] = 0u;
      }
      s_cursor = 0u;
      s_nhit = 0u;
      s_evals = 0u;
      for (int f = 0; f < 6; ++f) s_face[f] = 0u;
    }
    __syncthreads();
    if (!s_job[3]) break;
    const uint32_t cell = s_job[0], start = s_job[1], count = s_job[2];
    const uint32_t lc = cell - sg.cell_base;
    if (cell != loaded) {
      stage_block(s_block, a.blocks + (size_t)lc * a.block_words, a.block_words);
      __syncthreads();
      w.load(s_block, lane, g);
      loaded = cell;
    }
    const CellBox cb = cell_box(sg, lc);

    // per-slot state
    bool have = false, exhausted = false;
    RayRec r = {0, 0, 0, 0};
    float o[3] = {0, 0, 0}, d[3] = {0, 0, 0}, t_far = 0.0f, ce = 0.0f;
    int eax = 0;
    uint32_t pix = 0, wave_evals = 0;
    for (;;) {
      const uint32_t empty = (uint32_t)(__ballot(!have) & 0xFFFFull);
      if (empty && !exhausted) {
        const uint32_t ne = (uint32_t)__popc(empty);
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&s_cursor, ne);
        base = __shfl(base, 0);
        if (base + ne >= count) exhausted = true;
        if (!have) {
          const uint32_t idx = base + (uint32_t)__popc(empty & ((1u << p) - 1u));
          if (idx < count) {
            r = a.S[start + idx];
            const RayStatic st = a.rs[r.rid];
            o[0] = st.ox; o[1] = st.oy; o[2] = st.oz;
            d[0] = st.dx; d[1] = st.dy; d[2] = st.dz;
            t_far = st.t_far;
            pix = st.pix;
            ce = cell_exit(sg, cb, o, d, &eax);
            have = true;
          }
        }
      }
      const uint64_t act = __ballot(have) & 0xFFFFull;
      if (!act) break;
      wave_evals += (uint32_t)__popcll(act);
      float xl[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) xl[k] = have ? fmaf(fmaf(r.t, d[k], o[k]), sg.inv_half[k], cb.cs[k]) : 0.0f;
      float v[kPeSlots];
      pe_values(pl, xl[0], xl[1], xl[2], v);
      const float f = w.eval(v, a.spk);

      int out = kStay;
      uint32_t next_cell = 0;
      int face = 0;
      if (have) {
        const uint32_t steps = (r.key >> kCellBits) + 1u;
        if (f < a.eps) {
          out = kOutHit;
        } else {
          const float te = fmaxf(r.t, ce);
          if (r.t + f < te) {
            r.t = r.t + f;
          } else {
            r.t = te;
            const int sgn = d[eax] > 0.0f ? 1 : -1;
            int nidx[3] = {cb.ix, cb.iy, cb.iz};
            nidx[eax] += sgn;
            face = 2 * eax + (sgn > 0 ? 1 : 0);
            if (nidx[eax] < 0 || nidx[eax] >= N || r.t > t_far) {
              out = kOutExit;
            } else {
              out = kOutNext;
              next_cell = sg.cell_base + (uint32_t)(nidx[0] + N * (nidx[1] + N * nidx[2]));
            }
          }
          if ((out == kStay || out == kOutNext) && steps >= (uint32_t)a.max_steps) out = kOutBudget;
        }
        r.key = (out == kOutNext ? next_cell : cell) | (steps << kCellBits);
        if (out == kOutNext) r.t_entry = r.t;
      }
      // next round
      {
        const bool e = rep && have && out == kOutNext;
        const uint32_t pos = wave_append(a.n_out, e);
        if (e) {
          a.U[pos] = r;
          atomicAdd(&s_face[face], 1u);
        }
      }
      // hits (binned by cell for shading)
      {
        const bool e = rep && have && out == kOutHit;
        const uint32_t pos = wave_append(a.n_hits, e);
        if (e) {
          a.hits[pos] = r;
          atomicAdd(&s_nhit, 1u);
        }
      }
      if (rep && have && (out == kOutExit || out == kOutBudget))
        write_miss(a.out, pix, (int)(r.key >> kCellBits), r.t, r.t_entry, (int32_t)cell,
                   out == kOutExit ? kExitMiss : kBudgetMiss);
      if (out != kStay) have = false;
    }
    if (lane == 0) atomicAdd(&s_evals, wave_evals);
    __syncthreads();
    if (threadIdx.x < 6) {
      const uint32_t n = s_face[threadIdx.x];
      if (n) {
        const int ax = threadIdx.x >> 1, sgn = (threadIdx.x & 1) ? 1 : -1;
        int nidx[3] = {cb.ix, cb.iy, cb.iz};
        nidx[ax] += sgn;
        atomicAdd(&a.counts_next[sg.cell_base + (uint32_t)(nidx[0] + N * (nidx[1] + N * nidx[2]))], n);
      }
    } else if (threadIdx.x == 6) {
      if (s_nhit) atomicAdd(&a.hit_count[cell], s_nhit);
      atomicAdd(a.evals, (unsigned long long)s_evals);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Full float32 SDF MLP on a tile of 4 points x 4 columns (value and the three
// world-axis tangents, forward mode): returns the output rows 4g..4g+3 of
// this lane's column.  Weights are read from the LDS block as MFMA fragments.
// ---------------------------------------------------------------------------
template <int H>
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
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float ds;
      const float sp = softplus_d(acc[b][r], k, &ds);
      const float dv = quad_bcast<0>(ds);
      a1[b][r] = value_col ? sp : dv * acc[b][r];
    }
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
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float ds;
      const float sp = softplus_d(acc2[b][r], k, &ds);
      const float dv = quad_bcast<0>(ds);
      a2[b][r] = value_col ? sp : dv * acc2[b][r];
    }
  f32x4 y = value_col ? *reinterpret_cast<const f32x4*>(vec + 2 * H + 4 * g) : f32x4{0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < H / 4; ++q) y = mfma_f32(blk[(S2 + q) * 64 + lane], a2[q / 4][q % 4], y);
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
template <int H>
__global__ __launch_bounds__(256) void k_shade(ShadeArgs a) {
  extern __shared__ float s_mem[];
  float* s_block = s_mem;
  float* s_stage = s_mem + a.block_words;  // 4 waves x 4 hits x 48
  __shared__ uint32_t s_job[4];
  const int lane = lane_id(), g = lane >> 4, col = lane & 15, h = col >> 2, s = col & 3;
  const int wave = threadIdx.x >> 6;
  const bool value_col = s == 0;
  const PeLane pl = make_pe_lane(g);
  const SceneGeom& sg = a.sg;
  const float* vec = nullptr;
  uint32_t loaded = 0xFFFFFFFFu;
  constexpr int NB = H / 16;
  constexpr int SC1 = NB * kPeSlots + NB * (H / 4) + H / 4;  // first color fragment slot
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t j = atomicAdd(a.chunk_next, 1u);
      const uint32_t nch = *a.n_chunks;
      if (j < nch) {
        const uint2 c = a.chunks[j];
        s_job[0] = c.x & kCellMask;
        s_job[1] = c.y;
        s_job[2] = c.x >> kCellBits;
        s_job[3] = 1u;
      } else {
        s_job[3] = 0u;
      }
    }
    __syncthreads();
    if (!s_job[3]) break;
    const uint32_t cell = s_job[0], start = s_job[1], count = s_job[2];
    const uint32_t lc = cell - sg.cell_base;
    if (cell != loaded) {
      stage_block(s_block, a.blocks + (size_t)lc * a.block_words, a.block_words);
      __syncthreads();
      loaded = cell;
    }
    vec = s_block + 64 * shade_frag_slots(H);
    const CellBox cb = cell_box(sg, lc);
    float* stage = s_stage + wave * 4 * kColIn;
    for (uint32_t base = (uint32_t)wave * 4u; base < count; base += 16u) {
      const uint32_t idx = base + (uint32_t)h;
      const bool valid = idx < count;
      RayRec r = valid ? a.S[start + idx] : RayRec{0, 0, cell, 0};
      const RayStatic st = valid ? a.rs[r.rid] : RayStatic{0, 0, 0, 0, 0, 0, 1, 0};
      const float o[3] = {st.ox, st.oy, st.oz}, d[3] = {st.dx, st.dy, st.dz};
      int eax;
      const float ce = cell_exit(sg, cb, o, d, &eax);
      float t = r.t;
      float xl[3], gr[3], fval = 0.0f;
      f32x4 y;
      for (int it = 0; it < 3; ++it) {
#pragma unroll
        for (int k = 0; k < 3; ++k) xl[k] = valid ? fmaf(fmaf(t, d[k], o[k]), sg.inv_half[k], cb.cs[k]) : 0.0f;
        float v[kPeSlots];
        pe_values_tangent(pl, s, s ? sg.inv_half[s - 1] : 0.0f, xl[0], xl[1], xl[2], v);
        y = sdf_full<H>(s_block, lane, g, value_col, v, a.spk);
        const int src = 4 * h;
        fval = __shfl(y[0], src);
        gr[0] = __shfl(y[0], src + 1);
        gr[1] = __shfl(y[0], src + 2);
        gr[2] = __shfl(y[0], src + 3);
        if (it < 2) {
          const float gd = gr[0] * d[0] + gr[1] * d[1] + gr[2] * d[2];
          if (gd < -1e-3f) t = fminf(fmaxf(t - fval / gd, r.t_entry), ce);
        }
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
        for (int b = 0; b < 2; ++b) c1[b] = mfma_f32(s_block[(SC1 + b * 12 + q) * 64 + lane], bq, c1[b]);
      }
      f32x4 c2 = g == 0 ? *reinterpret_cast<const f32x4*>(vc + 32) : f32x4{0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < 8; ++q)
        c2 = mfma_f32(s_block[(SC1 + 24 + q) * 64 + lane], fmaxf(c1[q / 4][q % 4], 0.0f), c2);
      if (valid && g == 0 && value_col) {
        const uint32_t px = st.pix;
        a.out.rgb[3 * px + 0] = sigmoid(c2[0]);
        a.out.rgb[3 * px + 1] = sigmoid(c2[1]);
        a.out.rgb[3 * px + 2] = sigmoid(c2[2]);
        if (a.out.depth) a.out.depth[px] = t;
        if (a.out.normal) {
          a.out.normal[3 * px + 0] = n[0];
          a.out.normal[3 * px + 1] = n[1];
          a.out.normal[3 * px + 2] = n[2];
        }
        if (a.out.hit) a.out.hit[px] = 1;
        if (a.out.steps) a.out.steps[px] = (uint16_t)(r.key >> kCellBits);
        if (a.out.trace) a.out.trace[px] = TraceRec{r.t, r.t_entry, (int32_t)cell, kHit};
      }
    }
    __syncthreads();
  }
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
  atomic_count_grouped(a.counts, cell, valid);
}

template <int H, bool BF>
__global__ __launch_bounds__(256) void k_query_d(QueryArgs a) {
  using W = MarchW<H, BF>;
  extern __shared__ float s_block[];
  __shared__ uint32_t s_job[4];
  const int lane = lane_id(), g = lane >> 4, p = lane & 15, wave = threadIdx.x >> 6;
  const PeLane pl = make_pe_lane(g);
  const SceneGeom& sg = a.sg;
  W w;
  uint32_t loaded = 0xFFFFFFFFu;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t j = atomicAdd(a.chunk_next, 1u);
      if (j < *a.n_chunks) {
        const uint2 c = a.chunks[j];
        s_job[0] = c.x & kCellMask;
        s_job[1] = c.y;
        s_job[2] = c.x >> kCellBits;
        s_job[3] = 1u;
      } else {
        s_job[3] = 0u;
      }
    }
    __syncthreads();
    if (!s_job[3]) break;
    const uint32_t cell = s_job[0], start = s_job[1], count = s_job[2];
    const uint32_t lc = cell - sg.cell_base;
    if (cell != loaded) {
      stage_block(s_block, a.blocks + (size_t)lc * a.block_words, a.block_words);
      __syncthreads();
      w.load(s_block, lane, g);
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
      pe_values(pl, xl[0], xl[1], xl[2], v);
      const float f = w.eval(v, a.spk);
      if (valid && g == 0) a.d_out[pi] = f;
    }
    __syncthreads();
  }
}

template <int H>
__global__ __launch_bounds__(256) void k_query_full(QueryArgs a) {
  extern __shared__ float s_block[];
  __shared__ uint32_t s_job[4];
  const int lane = lane_id(), g = lane >> 4, col = lane & 15, h = col >> 2, s = col & 3;
  const int wave = threadIdx.x >> 6;
  const PeLane pl = make_pe_lane(g);
  const SceneGeom& sg = a.sg;
  uint32_t loaded = 0xFFFFFFFFu;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t j = atomicAdd(a.chunk_next, 1u);
      if (j < *a.n_chunks) {
        const uint2 c = a.chunks[j];
        s_job[0] = c.x & kCellMask;
        s_job[1] = c.y;
        s_job[2] = c.x >> kCellBits;
        s_job[3] = 1u;
      } else {
        s_job[3] = 0u;
      }
    }
    __syncthreads();
    if (!s_job[3]) break;
    const uint32_t cell = s_job[0], start = s_job[1], count = s_job[2];
    const uint32_t lc = cell - sg.cell_base;
    if (cell != loaded) {
      stage_block(s_block, a.blocks + (size_t)lc * a.block_words, a.block_words);
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
// launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_raygen(const RaygenArgs& a, hipStream_t st) {
  const uint32_t npix = (uint32_t)a.W * (uint32_t)a.Hh;
  hipLaunchKernelGGL(k_raygen, dim3((npix + 255u) / 256u), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_scan(const ScanArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_scatter(const ScatterArgs& a, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int H, bool BF>
static hipError_t march_t(const MarchArgs& a, uint32_t grid, hipStream_t st) {
  const size_t lds = (size_t)a.block_words * 4u;
  hipLaunchKernelGGL((k_march<H, BF>), dim3(grid), dim3(256), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_march(const MarchArgs& a, int H, int bf16, uint32_t grid, hipStream_t st) {
  if (H == 32) return bf16 ? march_t<32, true>(a, grid, st) : march_t<32, false>(a, grid, st);
  if (H == 64) return bf16 ? march_t<64, true>(a, grid, st) : march_t<64, false>(a, grid, st);
  return hipErrorInvalidValue;
}

hipError_t launch_shade(const ShadeArgs& a, int H, uint32_t grid, hipStream_t st) {
  const size_t lds = ((size_t)a.block_words + 4u * 4u * kColIn) * 4u;
  if (H == 32) hipLaunchKernelGGL(k_shade<32>, dim3(grid), dim3(256), lds, st, a);
  else if (H == 64) hipLaunchKernelGGL(k_shade<64>, dim3(grid), dim3(256), lds, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_query_bin(const QueryBinArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_query_bin, dim3((uint32_t)((a.n + 255u) / 256u)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_query_d(const QueryArgs& a, int H, int bf16, uint32_t grid, hipStream_t st) {
  const size_t lds = (size_t)a.block_words * 4u;
  if (H == 32) {
    if (bf16) hipLaunchKernelGGL((k_query_d<32, true>), dim3(grid), dim3(256), lds, st, a);
    else hipLaunchKernelGGL((k_query_d<32, false>), dim3(grid), dim3(256), lds, st, a);
  } else if (H == 64) {
    if (bf16) hipLaunchKernelGGL((k_query_d<64, true>), dim3(grid), dim3(256), lds, st, a);
    else hipLaunchKernelGGL((k_query_d<64, false>), dim3(grid), dim3(256), lds, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_query_full(const QueryArgs& a, int H, uint32_t grid, hipStream_t st) {
  const size_t lds = (size_t)a.block_words * 4u;
  if (H == 32) hipLaunchKernelGGL(k_query_full<32>, dim3(grid), dim3(256), lds, st, a);
  else if (H == 64) hipLaunchKernelGGL(k_query_full<64>, dim3(grid), dim3(256), lds, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace kn
