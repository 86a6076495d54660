// Kernel argument blocks and launch wrappers (implemented in kn_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "kn_internal.h"

namespace kn {

struct OutPtrs {
  float* rgb;
  float* depth;
  float* normal;
  uint8_t* hit;
  uint16_t* steps;
  TraceRec* trace;
  SegRec* seg;             // path tracing: [paths][bounces + 1] or null
  float bg[3];
};

// One resident scene of a ray pool: its range of global cells and the
// packed weights the kernels stage.
struct SceneEnt {
  SceneGeom sg;            // sg.cell_base = first global cell
  uint32_t cell_end;       // cell_base + N^3
  uint32_t march_words, shade_words;
  const float* march;      // march blocks in the pool's precision
  const float* shade;      // float32 shading blocks
  SoftplusK spk;
  float wt[3], ws;         // instance placement in a world: x = wt + ws x_local (identity otherwise)
};

// A ray of a world render waiting for its next object (world coordinates).
struct WorldRec {
  float o[3];
  float tpm;               // primitives count from t > tpm
  float d[3];
  float tim;               // instance boxes entered at t >= tim
  uint32_t rid;
  uint32_t pad[3];
};
static_assert(sizeof(WorldRec) == 48, "world records are 48 bytes");

// Per pool ray of a world render: the world origin of its current segment
// and that segment's primitive bound, for its continuation past the box.
struct WState {
  float o[3];
  float tpm;
};

// A Lambertian primitive on the device (kn_primitive).
struct PrimDev {
  uint32_t kind;
  float p[9];
  float albedo[3];
};

// One request slot of a ray pool (a frame being rendered).
struct ReqEnt {
  OutPtrs out;
  float eps;
  uint32_t max_steps;
  uint32_t npix;
  uint32_t pt;             // 1: path tracing (paths = npix * spp; rgb resolved from them)
  uint32_t spp, bounces;
  uint32_t seed_lo, seed_hi;
  const float* env;        // [env_h][env_w][3] or null (black)
  uint32_t env_w, env_h;
  uint32_t unclamped;      // 1: Hart's unclamped steps (the next cell is the one containing the new point)
  uint32_t world;          // 1: a world render (misses past a box and scatters continue in the world)
  uint32_t sample_offset;  // path tracing: index of the call's first sample in each pixel's stream
};

// Tables shared by the kernels of a pool.
struct PoolTabs {
  const SceneEnt* scenes;  // sorted by cell_base, contiguous cell ranges
  const ReqEnt* reqs;      // indexed by slot (RayStatic::pix >> kPixBits)
  uint32_t n_scenes;
  uint32_t* miss_done;     // [kMaxSlots]
  uint32_t* hit_done;      // [kMaxSlots]
  PathRec* path;           // per pool ray, path tracing only
};

struct RaygenArgs {
  SceneGeom sg;            // the request's scene (global cell ids)
  float eye[3], fwd[3], right[3], up[3];
  float tx, ty;
  int W, Hh;
  uint32_t slot;           // request slot
  uint32_t rid_base;       // first pool ray id of the request
  RayStatic* rs;           // indexed by pool ray id
  RayRec* U;               // this request's records (one per pixel, in tile order)
  uint32_t* counts;        // arrivals per global cell for the next round (cell c at c * cs)
  uint32_t cs;             // words between the per-cell counters of a pool (>= 1)
  uint32_t* miss_done;     // per slot
  OutPtrs out;
};

// path tracing: one thread per path (pixel, sample)
struct RaygenPtArgs {
  SceneGeom sg;
  float eye[3], fwd[3], right[3], up[3];
  float tx, ty;
  int W, Hh;
  uint32_t spp, bounces;
  uint32_t seed_lo, seed_hi;
  const float* env;
  uint32_t env_w, env_h;
  uint32_t jitter;         // pixel jitter at spp = 1 too (progressive accumulation)
  uint32_t sample_offset;
  uint32_t slot;
  RayStatic* rs;
  RayRec* U;               // one record per path (index = pool ray id)
  PathRec* path;
  uint32_t* counts;        // cell c at c * cs
  uint32_t cs;
  uint32_t* miss_done;     // paths finished, per slot
  OutPtrs out;
};

struct ResolveArgs {
  const PathRec* path;
  uint32_t npix, spp;
  float* rgb;
  float* accum;          // progressive accumulation (or null)
  uint32_t sample_offset;
};

struct ScanArgs {
  uint32_t* counts;      // per-cell counts (read; zeroed if zero_counts)
  uint32_t C, T;         // cells, chunk size (a power of two, <= 512)
  int zero_counts;
  uint32_t* cursor;      // out: bin start per cell (scatter cursor)
  uint2* chunks;         // out: (cell | count << 22, start)
  uint32_t* n_chunks;
  uint32_t* grab;        // out: per-range work cursors (kGroups x kGroupStride words)
  uint32_t* grab0;       // out: a copy of the initial cursors (to restart a pass)
  uint32_t* zero_word;   // optional counter reset to 0
  uint32_t* zero_word2;  // a second one
  uint32_t* total;       // optional: the sum of the counts is added to it
  uint32_t* runs;        // optional: per-cell rays handed on by the previous round's chunks,
                         // binned first (read; zeroed if zero_counts)
  uint32_t* base;        // optional out: bin start per cell (cursor = base + runs)
  uint32_t* ticket;      // Ctrl::scan_ticket
  unsigned long long* flags;  // Ctrl::scan_flags
  uint32_t* err;         // Ctrl::scan_err
  uint32_t cs;           // counts, runs and cursor hold cell c at c * cs (base: at c)
  // optional: host-mapped ring that receives (tag << 32 | chunk count) in
  // slot tag % kRoundRing, stored at system scope, so the host can follow
  // the rounds without a copy command
  unsigned long long* host_ring;
  uint32_t ring_tag;
};

struct ScatterArgs {
  RayRec* in;            // records (keys 0xFFFFFFFF are skipped)
  RayRec* out;
  uint32_t n;            // number of records, or
  const uint32_t* n_dev; // if not null: the number of records, read on the device
  uint32_t* cursor;      // cell c at c * cs
  int clear_in;          // mark each record taken as invalid (hits indexed by ray id)
  uint32_t cs;
};

struct ScatterChunksArgs {
  PoolTabs tabs;
  const uint2* chunks;        // previous round's chunks
  const uint4* chunk_out;     // their exit-face counts and offsets (4 x uint4 per chunk)
  const uint32_t* n_chunks;
  const RayRec* U;
  RayRec* S;
  const uint32_t* base;       // bin start per cell
};

struct MarchArgs {
  PoolTabs tabs;
  const RayRec* S;
  const RayStatic* rs;
  const uint2* chunks;
  const uint32_t* n_chunks;
  uint32_t* grab;        // per-range work cursors set by the scan
  uint4* chunk_out;          // per chunk (4 x uint4): rays leaving through each face /
                             // staying, hits; then each run's offset in its next bin
  RayRec* U;                 // next-round rays, in each chunk's own range
  uint32_t* runs_next;       // per cell: rays this round's chunks hand on to it (cell c at c * cs)
  RayRec* hits;              // hits, indexed by pool ray id (invalid key: none)
  uint32_t* hit_count;       // hits per cell (cell c at c * cs)
  unsigned long long* evals;     // Ctrl::tally: [kTallyLines][16], per line evaluations, tiles, chunks
  int max_passes;            // in-cell passes per chunk before the rest wait a round
  uint32_t cs;               // words between per-cell counters
  // requests with unclamped steps: rays whose step leaves the cell go on in
  // the cell that contains the new point, appended here for the next round
  RayRec* jump;              // next round's jumped rays
  uint32_t* n_jump;          // their count
  uint32_t* counts_next;     // arrivals per cell for the next round (cell c at c * cs)
  // world renders: rays that leave an instance's box go on from here
  WorldRec* wlist;
  uint32_t* n_w;
  const WState* ws;
};

struct ShadeArgs {
  PoolTabs tabs;
  const RayRec* S;
  RayStatic* rs;         // path tracing: rewritten for the next segment
  const uint2* chunks;
  const uint32_t* n_chunks;
  uint32_t* grab;        // per-range work cursors set by the scan
  RayRec* spawn;         // path tracing: records of the next segments
  uint32_t* n_spawn;     // their count
  uint32_t* counts_next; // arrivals per cell for the next round (cell c at c * cs)
  uint32_t cs;
  WorldRec* wlist;       // world renders: scattered rays go on from here
  uint32_t* n_w;
};

// world renders: camera rays (one per path) into a world list
struct WorldRaygenArgs {
  float eye[3], fwd[3], right[3], up[3];
  float tx, ty;
  int W, Hh;
  uint32_t spp, jitter, sample_offset;
  uint32_t seed_lo, seed_hi;
  bool pt;
  PathRec* path;
  WorldRec* out;         // [paths], index = path id
};

// world renders: each record's next object; primitive hits are shaded (and
// scattered, path tracing) here, instance entries become march records
struct WorldStepArgs {
  PoolTabs tabs;         // instances = the pool's scene entries
  const PrimDev* prims;
  uint32_t n_prims;
  const WorldRec* in;
  uint32_t n;            // records, or
  const uint32_t* n_dev; // if not null: their count, read on the device
  RayStatic* rs;
  WState* ws;
  RayRec* spawn;         // march records of the next round
  uint32_t* n_spawn;
  uint32_t* counts_next;
  uint32_t cs;
};

struct QueryBinArgs {
  SceneGeom sg;
  const float* pts;
  uint64_t n;
  RayRec* U;
  uint32_t* counts;      // cell c at c * cs
  uint32_t cs;
};

struct QueryArgs {
  SceneGeom sg;
  const float* blocks;
  uint32_t block_words;
  const RayRec* S;
  const float* pts;
  const uint2* chunks;
  const uint32_t* n_chunks;
  uint32_t* grab;        // per-range work cursors set by the scan
  SoftplusK spk;
  float* d_out;
  float* grad_out;
  float* z_out;
};

// dense lattice sampling: R points per axis, K work items of 256 points per
// cell (K >= the largest cell's point count / 256)
struct GridArgs {
  SceneGeom sg;
  const float* blocks;
  uint32_t block_words;
  SoftplusK spk;
  uint32_t R, K;
  float rm1;             // R - 1
  float* d_out;          // [R^3], index i + R (j + R k)
  float* grad_out;       // [R^3][3] or null (k_grid_full only)
};

// finite-difference eikonal term over n points
struct EikArgs {
  const float* pts;      // [n][3]
  uint64_t n;
  float delta;
  float* stencil_pts;    // [6n][3]: x +- delta e_a, order +x, -x, +y, -y, +z, -z
  const float* stencil;  // [6n]: the SDF at the stencil points
  float* gnorm;          // [n]
  double* partial;       // [ceil(n / 256)]
  double* loss;          // [1] or null
};

hipError_t launch_raygen(const RaygenArgs& a, hipStream_t st);
hipError_t launch_raygen_pt(const RaygenPtArgs& a, hipStream_t st);
hipError_t launch_resolve(const ResolveArgs& a, hipStream_t st);
hipError_t launch_world_raygen(const WorldRaygenArgs& a, uint32_t npath, hipStream_t st);
hipError_t launch_world_step(const WorldStepArgs& a, uint32_t grid, hipStream_t st);
hipError_t launch_scan(const ScanArgs& a, hipStream_t st);
hipError_t launch_scatter(const ScatterArgs& a, uint32_t grid, hipStream_t st);
hipError_t launch_scatter_chunks(const ScatterChunksArgs& a, uint32_t grid, hipStream_t st);
size_t march_lds_bytes(uint32_t block_words);
// H = 32 or 64 selects a kernel specialised for scenes of that width; H = 0
// one that reads each scene's width from the table (mixed pools).
// block_words = the largest block among the pool's scenes.
size_t shade_lds_bytes(uint32_t block_words);
hipError_t launch_march(const MarchArgs& a, int H, int prec, uint32_t block_words, uint32_t grid,
                        hipStream_t st);
// prec: the pool's march precision; float32 pools shade with the float32
// block, bf16 and fp8 pools with the split-bfloat16 block
hipError_t launch_shade(const ShadeArgs& a, int H, int prec, bool pt, uint32_t block_words, uint32_t grid,
                        hipStream_t st);
hipError_t launch_query_bin(const QueryBinArgs& a, hipStream_t st);
// p[0..n) = v; dst[0..n) = src[0..n) (device words, kernels: no memset or
// memcpy node)
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st);
hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, size_t n, hipStream_t st);
hipError_t launch_query_d(const QueryArgs& a, int H, int prec, uint32_t grid, hipStream_t st);
hipError_t launch_query_full(const QueryArgs& a, int H, uint32_t grid, hipStream_t st);
hipError_t launch_grid_d(const GridArgs& a, int H, int prec, uint32_t grid, hipStream_t st);
hipError_t launch_grid_full(const GridArgs& a, int H, uint32_t grid, hipStream_t st);
hipError_t launch_eik_points(const EikArgs& a, hipStream_t st);
// gradient norms, per-workgroup partial sums, then the loss (one workgroup)
hipError_t launch_eik_combine(const EikArgs& a, hipStream_t st);

}  // namespace kn
