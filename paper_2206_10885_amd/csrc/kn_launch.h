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
  float bg[3];
};

struct RaygenArgs {
  SceneGeom sg;
  float eye[3], fwd[3], right[3], up[3];
  float tx, ty;
  int W, Hh;
  RayStatic* rs;
  RayRec* U;
  uint32_t* counts;
  OutPtrs out;
};

struct ScanArgs {
  uint32_t* counts;      // per-cell counts (read; zeroed if zero_counts)
  uint32_t C, T;         // cells, chunk size (<= 1023)
  int zero_counts;
  uint32_t* cursor;      // out: bin start per cell (scatter cursor)
  uint2* chunks;         // out: (cell | count << 22, start)
  uint32_t* n_chunks;
  uint32_t* grab;        // out: per-range work cursors (kGroups x kGroupStride words)
  uint32_t* grab0;       // out: a copy of the initial cursors (to restart a pass)
  uint32_t* zero_word;   // optional counter reset to 0
  uint32_t* total;       // optional: receives the sum of the counts
};

struct ScatterArgs {
  const RayRec* in;      // records (keys 0xFFFFFFFF are skipped)
  RayRec* out;
  uint32_t n;
  uint32_t* cursor;
};

struct ScatterChunksArgs {
  SceneGeom sg;
  const uint2* chunks;        // previous round's chunks
  const uint4* chunk_out;     // their exit-face counts (2 x uint4 per chunk)
  const uint32_t* n_chunks;
  const RayRec* U;
  RayRec* S;
  uint32_t* cursor;
};

struct MarchArgs {
  SceneGeom sg;
  const float* blocks;
  uint32_t block_words;
  const RayRec* S;
  const RayStatic* rs;
  const uint2* chunks;
  const uint32_t* n_chunks;
  uint32_t* grab;        // per-range work cursors set by the scan
  uint4* chunk_out;          // per chunk: rays leaving through each face / staying, hits
  RayRec* U;                 // next-round rays, in each chunk's own range
  uint32_t* counts_next;
  RayRec* HL;                // hits, indexed by ray id
  uint32_t* hit_count;
  unsigned long long* evals;     // [0] evaluations, [1] tiles, [2] chunks
  int max_steps;
  int max_passes;            // in-cell passes per chunk before the rest wait a round
  float eps;
  SoftplusK spk;
  OutPtrs out;
};

struct ShadeArgs {
  SceneGeom sg;
  const float* blocks;
  uint32_t block_words;
  const RayRec* S;
  const RayStatic* rs;
  const uint2* chunks;
  const uint32_t* n_chunks;
  uint32_t* grab;        // per-range work cursors set by the scan
  SoftplusK spk;
  OutPtrs out;
};

struct QueryBinArgs {
  SceneGeom sg;
  const float* pts;
  uint64_t n;
  RayRec* U;
  uint32_t* counts;
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

hipError_t launch_raygen(const RaygenArgs& a, hipStream_t st);
hipError_t launch_scan(const ScanArgs& a, hipStream_t st);
hipError_t launch_scatter(const ScatterArgs& a, uint32_t grid, hipStream_t st);
hipError_t launch_scatter_chunks(const ScatterChunksArgs& a, uint32_t grid, hipStream_t st);
size_t march_lds_bytes(uint32_t block_words);
hipError_t launch_march(const MarchArgs& a, int H, int bf16, uint32_t grid, hipStream_t st);
hipError_t launch_shade(const ShadeArgs& a, int H, uint32_t grid, hipStream_t st);
hipError_t launch_query_bin(const QueryBinArgs& a, hipStream_t st);
hipError_t launch_query_d(const QueryArgs& a, int H, int bf16, uint32_t grid, hipStream_t st);
hipError_t launch_query_full(const QueryArgs& a, int H, uint32_t grid, hipStream_t st);

}  // namespace kn
