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
  Ctrl* ctrl;
  OutPtrs out;
};

struct ScanArgs {
  uint32_t* counts;      // per-cell counts (read; zeroed if zero_counts)
  uint32_t C, T;         // cells, chunk size (<= 1023)
  int zero_counts;
  uint32_t* cursor;      // out: bin start per cell (scatter cursor)
  uint2* chunks;         // out: (cell | count << 22, start)
  uint32_t* n_chunks;
  uint32_t* chunk_next;  // reset to 0
  uint32_t* zero_word;   // optional counter reset to 0
};

struct ScatterArgs {
  const RayRec* in;
  RayRec* out;
  const uint32_t* n_in;
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
  uint32_t* chunk_next;
  RayRec* U;
  uint32_t* n_out;
  uint32_t* counts_next;
  RayRec* hits;
  uint32_t* n_hits;
  uint32_t* hit_count;
  unsigned long long* evals;
  int max_steps;
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
  uint32_t* chunk_next;
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
  uint32_t* chunk_next;
  SoftplusK spk;
  float* d_out;
  float* grad_out;
  float* z_out;
};

hipError_t launch_raygen(const RaygenArgs& a, hipStream_t st);
hipError_t launch_scan(const ScanArgs& a, hipStream_t st);
hipError_t launch_scatter(const ScatterArgs& a, uint32_t grid, hipStream_t st);
hipError_t launch_march(const MarchArgs& a, int H, int bf16, uint32_t grid, hipStream_t st);
hipError_t launch_shade(const ShadeArgs& a, int H, uint32_t grid, hipStream_t st);
hipError_t launch_query_bin(const QueryBinArgs& a, hipStream_t st);
hipError_t launch_query_d(const QueryArgs& a, int H, int bf16, uint32_t grid, hipStream_t st);
hipError_t launch_query_full(const QueryArgs& a, int H, uint32_t grid, hipStream_t st);

}  // namespace kn
