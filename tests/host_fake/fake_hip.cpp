// Definitions of the host-only HIP stand-in (hip/hip_runtime.h in this
// directory) and stubs of the kernel launchers of kn_kernels.hip, so that the
// host runtime links and runs under the sanitizers without a GPU.
//  - Device allocations are host allocations, filled with 0xA5 so that code
//    relying on fresh memory being zero shows up; the fake keeps a table of
//    live allocations and every launcher checks that the buffers it is given
//    lie inside one (a stale pointer into a freed pool aborts the run).
//  - Streams and events are synchronous.
//  - Ray generation marks every ray of its request finished as a miss, so
//    frames and serving requests complete; the cell scan sets the look-back
//    overrun flag when KN_FAKE_SCAN_ERR is set in the environment.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "kn_launch.h"

struct FakeStream { int id; };
struct FakeEvent { int id; };

namespace {
std::mutex g_mu;
std::map<const char*, size_t> g_live;   // device allocation -> size

void track(void* p, size_t n) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_live[static_cast<const char*>(p)] = n;
}

bool untrack(void* p) {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_live.erase(static_cast<const char*>(p)) == 1;
}

// [p, p + bytes) inside one live device allocation
void need(const void* p, size_t bytes, const char* what) {
  if (!p) {
    std::fprintf(stderr, "fake hip: %s is NULL\n", what);
    std::abort();
  }
  std::lock_guard<std::mutex> lk(g_mu);
  const char* c = static_cast<const char*>(p);
  auto it = g_live.upper_bound(c);
  if (it == g_live.begin()) {
    std::fprintf(stderr, "fake hip: %s (%p) is not device memory\n", what, p);
    std::abort();
  }
  --it;
  if (c + bytes > it->first + it->second) {
    std::fprintf(stderr, "fake hip: %s (%p, %zu bytes) outside its allocation\n", what, p, bytes);
    std::abort();
  }
}
}  // namespace

hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipSetDevice(int dev) { return dev == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  std::memset(p, 0, sizeof *p);
  std::strcpy(p->name, "host fake");
  p->multiProcessorCount = 256;
  return hipSuccess;
}
hipError_t hipMemGetInfo(size_t* f, size_t* t) {
  *f = (size_t)8 << 30;
  *t = (size_t)8 << 30;
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "fake hip error"; }

hipError_t hipMalloc(void** p, size_t bytes) {
  *p = std::malloc(bytes ? bytes : 1);
  if (!*p) return hipErrorOutOfMemory;
  std::memset(*p, 0xA5, bytes);
  track(*p, bytes);
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  if (!untrack(p)) {
    std::fprintf(stderr, "fake hip: hipFree of %p, not a live allocation\n", p);
    std::abort();
  }
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) {
  *p = std::malloc(bytes ? bytes : 1);
  if (!*p) return hipErrorOutOfMemory;
  std::memset(*p, 0xA5, bytes);
  return hipSuccess;
}
hipError_t hipHostFree(void* p) {
  (void)untrack(p);   // mapped host memory is registered as device memory
  std::free(p);
  return hipSuccess;
}
// mapped host memory: the device address is the host address; registered as
// device memory so that kernel stubs may be handed it
hipError_t hipHostGetDevicePointer(void** dev, void* host, unsigned) {
  *dev = host;
  std::lock_guard<std::mutex> lk(g_mu);
  g_live.emplace(static_cast<const char*>(host), (size_t)kn::kRoundRing * 8);
  return hipSuccess;
}
hipError_t hipStreamQuery(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  if (kind == hipMemcpyHostToDevice || kind == hipMemcpyDeviceToDevice) need(dst, bytes, "copy destination");
  if (kind == hipMemcpyDeviceToHost || kind == hipMemcpyDeviceToDevice) need(src, bytes, "copy source");
  std::memmove(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t) {
  return hipMemcpy(dst, src, bytes, kind);
}
hipError_t hipMemset(void* dst, int v, size_t bytes) {
  need(dst, bytes, "memset destination");
  std::memset(dst, v, bytes);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t) { return hipMemset(dst, v, bytes); }
hipError_t hipStreamCreateWithFlags(hipStream_t* st, unsigned) { *st = new FakeStream{1}; return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t st) { delete st; return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = new FakeEvent{1}; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.0f; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
// A device symbol is a host array here.  It is registered as device memory
// of 16 MB (its size is not known here; the library's scratch is smaller):
// the address sanitizer checks the array's real bounds.
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  std::lock_guard<std::mutex> lk(g_mu);
  g_live.emplace(static_cast<const char*>(symbol), (size_t)16 << 20);
  return hipSuccess;
}

namespace kn {

static void need_tabs(const PoolTabs& t) {
  need(t.scenes, t.n_scenes * sizeof(SceneEnt), "scene table");
  need(t.reqs, kMaxSlots * sizeof(ReqEnt), "request table");
  need(t.miss_done, kMaxSlots * 4, "miss_done");
  need(t.hit_done, kMaxSlots * 4, "hit_done");
}

static void finish_as_misses(uint32_t* miss_done, uint32_t slot, uint32_t n) {
  need(miss_done + slot, 4, "miss_done");
  __atomic_fetch_add(miss_done + slot, n, __ATOMIC_SEQ_CST);
}

hipError_t launch_raygen(const RaygenArgs& a, hipStream_t) {
  const size_t n = (size_t)a.W * a.Hh;
  need(a.rs + a.rid_base, n * sizeof(RayStatic), "ray statics");
  need(a.U, n * sizeof(RayRec), "new ray records");
  finish_as_misses(a.miss_done, a.slot, (uint32_t)n);
  return hipSuccess;
}
hipError_t launch_raygen_pt(const RaygenPtArgs& a, hipStream_t) {
  const size_t n = (size_t)a.W * a.Hh * a.spp;
  need(a.rs, n * sizeof(RayStatic), "ray statics");
  need(a.U, n * sizeof(RayRec), "new ray records");
  need(a.path, n * sizeof(PathRec), "path records");
  finish_as_misses(a.miss_done, a.slot, (uint32_t)n);
  return hipSuccess;
}
hipError_t launch_resolve(const ResolveArgs& a, hipStream_t) {
  need(a.path, (size_t)a.npix * a.spp * sizeof(PathRec), "path records");
  return hipSuccess;
}
hipError_t launch_world_raygen(const WorldRaygenArgs& a, uint32_t npath, hipStream_t) {
  need(a.out, (size_t)npath * sizeof(WorldRec), "world records");
  if (a.pt) need(a.path, (size_t)npath * sizeof(PathRec), "path records");
  return hipSuccess;
}
// every record ends (escapes) here: nothing is spawned
hipError_t launch_world_step(const WorldStepArgs& a, uint32_t, hipStream_t) {
  need_tabs(a.tabs);
  need(a.prims, sizeof(PrimDev), "primitives");
  uint32_t n = a.n;
  if (a.n_dev) {
    need(a.n_dev, 4, "world record count");
    n = *a.n_dev;
  }
  if (n) need(a.in, (size_t)n * sizeof(WorldRec), "world records");
  need(a.n_spawn, 4, "spawn count");
  need(a.spawn, 16, "spawn list");
  need(a.counts_next, 4, "next round's counts");
  finish_as_misses(a.tabs.miss_done, 0, n);
  return hipSuccess;
}
hipError_t launch_scan(const ScanArgs& a, hipStream_t) {
  need(a.counts, (size_t)a.C * a.cs * 4, "scan counts");
  need(a.cursor, (size_t)a.C * a.cs * 4, "scan cursor");
  need(a.n_chunks, 4, "n_chunks");
  need(a.grab, kGroups * kGroupStride * 4, "work cursors");
  need(a.err, 4, "scan_err");
  *a.n_chunks = 0u;
  if (a.host_ring) {
    // the chunk count the host sees: 0, or with KN_FAKE_ROUND_CHUNKS set, a
    // count that falls from 2000 by 250 per round (so that a large frame
    // takes its early-shading branch)
    need(a.host_ring, kRoundRing * 8, "round ring");
    const uint32_t r = a.ring_tag & 2047u;
    const uint32_t n = std::getenv("KN_FAKE_ROUND_CHUNKS") && r < 8u ? 2000u - 250u * r : 0u;
    a.host_ring[a.ring_tag % kRoundRing] = ((unsigned long long)a.ring_tag << 32) | n;
  }
  if (std::getenv("KN_FAKE_SCAN_ERR")) *a.err |= 1u;
  return hipSuccess;
}
hipError_t launch_scatter(const ScatterArgs& a, uint32_t, hipStream_t) {
  need(a.out, 16, "scatter destination");
  return hipSuccess;
}
hipError_t launch_scatter_chunks(const ScatterChunksArgs& a, uint32_t, hipStream_t) {
  need_tabs(a.tabs);
  need(a.S, 16, "sorted records");
  return hipSuccess;
}
hipError_t launch_march(const MarchArgs& a, int, int, uint32_t, uint32_t, hipStream_t) {
  need_tabs(a.tabs);
  need(a.S, 16, "sorted records");
  need(a.hits, 16, "hit list");
  return hipSuccess;
}
hipError_t launch_shade(const ShadeArgs& a, int, int, bool, uint32_t, uint32_t, hipStream_t) {
  need_tabs(a.tabs);
  need(a.S, 16, "sorted records");
  return hipSuccess;
}
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t) {
  need(p, n * 4, "fill destination");
  for (size_t i = 0; i < n; ++i) p[i] = v;
  return hipSuccess;
}
hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, size_t n, hipStream_t) {
  need(dst, n * 4, "copy destination");
  need(src, n * 4, "copy source");
  std::memmove(dst, src, n * 4);
  return hipSuccess;
}
hipError_t launch_query_bin(const QueryBinArgs& a, hipStream_t) {
  need(a.U, a.n * sizeof(RayRec), "query records");
  return hipSuccess;
}
hipError_t launch_query_d(const QueryArgs& a, int, int, uint32_t, hipStream_t) {
  need(a.blocks, 4, "weight blocks");
  return hipSuccess;
}
hipError_t launch_query_full(const QueryArgs& a, int, uint32_t, hipStream_t) {
  need(a.blocks, 4, "weight blocks");
  return hipSuccess;
}

hipError_t launch_grid_d(const GridArgs& a, int, int, uint32_t, hipStream_t) {
  need(a.blocks, 4, "weight blocks");
  need(a.d_out, (size_t)a.R * a.R * a.R * 4, "lattice values");
  return hipSuccess;
}
hipError_t launch_grid_full(const GridArgs& a, int, uint32_t, hipStream_t) {
  need(a.blocks, 4, "weight blocks");
  need(a.d_out, (size_t)a.R * a.R * a.R * 4, "lattice values");
  if (a.grad_out) need(a.grad_out, (size_t)a.R * a.R * a.R * 12, "lattice gradients");
  return hipSuccess;
}
hipError_t launch_eik_points(const EikArgs& a, hipStream_t) {
  need(a.pts, a.n * 12, "eikonal points");
  need(a.stencil_pts, a.n * 72, "stencil points");
  return hipSuccess;
}
hipError_t launch_eik_combine(const EikArgs& a, hipStream_t) {
  need(a.stencil, a.n * 24, "stencil values");
  need(a.gnorm, a.n * 4, "gradient norms");
  need(a.partial, (a.n + 255) / 256 * 8, "partial sums");
  if (a.loss) need(a.loss, 8, "loss");
  return hipSuccess;
}

}  // namespace kn
