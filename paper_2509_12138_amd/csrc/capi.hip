// capi.hip — error reporting, status checks, argument validation, the
// graph-safe zero fill and the HIP-graph handles of libgsmi.
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "gs_device.h"

namespace gsmi {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = 0; }

int device_cu_count() {
  static std::mutex mu;
  static std::vector<int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (cache[dev] == 0) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cu <= 0)
      cu = 256;
    cache[dev] = cu;
  }
  return cache[dev];
}

gs_status check_views(const gs_views* v, const gs_tiling* t, const char* who) {
  GS_REQUIRE(v != nullptr && t != nullptr, "%s: views and tiling must not be NULL", who);
  GS_REQUIRE(v->n_slots >= 1 && v->n_slots <= GS_MAX_SLOTS, "%s: n_slots=%d outside [1, %d]", who,
             v->n_slots, GS_MAX_SLOTS);
  GS_REQUIRE(v->pair_offset && v->gauss_offset && v->cams,
             "%s: views arrays (pair_offset, gauss_offset, cams) must not be NULL", who);
  GS_REQUIRE(v->total_pairs >= 0 && v->total_pairs < (int64_t(1) << 32),
             "%s: total_pairs=%lld outside [0, 2^32)", who, (long long)v->total_pairs);
  GS_REQUIRE(t->width >= 1 && t->height >= 1 && t->width <= 16384 && t->height <= 16384,
             "%s: image %dx%d outside [1, 16384]^2", who, t->width, t->height);
  GS_REQUIRE(t->tile_w >= 1 && t->tile_h >= 1 && t->tile_w * t->tile_h <= 1024,
             "%s: tile %dx%d invalid", who, t->tile_w, t->tile_h);
  int64_t tiles = ceil_div(t->width, t->tile_w) * ceil_div(t->height, t->tile_h);
  GS_REQUIRE(tiles * v->n_slots < (int64_t(1) << 31), "%s: too many tiles", who);
  return GS_OK;
}

__global__ void k_zero(uint32_t* __restrict__ p, int64_t n_words) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n_words; i += stride) p[i] = 0u;
}

}  // namespace gsmi

// A captured and instantiated step: the graph and its executable form.
struct gs_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

using namespace gsmi;

extern "C" {

const char* gs_last_error(void) { return g_err; }

const char* gs_version(void) { return "gsmi 0.1 (gfx950)"; }

gs_status gs_zero(void* ptr, size_t bytes, void* stream) {
  clear_error();
  GS_REQUIRE(bytes % 4 == 0, "gs_zero: bytes=%zu is not a multiple of 4", bytes);
  if (bytes == 0) return GS_OK;
  GS_REQUIRE(ptr != nullptr, "gs_zero: NULL pointer");
  int64_t words = (int64_t)(bytes / 4);
  int64_t blocks = ceil_div(words, 256);
  int64_t cap = (int64_t)device_cu_count() * 16;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream),
                     (uint32_t*)ptr, words);
  GS_LAUNCH_CHECK("gs_zero");
  return GS_OK;
}

gs_status gs_check_status(const int64_t* status, void* stream, int64_t* required_out) {
  clear_error();
  GS_REQUIRE(status != nullptr, "gs_check_status: NULL status");
  int64_t host[GS_STATUS_WORDS];
  hipError_t e = hipMemcpyAsync(host, status, sizeof(host), hipMemcpyDeviceToHost,
                                as_stream(stream));
  if (e == hipSuccess) e = hipStreamSynchronize(as_stream(stream));
  if (e != hipSuccess) {
    set_error("gs_check_status: %s", hipGetErrorString(e));
    return GS_ERR_HIP;
  }
  if (required_out) *required_out = host[1];
  if (host[0] & GS_FLAG_CAPACITY) {
    set_error("duplicate list needs %lld entries (capacity exceeded)", (long long)host[1]);
    return GS_ERR_CAPACITY;
  }
  if (host[0] & GS_FLAG_NONFINITE) {
    set_error("non-finite loss");
    return GS_ERR_NONFINITE;
  }
  return GS_OK;
}

gs_status gs_graph_begin(void* stream) {
  clear_error();
  GS_REQUIRE(stream != nullptr,
             "gs_graph_begin: capture needs a created stream (not the null stream)");
  // thread-local mode: an unsafe call (e.g. a device allocation) made by this
  // thread during the capture fails and invalidates it
  hipError_t e = hipStreamBeginCapture(as_stream(stream), hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    set_error("gs_graph_begin: hipStreamBeginCapture: %s", hipGetErrorString(e));
    return GS_ERR_HIP;
  }
  return GS_OK;
}

gs_status gs_graph_end(void* stream, gs_graph** out) {
  clear_error();
  GS_REQUIRE(stream != nullptr && out != nullptr, "gs_graph_end: NULL argument");
  *out = nullptr;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(as_stream(stream), &graph);
  if (e != hipSuccess || graph == nullptr) {
    set_error("gs_graph_end: hipStreamEndCapture: %s (the capture was invalidated)",
              hipGetErrorString(e));
    if (graph) (void)hipGraphDestroy(graph);
    return GS_ERR_HIP;
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    set_error("gs_graph_end: hipGraphInstantiate: %s", hipGetErrorString(e));
    (void)hipGraphDestroy(graph);
    return GS_ERR_HIP;
  }
  gs_graph* g = new (std::nothrow) gs_graph{graph, exec};
  if (!g) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    set_error("gs_graph_end: out of host memory");
    return GS_ERR_HIP;
  }
  *out = g;
  return GS_OK;
}

gs_status gs_graph_launch(gs_graph* g, void* stream) {
  clear_error();
  GS_REQUIRE(g != nullptr, "gs_graph_launch: NULL graph");
  hipError_t e = hipGraphLaunch(g->exec, as_stream(stream));
  if (e != hipSuccess) {
    set_error("gs_graph_launch: %s", hipGetErrorString(e));
    return GS_ERR_HIP;
  }
  return GS_OK;
}

void gs_graph_destroy(gs_graph* g) {
  if (!g) return;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"
