// schedule.hip — the rasterisers' work schedule from the sorted tile lists:
// the longest-first (LPT) order of the tiles and the chunk work items of the
// chunked backward and the split forward (offsets and item list).  These
// decide only which work-group does which tile or list chunk, never a value
// the method computes.
#include "gs_device.h"

namespace gsmi {

constexpr int kScheduleWave = 64;   // chunk lengths are multiples of the wave

// ---------------------------------------------------------------- tile order

// Longest-first (LPT) order of the tiles by list length, bucketed by
// floor(log2(len + 1)): 32 buckets, block-local LDS counts, one global
// atomic per (block, bucket), so tiles of one block stay together inside a
// bucket.
constexpr int kOrderThreads = 256;
constexpr int kOrderBuckets = 32;

__device__ __forceinline__ int len_bucket(uint32_t len) {
  return 31 - __clz(len + 1u);    // 0 for empty tiles
}

__global__ __launch_bounds__(kOrderThreads) void k_order_count(const uint32_t* __restrict__ ranges,
                                                               int64_t n_tiles,
                                                               uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kOrderBuckets];
  if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kOrderThreads + threadIdx.x;
  if (t < n_tiles) atomicAdd(&h[len_bucket(ranges[2 * t + 1] - ranges[2 * t])], 1u);
  __syncthreads();
  if (threadIdx.x < kOrderBuckets && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_order_scan(uint32_t* __restrict__ hist, uint32_t* __restrict__ start) {
  if (threadIdx.x != 0) return;
  uint32_t run = 0;
  for (int b = kOrderBuckets - 1; b >= 0; --b) {   // descending cost
    start[b] = run;
    run += hist[b];
  }
}

__global__ __launch_bounds__(kOrderThreads) void k_order_scatter(const uint32_t* __restrict__ ranges,
                                                                 int64_t n_tiles,
                                                                 const uint32_t* __restrict__ start,
                                                                 uint32_t* __restrict__ cursor,
                                                                 uint32_t* __restrict__ order) {
  __shared__ uint32_t h[kOrderBuckets], base[kOrderBuckets];
  if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kOrderThreads + threadIdx.x;
  int b = 0;
  uint32_t local = 0;
  if (t < n_tiles) {
    b = len_bucket(ranges[2 * t + 1] - ranges[2 * t]);
    local = atomicAdd(&h[b], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kOrderBuckets && h[threadIdx.x])
    base[threadIdx.x] = start[threadIdx.x] + atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]);
  __syncthreads();
  if (t < n_tiles) order[base[b] + local] = (uint32_t)t;
}

// The same order from one work-group, for up to kOrderOneMax tiles: bucket
// counts in LDS, the descending-cost starts, then every tile's slot from an
// LDS cursor per bucket (no workspace, one launch).
constexpr int kOrderOneThreads = 1024;
constexpr int64_t kOrderOneMax = 65536;

__global__ __launch_bounds__(kOrderOneThreads) void k_order_one(const uint32_t* __restrict__ ranges,
                                                                int n_tiles,
                                                                uint32_t* __restrict__ order) {
  __shared__ uint32_t h[kOrderBuckets], cur[kOrderBuckets];
  if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < n_tiles; t += kOrderOneThreads)
    atomicAdd(&h[len_bucket(ranges[2 * t + 1] - ranges[2 * t])], 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int b = kOrderBuckets - 1; b >= 0; --b) {   // descending cost
      cur[b] = run;
      run += h[b];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n_tiles; t += kOrderOneThreads)
    order[atomicAdd(&cur[len_bucket(ranges[2 * t + 1] - ranges[2 * t])], 1u)] = (uint32_t)t;
}

// ---------------------------------------------------------------- chunk items

// offset[t] = exclusive scan of ceil(len(t) / chunk) over n_tiles + 1
// entries, from one work-group: the counts are staged in LDS with coalesced
// reads of the ranges (one padding slot after every 32), thread j scans its
// contiguous segment there, and the offsets leave with coalesced writes;
// then a grid of threads, one per tile, writes items[offset[t] + c] = t
// (items past max_items are dropped).  The fill stays a grid: from one
// work-group, one CU's memory pipeline would issue every scattered item store.
constexpr int kChunkThreads = 1024;
constexpr int64_t kChunkScanOne = 16384;   // tiles the one-work-group scan takes

__global__ __launch_bounds__(kChunkThreads) void k_chunk_scan(const uint32_t* __restrict__ ranges,
                                                              int64_t n_tiles, int chunk,
                                                              uint32_t* __restrict__ offset) {
  __shared__ uint32_t cnt[kChunkScanOne + kChunkScanOne / 32];
  __shared__ uint32_t part[kChunkThreads];
  auto at = [](int i) { return i + (i >> 5); };
  const int j = threadIdx.x;
  uint32_t carry = 0;
  // segments of kChunkScanOne tiles (one for the tile counts this kernel is
  // launched for), the running total carried
  for (int64_t s0 = 0; s0 < n_tiles; s0 += kChunkScanOne) {
    const int n = (int)min(kChunkScanOne, n_tiles - s0);
    const uint32_t* rg = ranges + 2 * s0;
    // 8 loads per thread in flight at a time (a plain loop waits for each)
    for (int t0 = j; t0 < n; t0 += kChunkThreads * 8) {
      uint2 rr[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int t = t0 + q * kChunkThreads;
        rr[q] = t < n ? reinterpret_cast<const uint2*>(rg)[t] : make_uint2(0u, 0u);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int t = t0 + q * kChunkThreads;
        if (t < n) cnt[at(t)] = (rr[q].y - rr[q].x + chunk - 1) / chunk;
      }
    }
    __syncthreads();
    const int per = (n + kChunkThreads - 1) / kChunkThreads;
    const int b0 = min(j * per, n), b1 = min(b0 + per, n);
    uint32_t sum = 0;
    for (int t = b0; t < b1; ++t) sum += cnt[at(t)];
    part[j] = sum;
    __syncthreads();
    for (int d = 1; d < kChunkThreads; d <<= 1) {
      const uint32_t x = j >= d ? part[j - d] : 0u;
      __syncthreads();
      part[j] += x;
      __syncthreads();
    }
    uint32_t run = carry + (j > 0 ? part[j - 1] : 0u);
    for (int t = b0; t < b1; ++t) {
      const uint32_t c = cnt[at(t)];
      cnt[at(t)] = run;
      run += c;
    }
    __syncthreads();
    for (int t = j; t < n; t += kChunkThreads) offset[s0 + t] = cnt[at(t)];
    carry += part[kChunkThreads - 1];
    __syncthreads();                      // LDS reused by the next segment
  }
  if (j == 0) offset[n_tiles] = carry;
}

// Above kChunkScanOne tiles the single work-group's sequential segments
// cost more than three grid launches (0.25 ms at 129,600 tiles): block b
// sums the counts of its kChunkBlock tiles, one work-group scans the block
// sums in place, then block b scans its tiles from its base.  Same offsets.
constexpr int kChunkPer = 4;                               // tiles per thread
constexpr int kChunkBlock = 256 * kChunkPer;

__device__ __forceinline__ uint32_t chunk_count(const uint32_t* __restrict__ ranges, int64_t t,
                                                int chunk) {
  return (ranges[2 * t + 1] - ranges[2 * t] + chunk - 1) / chunk;
}

__global__ __launch_bounds__(256) void k_chunk_bsum(const uint32_t* __restrict__ ranges,
                                                    int64_t n_tiles, int chunk,
                                                    uint32_t* __restrict__ bsum) {
  __shared__ uint32_t red[256];
  const int64_t base = (int64_t)blockIdx.x * kChunkBlock;
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kChunkPer; ++k) {
    const int64_t t = base + k * 256 + threadIdx.x;
    if (t < n_tiles) sum += chunk_count(ranges, t, chunk);
  }
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// Exclusive scan of n values in place, one work-group (thread j owns a
// contiguous segment).
__global__ __launch_bounds__(kChunkThreads) void k_chunk_bscan(uint32_t* __restrict__ v,
                                                               int64_t n) {
  __shared__ uint32_t part[kChunkThreads];
  const int j = threadIdx.x;
  const int64_t per = (n + kChunkThreads - 1) / kChunkThreads;
  const int64_t b0 = min((int64_t)j * per, n), b1 = min(b0 + per, n);
  uint32_t sum = 0;
  for (int64_t t = b0; t < b1; ++t) sum += v[t];
  part[j] = sum;
  __syncthreads();
  for (int d = 1; d < kChunkThreads; d <<= 1) {
    const uint32_t x = j >= d ? part[j - d] : 0u;
    __syncthreads();
    part[j] += x;
    __syncthreads();
  }
  uint32_t run = j > 0 ? part[j - 1] : 0u;
  for (int64_t t = b0; t < b1; ++t) {
    const uint32_t c = v[t];
    v[t] = run;
    run += c;
  }
}

__global__ __launch_bounds__(256) void k_chunk_offsets(const uint32_t* __restrict__ ranges,
                                                       int64_t n_tiles, int chunk,
                                                       const uint32_t* __restrict__ bbase,
                                                       uint32_t* __restrict__ offset) {
  __shared__ uint32_t part[256];
  const int j = threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * kChunkBlock + (int64_t)j * kChunkPer;
  uint32_t c[kChunkPer];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kChunkPer; ++k) {
    c[k] = t0 + k < n_tiles ? chunk_count(ranges, t0 + k, chunk) : 0u;
    sum += c[k];
  }
  part[j] = sum;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    const uint32_t x = j >= d ? part[j - d] : 0u;
    __syncthreads();
    part[j] += x;
    __syncthreads();
  }
  uint32_t run = bbase[blockIdx.x] + (j > 0 ? part[j - 1] : 0u);
#pragma unroll
  for (int k = 0; k < kChunkPer; ++k) {
    if (t0 + k < n_tiles) offset[t0 + k] = run;
    run += c[k];
    if (t0 + k == n_tiles - 1) offset[n_tiles] = run;
  }
}

__global__ __launch_bounds__(256) void k_chunk_items(const uint32_t* __restrict__ offset,
                                                     int64_t n_tiles, int64_t max_items,
                                                     uint32_t* __restrict__ items) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_tiles) return;
  for (uint32_t i = offset[t]; i < offset[t + 1] && (int64_t)i < max_items; ++i) items[i] = (uint32_t)t;
}

}  // namespace gsmi

using namespace gsmi;

extern "C" {

size_t gs_tile_order_workspace_bytes(int64_t n_tiles) {
  (void)n_tiles;
  return 3 * kOrderBuckets * sizeof(uint32_t);
}

gs_status gs_tile_order(const uint32_t* tile_ranges, int64_t n_tiles, void* ws, size_t ws_bytes,
                        uint32_t* order, void* stream) {
  clear_error();
  GS_REQUIRE(n_tiles >= 0 && n_tiles < (int64_t(1) << 32), "gs_tile_order: bad n_tiles");
  if (n_tiles == 0) return GS_OK;
  GS_REQUIRE(tile_ranges && ws && order, "gs_tile_order: NULL argument");
  GS_REQUIRE(ws_bytes >= gs_tile_order_workspace_bytes(n_tiles), "gs_tile_order: workspace too small");
  uint32_t* hist = (uint32_t*)ws;
  uint32_t* start = hist + kOrderBuckets;
  uint32_t* cursor = start + kOrderBuckets;
  hipStream_t s = as_stream(stream);
  if (n_tiles <= kOrderOneMax) {
    hipLaunchKernelGGL(k_order_one, dim3(1), dim3(kOrderOneThreads), 0, s, tile_ranges,
                       (int)n_tiles, order);
    GS_LAUNCH_CHECK("gs_tile_order/one");
    return GS_OK;
  }
  gs_status st = gs_zero(ws, 3 * kOrderBuckets * sizeof(uint32_t), stream);
  if (st != GS_OK) return st;
  const unsigned blocks = (unsigned)ceil_div(n_tiles, kOrderThreads);
  hipLaunchKernelGGL(k_order_count, dim3(blocks), dim3(kOrderThreads), 0, s, tile_ranges, n_tiles,
                     hist);
  GS_LAUNCH_CHECK("gs_tile_order/count");
  hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64), 0, s, hist, start);
  GS_LAUNCH_CHECK("gs_tile_order/scan");
  hipLaunchKernelGGL(k_order_scatter, dim3(blocks), dim3(kOrderThreads), 0, s, tile_ranges,
                     n_tiles, start, cursor, order);
  GS_LAUNCH_CHECK("gs_tile_order/scatter");
  return GS_OK;
}

int64_t gs_chunk_max_items(int64_t n_tiles, int64_t dup_capacity, int32_t chunk) {
  if (n_tiles < 0 || dup_capacity < 0 || chunk <= 0) return 0;
  return n_tiles + dup_capacity / chunk + 1;
}

gs_status gs_chunk_items(const uint32_t* tile_ranges, int64_t n_tiles, int32_t chunk,
                         int64_t max_items, uint32_t* chunk_offset, uint32_t* chunk_items,
                         void* stream) {
  clear_error();
  GS_REQUIRE(n_tiles >= 0 && n_tiles < (int64_t(1) << 31), "gs_chunk_items: bad n_tiles");
  GS_REQUIRE(chunk > 0 && chunk % kScheduleWave == 0, "gs_chunk_items: chunk %d not a positive multiple of 64", chunk);
  GS_REQUIRE(tile_ranges && chunk_offset && chunk_items, "gs_chunk_items: NULL argument");
  GS_REQUIRE(max_items > 0, "gs_chunk_items: max_items must be positive");
  hipStream_t s = as_stream(stream);
  const int64_t nb = ceil_div(n_tiles, (int64_t)kChunkBlock);
  if (n_tiles > kChunkScanOne && nb <= max_items) {
    // the block sums live in chunk_items until the fill below overwrites it
    hipLaunchKernelGGL(k_chunk_bsum, dim3((unsigned)nb), dim3(256), 0, s, tile_ranges, n_tiles,
                       chunk, chunk_items);
    GS_LAUNCH_CHECK("gs_chunk_items/bsum");
    hipLaunchKernelGGL(k_chunk_bscan, dim3(1), dim3(kChunkThreads), 0, s, chunk_items, nb);
    GS_LAUNCH_CHECK("gs_chunk_items/bscan");
    hipLaunchKernelGGL(k_chunk_offsets, dim3((unsigned)nb), dim3(256), 0, s, tile_ranges, n_tiles,
                       chunk, chunk_items, chunk_offset);
    GS_LAUNCH_CHECK("gs_chunk_items/offsets");
  } else {
    hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(kChunkThreads), 0, s, tile_ranges, n_tiles,
                       chunk, chunk_offset);
    GS_LAUNCH_CHECK("gs_chunk_items/scan");
  }
  if (n_tiles > 0) {
    hipLaunchKernelGGL(k_chunk_items, dim3((unsigned)ceil_div(n_tiles, 256)), dim3(256), 0, s,
                       chunk_offset, n_tiles, max_items, chunk_items);
    GS_LAUNCH_CHECK("gs_chunk_items/items");
  }
  return GS_OK;
}

}  // extern "C"
