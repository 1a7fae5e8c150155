// knn.hip — exact k nearest neighbours of isosurface points (the plain
// initialisation sets each Gaussian's scale from its 3 nearest neighbours;
// the learned initialisation reads 16-NN features).
//
// Device pipeline (sizes that depend on the data stay on the device):
//   k_bbox_partial / k_grid_params   bounding box -> uniform grid (cell edge
//                                    (volume / n)^(1/3), capped cell count)
//   k_cell_count                     cell of each point, per-cell counts
//   k_scan_*                         exclusive scan of the counts
//   k_cell_scatter                   points grouped by cell (float4 x,y,z,id)
//   k_query                          one thread per point, in cell order for
//                                    cache locality: cells in growing
//                                    Chebyshev shells until the k-th best
//                                    distance is within the distance to the
//                                    searched box (exact); the K best
//                                    (distance^2, index) pairs stay sorted in
//                                    registers, ties broken by index.
#include <math.h>

#include "gs_device.h"

namespace gsmi {

constexpr int kKnnThreads = 256;
constexpr int kKnnScanPer = 8;
constexpr int kKnnScanItems = kKnnThreads * kKnnScanPer;

struct GridParams {
  float lo[3];
  float h, inv_h;
  int g[3];
  int64_t n_cells;
};

static inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct KnnLayout {
  int64_t max_cells, nb_pts, nb_scan;
  size_t off_part, off_params, off_cell, off_count, off_cursor, off_sorted, off_bsum, total;
};

static KnnLayout knn_layout(int64_t n) {
  KnnLayout L;
  L.max_cells = 2 * (n > 0 ? n : 1) + 1024;
  L.nb_pts = ceil_div(n > 0 ? n : 1, kKnnThreads);
  L.nb_scan = ceil_div(L.max_cells + 1, kKnnScanItems);
  size_t o = 0;
  L.off_part = o; o += a256(sizeof(float) * 6 * (size_t)L.nb_pts);
  L.off_params = o; o += a256(sizeof(GridParams));
  L.off_cell = o; o += a256(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
  L.off_count = o; o += a256(sizeof(uint32_t) * (size_t)(L.max_cells + 1));
  L.off_cursor = o; o += a256(sizeof(uint32_t) * (size_t)L.max_cells);
  L.off_sorted = o; o += a256(sizeof(float4) * (size_t)(n > 0 ? n : 1));
  L.off_bsum = o; o += a256(sizeof(uint32_t) * (size_t)L.nb_scan);
  L.total = o;
  return L;
}

__global__ __launch_bounds__(kKnnThreads) void k_bbox_partial(const float* __restrict__ pts,
                                                              int64_t n, float* __restrict__ part) {
  __shared__ float sm[6][kKnnThreads / 64];
  const int64_t i = (int64_t)blockIdx.x * kKnnThreads + threadIdx.x;
  float v[6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float x = i < n ? pts[a * n + i] : 0.0f;
    v[a] = i < n ? x : INFINITY;
    v[3 + a] = i < n ? x : -INFINITY;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      v[a] = fminf(v[a], __shfl_xor(v[a], d, 64));
      v[3 + a] = fmaxf(v[3 + a], __shfl_xor(v[3 + a], d, 64));
    }
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int a = 0; a < 6; ++a) sm[a][threadIdx.x >> 6] = v[a];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    float r = sm[a][0];
    for (int w = 1; w < kKnnThreads / 64; ++w) r = a < 3 ? fminf(r, sm[a][w]) : fmaxf(r, sm[a][w]);
    part[(int64_t)blockIdx.x * 6 + a] = r;
  }
}

__global__ void k_grid_params(const float* __restrict__ part, int64_t nb, int64_t n,
                              int64_t max_cells, GridParams* __restrict__ P) {
  if (threadIdx.x != 0) return;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t b = 0; b < nb; ++b)
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], part[b * 6 + a]);
      hi[a] = fmaxf(hi[a], part[b * 6 + 3 + a]);
    }
  float ext[3], vol = 1.0f, emax = 0.0f;
  for (int a = 0; a < 3; ++a) {
    ext[a] = fmaxf(hi[a] - lo[a], 0.0f);
    emax = fmaxf(emax, ext[a]);
  }
  if (!(emax > 0.0f)) emax = 1.0f;
  for (int a = 0; a < 3; ++a) vol *= fmaxf(ext[a], emax * 1e-3f);
  float h = cbrtf(vol / (float)(n > 0 ? n : 1));
  h = fmaxf(h, emax * 1e-6f);
  int g[3];
  for (int it = 0; it < 64; ++it) {
    int64_t cells = 1;
    for (int a = 0; a < 3; ++a) {
      g[a] = max(1, (int)ceilf(ext[a] / h) + 1);
      cells *= g[a];
    }
    if (cells <= max_cells) break;
    h *= 1.25f;
  }
  for (int a = 0; a < 3; ++a) {
    P->lo[a] = lo[a];
    P->g[a] = g[a];
  }
  P->h = h;
  P->inv_h = 1.0f / h;
  P->n_cells = (int64_t)g[0] * g[1] * g[2];
}

__device__ __forceinline__ int cell_coord(float x, float lo, float inv_h, int g) {
  return min(max((int)floorf((x - lo) * inv_h), 0), g - 1);
}

__global__ __launch_bounds__(kKnnThreads) void k_cell_count(const float* __restrict__ pts, int64_t n,
                                                            const GridParams* __restrict__ P,
                                                            uint32_t* __restrict__ cell,
                                                            uint32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * kKnnThreads + threadIdx.x;
  if (i >= n) return;
  const GridParams G = *P;
  const int cx = cell_coord(pts[i], G.lo[0], G.inv_h, G.g[0]);
  const int cy = cell_coord(pts[n + i], G.lo[1], G.inv_h, G.g[1]);
  const int cz = cell_coord(pts[2 * n + i], G.lo[2], G.inv_h, G.g[2]);
  const uint32_t c = (uint32_t)(((int64_t)cz * G.g[1] + cy) * G.g[0] + cx);
  cell[i] = c;
  atomicAdd(&count[c], 1u);
}

// exclusive scan of count[0 .. n_cells] (n_cells read from P) in place; the
// extra entry (zero before the scan) becomes n and closes the last cell
__global__ __launch_bounds__(kKnnThreads) void k_knn_scan_reduce(const uint32_t* __restrict__ count,
                                                                 const GridParams* __restrict__ P,
                                                                 uint32_t* __restrict__ bsum) {
  const int64_t nc = P->n_cells + 1;
  const int64_t base = (int64_t)blockIdx.x * kKnnScanItems;
  uint32_t s = 0;
  for (int k = 0; k < kKnnScanPer; ++k) {
    const int64_t i = base + k * kKnnThreads + threadIdx.x;
    if (i < nc) s += count[i];
  }
  __shared__ uint32_t sm[kKnnThreads];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int d = kKnnThreads / 2; d > 0; d >>= 1) {
    if (threadIdx.x < d) sm[threadIdx.x] += sm[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(kKnnThreads) void k_knn_scan_top(uint32_t* __restrict__ bsum, int64_t nb) {
  if (threadIdx.x != 0) return;
  uint32_t run = 0;
  for (int64_t b = 0; b < nb; ++b) {
    const uint32_t x = bsum[b];
    bsum[b] = run;
    run += x;
  }
}

__global__ __launch_bounds__(kKnnThreads) void k_knn_scan_down(uint32_t* __restrict__ count,
                                                               const GridParams* __restrict__ P,
                                                               const uint32_t* __restrict__ bsum) {
  __shared__ uint32_t sm[kKnnScanItems];
  const int64_t nc = P->n_cells + 1;
  const int64_t base = (int64_t)blockIdx.x * kKnnScanItems;
  for (int k = 0; k < kKnnScanPer; ++k) {
    const int li = k * kKnnThreads + threadIdx.x;
    const int64_t i = base + li;
    sm[li] = i < nc ? count[i] : 0u;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = bsum[blockIdx.x];
    for (int li = 0; li < kKnnScanItems; ++li) {
      const uint32_t x = sm[li];
      sm[li] = run;
      run += x;
    }
  }
  __syncthreads();
  for (int k = 0; k < kKnnScanPer; ++k) {
    const int li = k * kKnnThreads + threadIdx.x;
    const int64_t i = base + li;
    if (i < nc) count[i] = sm[li];
  }
}

__global__ __launch_bounds__(kKnnThreads) void k_cell_scatter(const float* __restrict__ pts, int64_t n,
                                                              const uint32_t* __restrict__ cell,
                                                              const uint32_t* __restrict__ start,
                                                              uint32_t* __restrict__ cursor,
                                                              float4* __restrict__ sorted) {
  const int64_t i = (int64_t)blockIdx.x * kKnnThreads + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = cell[i];
  const uint32_t pos = start[c] + atomicAdd(&cursor[c], 1u);
  sorted[pos] = make_float4(pts[i], pts[n + i], pts[2 * n + i], __int_as_float((int)i));
}

template <int K>
__device__ __forceinline__ void knn_insert(float (&bd)[K], int (&bi)[K], float d2, int j) {
  // (d2, j) goes in if it beats the current K-th entry; bubble it into place
  if (!(d2 < bd[K - 1] || (d2 == bd[K - 1] && j < bi[K - 1]))) return;
  bd[K - 1] = d2;
  bi[K - 1] = j;
#pragma unroll
  for (int s = K - 1; s > 0; --s) {
    const bool sw = bd[s] < bd[s - 1] || (bd[s] == bd[s - 1] && bi[s] < bi[s - 1]);
    const float td = sw ? bd[s - 1] : bd[s];
    const int ti = sw ? bi[s - 1] : bi[s];
    bd[s - 1] = sw ? bd[s] : bd[s - 1];
    bi[s - 1] = sw ? bi[s] : bi[s - 1];
    bd[s] = td;
    bi[s] = ti;
  }
}

template <int K>
__global__ __launch_bounds__(kKnnThreads) void k_query(const float4* __restrict__ sorted, int64_t n,
                                                       int k, const GridParams* __restrict__ P,
                                                       const uint32_t* __restrict__ start,
                                                       int32_t* __restrict__ idx,
                                                       float* __restrict__ dist,
                                                       float* __restrict__ mean_dist) {
  const int64_t s = (int64_t)blockIdx.x * kKnnThreads + threadIdx.x;
  if (s >= n) return;
  const GridParams G = *P;
  const float4 q = sorted[s];
  const int qi = __float_as_int(q.w);
  const int cx = cell_coord(q.x, G.lo[0], G.inv_h, G.g[0]);
  const int cy = cell_coord(q.y, G.lo[1], G.inv_h, G.g[1]);
  const int cz = cell_coord(q.z, G.lo[2], G.inv_h, G.g[2]);
  float bd[K];
  int bi[K];
#pragma unroll
  for (int t = 0; t < K; ++t) {
    bd[t] = INFINITY;
    bi[t] = 0x7fffffff;
  }
  const int rmax = max(G.g[0], max(G.g[1], G.g[2]));
  for (int r = 0; r <= rmax; ++r) {
    const int z0 = max(cz - r, 0), z1 = min(cz + r, G.g[2] - 1);
    const int y0 = max(cy - r, 0), y1 = min(cy + r, G.g[1] - 1);
    const int x0 = max(cx - r, 0), x1 = min(cx + r, G.g[0] - 1);
    for (int z = z0; z <= z1; ++z)
      for (int y = y0; y <= y1; ++y) {
        const bool face = (abs(z - cz) == r) || (abs(y - cy) == r);
        // interior rows of the shell only contribute their two end cells
        const int step = face ? 1 : max(x1 - x0, 1);
        for (int x = x0; x <= x1; x += step) {
          if (!face && abs(x - cx) != r) continue;
          const int64_t c = ((int64_t)z * G.g[1] + y) * G.g[0] + x;
          const uint32_t a = start[c], b = start[c + 1];
          for (uint32_t j = a; j < b; ++j) {
            const float4 p = sorted[j];
            const int pj = __float_as_int(p.w);
            if (pj == qi) continue;
            const float dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
            knn_insert<K>(bd, bi, fmaf(dx, dx, fmaf(dy, dy, dz * dz)), pj);
          }
        }
      }
    // every unsearched point is at least `wall` away
    float wall = INFINITY;
    if (cx - r > 0) wall = fminf(wall, q.x - (G.lo[0] + (cx - r) * G.h));
    if (cx + r < G.g[0] - 1) wall = fminf(wall, G.lo[0] + (cx + r + 1) * G.h - q.x);
    if (cy - r > 0) wall = fminf(wall, q.y - (G.lo[1] + (cy - r) * G.h));
    if (cy + r < G.g[1] - 1) wall = fminf(wall, G.lo[1] + (cy + r + 1) * G.h - q.y);
    if (cz - r > 0) wall = fminf(wall, q.z - (G.lo[2] + (cz - r) * G.h));
    if (cz + r < G.g[2] - 1) wall = fminf(wall, G.lo[2] + (cz + r + 1) * G.h - q.z);
    wall = fmaxf(wall, 0.0f);
    float kth = bd[0];
#pragma unroll
    for (int t = 1; t < K; ++t) kth = (t == k - 1) ? bd[t] : kth;
    if (kth <= wall * wall * 0.9999f || wall == INFINITY) break;
  }
  float dsum = 0.0f;
  int found = 0;
#pragma unroll
  for (int t = 0; t < K; ++t)
    if (t < k) {
      const float d = sqrtf(bd[t]);
      if (idx) idx[(int64_t)qi * k + t] = bi[t] == 0x7fffffff ? -1 : bi[t];
      if (dist) dist[(int64_t)qi * k + t] = d;
      if (bi[t] != 0x7fffffff) {
        dsum += d;
        ++found;
      }
    }
  // mean over the neighbours found, in ascending order of distance
  if (mean_dist) mean_dist[qi] = found ? dsum / (float)found : 0.0f;
}

// Plain initialisation of the Gaussians of surface points (one thread per
// point): mean = point, colour coefficient sqrt(pi) n (so that the degree-0
// colour max(0, C0 f + 1/2) is (n + 1)/2), and, when the k-NN mean distances
// d are given, an isotropic log-scale log(max(d, 1e-6)), the identity
// rotation and a fixed opacity logit.
__global__ __launch_bounds__(kKnnThreads) void k_plain_init(
    const float* __restrict__ pts, const float* __restrict__ nrm, int64_t n,
    const float* __restrict__ d, float logit, float* __restrict__ mean,
    float* __restrict__ log_scale, float* __restrict__ quat, float* __restrict__ opacity_logit,
    float* __restrict__ color) {
  const int64_t i = (int64_t)blockIdx.x * kKnnThreads + threadIdx.x;
  if (i >= n) return;
  const float kSqrtPi = 1.7724538509055160f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    mean[a * n + i] = pts[a * n + i];
    color[a * n + i] = kSqrtPi * nrm[a * n + i];
  }
  if (!d) return;
  const float ls = logf(fmaxf(d[i], 1e-6f));
#pragma unroll
  for (int a = 0; a < 3; ++a) log_scale[a * n + i] = ls;
  quat[i] = 1.0f;
  quat[n + i] = quat[2 * n + i] = quat[3 * n + i] = 0.0f;
  opacity_logit[i] = logit;
}

}  // namespace gsmi

using namespace gsmi;

extern "C" {

size_t gs_knn_workspace_bytes(int64_t n, int32_t k) {
  (void)k;
  if (n < 0) return 0;
  return knn_layout(n).total;
}

gs_status gs_knn(const float* pts, int64_t n, int32_t k, void* ws, size_t ws_bytes, int32_t* idx,
                 float* dist, float* mean_dist, void* stream) {
  clear_error();
  GS_REQUIRE(k >= 1 && k <= 32, "gs_knn: k=%d outside [1, 32]", k);
  GS_REQUIRE(n >= 0 && n < (int64_t(1) << 31), "gs_knn: n=%lld outside [0, 2^31)", (long long)n);
  if (n == 0) return GS_OK;
  GS_REQUIRE(pts && ws, "gs_knn: NULL points or workspace");
  GS_REQUIRE(idx || dist || mean_dist, "gs_knn: no output requested");
  const KnnLayout L = knn_layout(n);
  GS_REQUIRE(ws_bytes >= L.total, "gs_knn: workspace %zu < required %zu", ws_bytes, L.total);
  GS_REQUIRE(((uintptr_t)ws & 255) == 0, "gs_knn: workspace must be 256-byte aligned");
  char* w = (char*)ws;
  float* part = (float*)(w + L.off_part);
  GridParams* P = (GridParams*)(w + L.off_params);
  uint32_t* cell = (uint32_t*)(w + L.off_cell);
  uint32_t* count = (uint32_t*)(w + L.off_count);
  uint32_t* cursor = (uint32_t*)(w + L.off_cursor);
  float4* sorted = (float4*)(w + L.off_sorted);
  uint32_t* bsum = (uint32_t*)(w + L.off_bsum);
  hipStream_t s = as_stream(stream);
  const unsigned nb = (unsigned)L.nb_pts;
  hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(kKnnThreads), 0, s, pts, n, part);
  GS_LAUNCH_CHECK("gs_knn/bbox");
  hipLaunchKernelGGL(k_grid_params, dim3(1), dim3(64), 0, s, part, L.nb_pts, n, L.max_cells, P);
  GS_LAUNCH_CHECK("gs_knn/grid");
  gs_status st = gs_zero(count, sizeof(uint32_t) * (size_t)(L.max_cells + 1), stream);
  if (st != GS_OK) return st;
  st = gs_zero(cursor, sizeof(uint32_t) * (size_t)L.max_cells, stream);
  if (st != GS_OK) return st;
  hipLaunchKernelGGL(k_cell_count, dim3(nb), dim3(kKnnThreads), 0, s, pts, n, P, cell, count);
  GS_LAUNCH_CHECK("gs_knn/count");
  // scan n_cells + 1 entries so that start[n_cells] = n closes the last cell
  hipLaunchKernelGGL(k_knn_scan_reduce, dim3((unsigned)L.nb_scan), dim3(kKnnThreads), 0, s, count,
                     P, bsum);
  GS_LAUNCH_CHECK("gs_knn/scan_reduce");
  hipLaunchKernelGGL(k_knn_scan_top, dim3(1), dim3(64), 0, s, bsum, L.nb_scan);
  GS_LAUNCH_CHECK("gs_knn/scan_top");
  hipLaunchKernelGGL(k_knn_scan_down, dim3((unsigned)L.nb_scan), dim3(kKnnThreads), 0, s, count, P,
                     bsum);
  GS_LAUNCH_CHECK("gs_knn/scan_down");
  hipLaunchKernelGGL(k_cell_scatter, dim3(nb), dim3(kKnnThreads), 0, s, pts, n, cell, count, cursor,
                     sorted);
  GS_LAUNCH_CHECK("gs_knn/scatter");
#define GS_KNN_Q(KK)                                                                        \
  hipLaunchKernelGGL(k_query<KK>, dim3(nb), dim3(kKnnThreads), 0, s, sorted, n, k, P, count, \
                     idx, dist, mean_dist)
  if (k <= 4) GS_KNN_Q(4);
  else if (k <= 8) GS_KNN_Q(8);
  else if (k <= 16) GS_KNN_Q(16);
  else GS_KNN_Q(32);
#undef GS_KNN_Q
  GS_LAUNCH_CHECK("gs_knn/query");
  return GS_OK;
}

size_t gs_plain_init_workspace_bytes(int64_t n) {
  if (n < 0) return 0;
  return a256(knn_layout(n).total) + a256(sizeof(float) * (size_t)(n > 0 ? n : 1));
}

gs_status gs_plain_init(const float* pts, const float* normals, int64_t n, float opacity,
                        void* ws, size_t ws_bytes, float* mean, float* log_scale, float* quat,
                        float* opacity_logit, float* color, void* stream) {
  clear_error();
  GS_REQUIRE(n >= 0 && n < (int64_t(1) << 31), "gs_plain_init: n=%lld outside [0, 2^31)",
             (long long)n);
  if (n == 0) return GS_OK;
  GS_REQUIRE(pts && normals && mean && color, "gs_plain_init: NULL points, normals, mean or colour");
  const bool shape = log_scale != nullptr;
  GS_REQUIRE(!shape || (quat && opacity_logit && ws),
             "gs_plain_init: log_scale given without quat, opacity_logit or workspace");
  GS_REQUIRE(!shape || (opacity > 0.f && opacity < 1.f), "gs_plain_init: opacity %f outside (0, 1)",
             (double)opacity);
  float* d = nullptr;
  if (shape) {
    const size_t need = gs_plain_init_workspace_bytes(n);
    GS_REQUIRE(ws_bytes >= need, "gs_plain_init: workspace %zu < required %zu", ws_bytes, need);
    GS_REQUIRE(((uintptr_t)ws & 255) == 0, "gs_plain_init: workspace must be 256-byte aligned");
    const size_t off = a256(knn_layout(n).total);
    d = (float*)((char*)ws + off);
    gs_status st = gs_knn(pts, n, 3, ws, off, nullptr, nullptr, d, stream);
    if (st != GS_OK) return st;
  }
  const float logit = shape ? logf(opacity / (1.0f - opacity)) : 0.0f;
  hipLaunchKernelGGL(k_plain_init, dim3((unsigned)ceil_div(n, kKnnThreads)), dim3(kKnnThreads), 0,
                     as_stream(stream), pts, normals, n, d, logit, mean, log_scale, quat,
                     opacity_logit, color);
  GS_LAUNCH_CHECK("gs_plain_init");
  return GS_OK;
}

}  // extern "C"
