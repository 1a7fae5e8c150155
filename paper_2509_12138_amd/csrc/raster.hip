// raster.hip — front-to-back compositing (3D-GS rasteriser that the paper's
// Sec. II "Parallel Training" runs per partition) and its reverse replay.
//
// Layout on gfx950: one wave64 per bin tile.  A 16x16 tile gives each lane 4
// pixels of one column, so every Gaussian staged in LDS is read once per 4
// evaluations and the backward's wave reduction is amortised over 256
// pixels.  Gaussians are staged 64 at a time (one gathered record per lane).
// Work-group ids are remapped so that neighbouring tiles run on the same
// XCD and share its L2.
//
// The backward recovers each pixel's transmittance by dividing T_final by
// (1 - alpha) in reverse order (STORED) or first replays the forward for its
// tile (RECOMPUTE).  Per (tile, Gaussian) the 9 gradient components are
// summed over the wave with DPP and added with one FP32 atomic each.
#include "gs_device.h"

namespace gsmi {

constexpr int kRasterWave = 64;

// XCD-aware tile order: work-group i runs on XCD (i mod 8); give each XCD a
// contiguous range of tiles.
__device__ __forceinline__ int64_t tile_of_block(int64_t n_tiles) {
  const int64_t chunk = (n_tiles + 7) / 8;
  const int64_t i = blockIdx.x;
  return (i & 7) * chunk + (i >> 3);
}

__device__ __forceinline__ Splat load_splat(const float* __restrict__ rec, uint32_t id) {
  const float4* r = reinterpret_cast<const float4*>(rec + (int64_t)id * GS_REC_STRIDE);
  float4 a = r[0], b = r[1], c = r[2];
  Splat s;
  s.pad1 = s.pad2 = 0.0f;
  s.mx = a.x;
  s.my = a.y;
  s.A = -0.5f * kLog2e * a.z;
  s.B = -kLog2e * a.w;
  s.C = -0.5f * kLog2e * b.x;
  s.o = b.y;
  s.r = b.z;
  s.g = b.w;
  s.b = c.x;
  s.thr = -__builtin_amdgcn_logf(255.0f * b.y);   // -log2(255 o)
  return s;
}

template <int TW, int TH>
struct TileGeom {
  static constexpr int PX = TW * TH / kRasterWave;      // pixels per lane
  static constexpr int RSTEP = kRasterWave / TW;        // rows between a lane's pixels
  static_assert(TW * TH % kRasterWave == 0 && kRasterWave % TW == 0, "tile shape");
};

// Forward pass of one tile for one lane's PX pixels.  WITH_COLOR=false is the
// replay used by the backward in RECOMPUTE mode.
template <int TW, int TH, bool WITH_COLOR>
__device__ __forceinline__ void tile_forward(const float* __restrict__ rec,
                                             const uint32_t* __restrict__ ids, uint32_t start,
                                             uint32_t end, const float fx, const float* fy,
                                             const bool* inside, Splat* s_splat, float* T,
                                             float (*C)[3], int* last) {
  constexpr int PX = TileGeom<TW, TH>::PX;
  const int lane = threadIdx.x;
  bool done[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    T[k] = 1.0f;
    last[k] = 0;
    done[k] = !inside[k];
    if (WITH_COLOR) C[k][0] = C[k][1] = C[k][2] = 0.0f;
  }
  for (uint32_t b0 = start; b0 < end; b0 += kRasterWave) {
    bool lane_done = true;
#pragma unroll
    for (int k = 0; k < PX; ++k) lane_done = lane_done && done[k];
    if (__all(lane_done)) break;
    const int n = (int)min((uint32_t)kRasterWave, end - b0);
    __syncthreads();
    if (lane < n) s_splat[lane] = load_splat(rec, ids[b0 + lane]);
    __syncthreads();
    for (int j = 0; j < n; ++j) {
      const Splat sp = s_splat[j];
      const float dx = __fsub_rn(fx, sp.mx);
      float p2[PX];
      splat_p2_column<PX>(sp, dx, fy, p2);
      bool pass[PX], any = false;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        pass[k] = !done[k] && splat_pass(sp, p2[k]);
        any = any || pass[k];
      }
      if (!__any(any)) continue;                    // whole wave skips this entry
      const int pos = (int)(b0 - start) + j + 1;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        if (!pass[k]) continue;
        const float alpha = fminf(kAlphaMax, sp.o * splat_gauss(p2[k]));
        const float Tn = T[k] * (1.0f - alpha);
        if (Tn < kTMin) {
          done[k] = true;
          continue;
        }
        if (WITH_COLOR) {
          const float w = alpha * T[k];
          C[k][0] = fmaf(sp.r, w, C[k][0]);
          C[k][1] = fmaf(sp.g, w, C[k][1]);
          C[k][2] = fmaf(sp.b, w, C[k][2]);
        }
        T[k] = Tn;
        last[k] = pos;
      }
    }
  }
}

template <int TW, int TH>
__global__ __launch_bounds__(kRasterWave) void k_raster_fwd(
    const float* __restrict__ rec, const uint32_t* __restrict__ ids,
    const uint32_t* __restrict__ ranges, int W, int H, int tiles_x, int tiles_per_slot,
    int64_t n_tiles, float bg0, float bg1, float bg2, float* __restrict__ image,
    float* __restrict__ T_final, int32_t* __restrict__ n_contrib) {
  constexpr int PX = TileGeom<TW, TH>::PX, RSTEP = TileGeom<TW, TH>::RSTEP;
  __shared__ Splat s_splat[kRasterWave];
  const int64_t tile = tile_of_block(n_tiles);
  if (tile >= n_tiles) return;
  const int slot = (int)(tile / tiles_per_slot);
  const int t = (int)(tile - (int64_t)slot * tiles_per_slot);
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  const int lane = threadIdx.x;
  const int px = tx * TW + (lane % TW);
  const int py0 = ty * TH + lane / TW;
  const float fx = (float)px + 0.5f;
  float fy[PX];
  bool inside[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    const int py = py0 + k * RSTEP;
    fy[k] = (float)py + 0.5f;
    inside[k] = (px < W) && (py < H);
  }
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  float T[PX], C[PX][3];
  int last[PX];
  tile_forward<TW, TH, true>(rec, ids, start, end, fx, fy, inside, s_splat, T, C, last);
  const int64_t HW = (int64_t)H * W;
  float* img = image + (int64_t)slot * 3 * HW;
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    if (!inside[k]) continue;
    const int64_t o = (int64_t)(py0 + k * RSTEP) * W + px;
    img[o] = C[k][0] + T[k] * bg0;
    img[HW + o] = C[k][1] + T[k] * bg1;
    img[2 * HW + o] = C[k][2] + T[k] * bg2;
    if (T_final) T_final[(int64_t)slot * HW + o] = T[k];
    if (n_contrib) n_contrib[(int64_t)slot * HW + o] = last[k];
  }
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
  return v;
}

template <int TW, int TH, bool RECOMPUTE>
__global__ __launch_bounds__(kRasterWave) void k_raster_bwd(
    const float* __restrict__ rec, const uint32_t* __restrict__ ids,
    const uint32_t* __restrict__ ranges, int W, int H, int tiles_x, int tiles_per_slot,
    int64_t n_tiles, float bg0, float bg1, float bg2, const float* __restrict__ T_final,
    const int32_t* __restrict__ n_contrib, const float* __restrict__ d_image,
    float* __restrict__ d_rec) {
  constexpr int PX = TileGeom<TW, TH>::PX, RSTEP = TileGeom<TW, TH>::RSTEP;
  __shared__ Splat s_splat[kRasterWave];
  __shared__ uint32_t s_id[kRasterWave];
  const int64_t tile = tile_of_block(n_tiles);
  if (tile >= n_tiles) return;
  const int slot = (int)(tile / tiles_per_slot);
  const int t = (int)(tile - (int64_t)slot * tiles_per_slot);
  const int ty = t / tiles_x, tx = t - ty * tiles_x;
  const int lane = threadIdx.x;
  const int px = tx * TW + (lane % TW);
  const int py0 = ty * TH + lane / TW;
  const float fx = (float)px + 0.5f;
  float fy[PX];
  bool inside[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    const int py = py0 + k * RSTEP;
    fy[k] = (float)py + 0.5f;
    inside[k] = (px < W) && (py < H);
  }
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  if (start >= end) return;
  const int64_t HW = (int64_t)H * W;
  float T[PX];
  int last[PX];
  if (RECOMPUTE) {
    tile_forward<TW, TH, false>(rec, ids, start, end, fx, fy, inside, s_splat, T, nullptr, last);
  } else {
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      const int64_t o = (int64_t)slot * HW + (int64_t)(py0 + k * RSTEP) * W + px;
      T[k] = inside[k] ? T_final[o] : 1.0f;
      last[k] = inside[k] ? n_contrib[o] : 0;
    }
  }
  // dIacc = dI . (sum of the colour blended behind + bg T_final), per pixel
  float dI[PX][3], dIacc[PX];
  const float* dimg = d_image + (int64_t)slot * 3 * HW;
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    const int64_t o = (int64_t)(py0 + k * RSTEP) * W + px;
    dI[k][0] = inside[k] ? dimg[o] : 0.0f;
    dI[k][1] = inside[k] ? dimg[HW + o] : 0.0f;
    dI[k][2] = inside[k] ? dimg[2 * HW + o] : 0.0f;
    dIacc[k] = T[k] * (dI[k][0] * bg0 + dI[k][1] * bg1 + dI[k][2] * bg2);
  }
  int lmax = 0;
#pragma unroll
  for (int k = 0; k < PX; ++k) lmax = max(lmax, last[k]);
  lmax = min(wave_max_int(lmax), (int)(end - start));
  for (int hi = lmax; hi > 0; hi -= kRasterWave) {
    const int lo = max(0, hi - kRasterWave);
    const int n = hi - lo;
    __syncthreads();
    if (lane < n) {
      const uint32_t id = ids[start + lo + lane];
      s_id[lane] = id;
      s_splat[lane] = load_splat(rec, id);
    }
    __syncthreads();
    for (int j = n - 1; j >= 0; --j) {
      const Splat sp = s_splat[j];
      const int pos = lo + j + 1;
      const float dx = __fsub_rn(fx, sp.mx);
      float p2[PX];
      splat_p2_column<PX>(sp, dx, fy, p2);
      bool pass[PX], any = false;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        pass[k] = (pos <= last[k]) && splat_pass(sp, p2[k]);
        any = any || pass[k];
      }
      if (!__any(any)) continue;
      // per-lane sums over the lane's pixels; the geometric gradients of the
      // lane follow from sG = sum G, sGdy = sum G dy, sGdy2 = sum G dy^2 with
      // G = dL/d(power) (dx is shared by the lane's column)
      float sG = 0.f, sGdy = 0.f, sGdy2 = 0.f, so = 0.f, sr = 0.f, sg = 0.f, sb = 0.f;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        if (!pass[k]) continue;
        const float gss = splat_gauss(p2[k]);
        const float a = sp.o * gss;
        const float alpha = fminf(kAlphaMax, a);
        const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);
        const float Tb = T[k] * inv;                 // transmittance in front of it
        const float w = alpha * Tb;
        const float dIc = fmaf(dI[k][2], sp.b, fmaf(dI[k][1], sp.g, dI[k][0] * sp.r));
        const float dLda = fmaf(Tb, dIc, -inv * dIacc[k]);
        dIacc[k] = fmaf(w, dIc, dIacc[k]);
        T[k] = Tb;
        sr = fmaf(dI[k][0], w, sr);
        sg = fmaf(dI[k][1], w, sg);
        sb = fmaf(dI[k][2], w, sb);
        if (a < kAlphaMax) {
          const float G = dLda * alpha;
          const float dy = __fsub_rn(fy[k], sp.my);
          const float Gdy = G * dy;
          so = fmaf(dLda, gss, so);
          sG += G;
          sGdy += Gdy;
          sGdy2 = fmaf(Gdy, dy, sGdy2);
        }
      }
      const float bdx = sp.B * dx;
      float g_mx = fmaf(2.0f * sp.A * dx, sG, sp.B * sGdy);   // x -ln2 below
      float g_my = fmaf(2.0f * sp.C, sGdy, bdx * sG);         // x -ln2 below
      float g_q11 = dx * dx * sG;                             // x -1/2 below
      float g_q12 = dx * sGdy;                                // x -1 below
      float g_q22 = sGdy2;                                    // x -1/2 below
      g_mx = wave_sum_to_lane63(g_mx);
      g_my = wave_sum_to_lane63(g_my);
      g_q11 = wave_sum_to_lane63(g_q11);
      g_q12 = wave_sum_to_lane63(g_q12);
      g_q22 = wave_sum_to_lane63(g_q22);
      so = wave_sum_to_lane63(so);
      sr = wave_sum_to_lane63(sr);
      sg = wave_sum_to_lane63(sg);
      sb = wave_sum_to_lane63(sb);
      if (lane == 63) {
        float* dst = d_rec + (int64_t)s_id[j] * GS_DREC_STRIDE;
        atomicAdd(dst + 0, -kLn2 * g_mx);
        atomicAdd(dst + 1, -kLn2 * g_my);
        atomicAdd(dst + 2, -0.5f * g_q11);
        atomicAdd(dst + 3, -g_q12);
        atomicAdd(dst + 4, -0.5f * g_q22);
        atomicAdd(dst + 5, so);
        atomicAdd(dst + 6, sr);
        atomicAdd(dst + 7, sg);
        atomicAdd(dst + 8, sb);
      }
    }
  }
}

// ---------------------------------------------------------------- dispatch

struct RasterArgs {
  const float* rec;
  const uint32_t* ids;
  const uint32_t* ranges;
  int W, H, tiles_x, tiles_per_slot;
  int64_t n_tiles;
  float bg[3];
};

template <int TW, int TH>
static void launch_fwd(const RasterArgs& a, float* image, float* T_final, int32_t* n_contrib,
                       hipStream_t s) {
  const int64_t blocks = 8 * ((a.n_tiles + 7) / 8);
  hipLaunchKernelGGL((k_raster_fwd<TW, TH>), dim3((unsigned)blocks), dim3(kRasterWave), 0, s,
                     a.rec, a.ids, a.ranges, a.W, a.H, a.tiles_x, a.tiles_per_slot, a.n_tiles,
                     a.bg[0], a.bg[1], a.bg[2], image, T_final, n_contrib);
}

template <int TW, int TH>
static void launch_bwd(const RasterArgs& a, const float* T_final, const int32_t* n_contrib,
                       const float* d_image, int mode, float* d_rec, hipStream_t s) {
  const int64_t blocks = 8 * ((a.n_tiles + 7) / 8);
  if (mode == GS_BWD_RECOMPUTE)
    hipLaunchKernelGGL((k_raster_bwd<TW, TH, true>), dim3((unsigned)blocks), dim3(kRasterWave), 0,
                       s, a.rec, a.ids, a.ranges, a.W, a.H, a.tiles_x, a.tiles_per_slot,
                       a.n_tiles, a.bg[0], a.bg[1], a.bg[2], T_final, n_contrib, d_image, d_rec);
  else
    hipLaunchKernelGGL((k_raster_bwd<TW, TH, false>), dim3((unsigned)blocks), dim3(kRasterWave), 0,
                       s, a.rec, a.ids, a.ranges, a.W, a.H, a.tiles_x, a.tiles_per_slot,
                       a.n_tiles, a.bg[0], a.bg[1], a.bg[2], T_final, n_contrib, d_image, d_rec);
}

// Tile shapes with a compiled rasteriser (one wave per tile).
#define GS_RASTER_SHAPES(X) X(16, 16) X(8, 8) X(16, 8) X(32, 8) X(8, 16) X(32, 16) X(16, 32)

static bool raster_shape_supported(int tw, int th) {
#define GS_SHAPE_CASE(a, b) if (tw == a && th == b) return true;
  GS_RASTER_SHAPES(GS_SHAPE_CASE)
#undef GS_SHAPE_CASE
  return false;
}

static gs_status raster_prepare(const gs_projected* proj, const gs_views* views,
                                const gs_tiling* tiling, const uint32_t* ids,
                                const uint32_t* tile_ranges, const float bg[3], const char* who,
                                RasterArgs& a) {
  GS_REQUIRE(proj != nullptr && bg != nullptr, "%s: NULL argument", who);
  gs_status st = check_views(views, tiling, who);
  if (st != GS_OK) return st;
  GS_REQUIRE(raster_shape_supported(tiling->tile_w, tiling->tile_h),
             "%s: tile %dx%d has no rasteriser (16x16, 8x8, 16x8, 32x8, 8x16, 32x16, 16x32)", who,
             tiling->tile_w, tiling->tile_h);
  GS_REQUIRE(tile_ranges != nullptr, "%s: NULL tile_ranges", who);
  GS_REQUIRE(proj->m == 0 || (proj->rec && ids), "%s: NULL rec/ids", who);
  a.rec = proj->rec;
  a.ids = ids;
  a.ranges = tile_ranges;
  a.W = tiling->width;
  a.H = tiling->height;
  a.tiles_x = (int)ceil_div(tiling->width, tiling->tile_w);
  a.tiles_per_slot = a.tiles_x * (int)ceil_div(tiling->height, tiling->tile_h);
  a.n_tiles = (int64_t)a.tiles_per_slot * views->n_slots;
  a.bg[0] = bg[0];
  a.bg[1] = bg[1];
  a.bg[2] = bg[2];
  return GS_OK;
}

}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_raster_fwd(const gs_projected* proj, const gs_views* views, const gs_tiling* tiling,
                        const uint32_t* ids, const uint32_t* tile_ranges, const float bg[3],
                        float* image, float* T_final, int32_t* n_contrib, void* stream) {
  clear_error();
  RasterArgs a;
  gs_status st = raster_prepare(proj, views, tiling, ids, tile_ranges, bg, "gs_raster_fwd", a);
  if (st != GS_OK) return st;
  GS_REQUIRE(image != nullptr, "gs_raster_fwd: NULL image");
  GS_REQUIRE((T_final == nullptr) == (n_contrib == nullptr),
             "gs_raster_fwd: T_final and n_contrib must both be set or both be NULL");
  hipStream_t s = as_stream(stream);
#define GS_FWD_CASE(a_, b_)                                              \
  if (tiling->tile_w == a_ && tiling->tile_h == b_)                      \
    launch_fwd<a_, b_>(a, image, T_final, n_contrib, s);                 \
  else
  GS_RASTER_SHAPES(GS_FWD_CASE) {}
#undef GS_FWD_CASE
  GS_LAUNCH_CHECK("gs_raster_fwd");
  return GS_OK;
}

gs_status gs_raster_bwd(const gs_projected* proj, const gs_views* views, const gs_tiling* tiling,
                        const uint32_t* ids, const uint32_t* tile_ranges, const float bg[3],
                        const float* T_final, const int32_t* n_contrib, const float* d_image,
                        int32_t mode, float* d_rec, void* stream) {
  clear_error();
  RasterArgs a;
  gs_status st = raster_prepare(proj, views, tiling, ids, tile_ranges, bg, "gs_raster_bwd", a);
  if (st != GS_OK) return st;
  GS_REQUIRE(mode == GS_BWD_STORED || mode == GS_BWD_RECOMPUTE, "gs_raster_bwd: bad mode %d",
             mode);
  GS_REQUIRE(d_image && d_rec, "gs_raster_bwd: NULL d_image/d_rec");
  GS_REQUIRE(mode == GS_BWD_RECOMPUTE || (T_final && n_contrib),
             "gs_raster_bwd: STORED mode needs T_final and n_contrib");
  hipStream_t s = as_stream(stream);
#define GS_BWD_CASE(a_, b_)                                                   \
  if (tiling->tile_w == a_ && tiling->tile_h == b_)                           \
    launch_bwd<a_, b_>(a, T_final, n_contrib, d_image, mode, d_rec, s);       \
  else
  GS_RASTER_SHAPES(GS_BWD_CASE) {}
#undef GS_BWD_CASE
  GS_LAUNCH_CHECK("gs_raster_bwd");
  return GS_OK;
}

}  // extern "C"
