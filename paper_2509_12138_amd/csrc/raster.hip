// raster.hip — front-to-back compositing (3D-GS rasteriser that the paper's
// Sec. II "Parallel Training" runs per partition) and its reverse replay.
//
// Layout on gfx950: one wave64 per bin tile.  A 16x16 tile gives each lane 4
// pixels of one column, so every Gaussian staged in LDS is read once per 4
// evaluations and the backward's wave reduction is amortised over 256
// pixels.  Gaussians are staged 64 at a time (one gathered record per lane).
// The forward can also split a tile's pixels over 2 or 4 waves of one
// work-group (each wave walks the whole list for its rows, with its own LDS
// batch): all tiles of a 1080p view are resident at once, so the forward's
// time is set by its longest lists, and more waves per tile shorten them.
// Work-group ids are remapped so that neighbouring tiles run on the same
// XCD and share its L2.
//
// The backward recovers each pixel's transmittance by dividing T_final by
// (1 - alpha) in reverse order (STORED) or first replays the forward for its
// tile (RECOMPUTE).  Per (tile, Gaussian) the 9 gradient components are
// summed over the wave with DPP and added with one FP32 atomic each.
#include <algorithm>

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

// A projected record as three 16-byte words (mean, conic, opacity, rgb).
struct RawSplat {
  float4 a, b, c;
};

__device__ __forceinline__ RawSplat fetch_splat(const float* __restrict__ rec, uint32_t id) {
  const float4* r = reinterpret_cast<const float4*>(rec + (int64_t)id * GS_REC_STRIDE);
  return RawSplat{r[0], r[1], r[2]};
}

__device__ __forceinline__ Splat make_splat(const RawSplat& raw) {
  const float4 a = raw.a, b = raw.b, c = raw.c;
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

__device__ __forceinline__ Splat load_splat(const float* __restrict__ rec, uint32_t id) {
  return make_splat(fetch_splat(rec, id));
}

template <int TW, int TH>
struct TileGeom {
  static constexpr int PX = TW * TH / kRasterWave;      // pixels per lane
  static constexpr int RSTEP = kRasterWave / TW;        // rows between a lane's pixels
  static_assert(TW * TH % kRasterWave == 0 && kRasterWave % TW == 0, "tile shape");
};

// Orders one wave's LDS accesses: the wave's staged batch is private to it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pixel-centre box of the pixels a wave owns (for the entry cull).
struct PixBox {
  float x0, x1, y0, y1;
};

// Forward pass of one tile for one lane's PX pixels (pixel slots q0 + 64 k
// of the tile, slot = row * TW + column), which lie in the wave's box.
// WITH_COLOR=false is the replay used by the backward in RECOMPUTE mode.
// s_splat: this wave's 64-entry LDS batch.
// CHUNKED (with colour) also prepares the chunked backward: boundary c is
// the list position (c+1)*chunk; for each pixel the forward stores at slot c
// of `ck` (ck[c * TW*TH + pixel]) the transmittance T_c there and the colour
// still to come behind it, normalised by T_c:
//   U_c = (sum over later blends of rgb alpha T + bg T_final) / T_c,
// built without cancellation from chunk-local composites (P = prod(1-alpha),
// L = sum rgb alpha T_local over a chunk) by U_c = L_{c+1} + P_{c+1} U_{c+1}
// after the tile is done.
template <int TW, int TH, int PX, bool WITH_COLOR, bool CHUNKED = false>
__device__ __forceinline__ void tile_forward(const float* __restrict__ rec,
                                             const uint32_t* __restrict__ ids, uint32_t start,
                                             uint32_t end, const float fx, const float* fy,
                                             const bool* inside, Splat* s_splat, float* T,
                                             float (*C)[3], int* last, const PixBox& box,
                                             float4* ck = nullptr, int chunk = 0, float bg0 = 0.f,
                                             float bg1 = 0.f, float bg2 = 0.f, int q0 = 0) {
  const int lane = threadIdx.x & (kRasterWave - 1);
  // a pixel that is done (outside the image, or stopped) gets a NaN row
  // coordinate: its falloff exponent is NaN and fails both skip tests, so
  // no separate flag is tested per entry
  float fyk[PX];
  float Tl[PX], Lc[PX][3];
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    T[k] = 1.0f;
    last[k] = 0;
    fyk[k] = inside[k] ? fy[k] : __builtin_nanf("");
    if (WITH_COLOR) C[k][0] = C[k][1] = C[k][2] = 0.0f;
    if (CHUNKED) {
      Tl[k] = 1.0f;
      Lc[k][0] = Lc[k][1] = Lc[k][2] = 0.0f;
    }
  }
  uint32_t reached = 0;     // list entries processed (CHUNKED bookkeeping)
  // the next batch's records and the id of the one after are loaded while a
  // batch is composited, so a batch boundary does not wait on the two
  // dependent loads (id, then record)
  RawSplat nraw{};
  uint32_t nid2 = 0;
  if (start + lane < end) nraw = fetch_splat(rec, ids[start + lane]);
  if (start + kRasterWave + lane < end) nid2 = ids[start + kRasterWave + lane];
  for (uint32_t b0 = start; b0 < end; b0 += kRasterWave) {
    bool lane_done = true;
#pragma unroll
    for (int k = 0; k < PX; ++k) lane_done = lane_done && (fyk[k] != fyk[k]);
    if (__all(lane_done)) break;
    const int n = (int)min((uint32_t)kRasterWave, end - b0);
    const RawSplat raw = nraw;
    const uint32_t nid = nid2;
    if (b0 + kRasterWave + lane < end) nraw = fetch_splat(rec, nid);
    if (b0 + 2 * kRasterWave + lane < end) nid2 = ids[b0 + 2 * kRasterWave + lane];
    wave_sync();
    bool hit = false;
    if (lane < n) {
      const Splat s = make_splat(raw);
      hit = splat_may_hit(s, box.x0, box.x1, box.y0, box.y1);
      s_splat[lane] = s;
    }
    // entries that cannot reach the wave's box are never visited
    uint64_t todo = __ballot(hit);
    const bool hit_any = todo != 0;
    wave_sync();
    // composite entry j of the batch (skip-test words g = mx, my, A, B and
    // h = C, thr already read)
    auto composite = [&](const float4& g, const float2& h, int j) {
      Splat sp;
      sp.mx = g.x;
      sp.my = g.y;
      sp.A = g.z;
      sp.B = g.w;
      sp.C = h.x;
      sp.thr = h.y;
      const float dx = __fsub_rn(fx, sp.mx);
      float p2[PX];
      splat_p2_column<PX>(sp, dx, fyk, p2);
      bool pass[PX], any = false;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        pass[k] = splat_pass(sp, p2[k]);
        any = any || pass[k];
      }
      if (!__any(any)) return;
      const float4 col = *reinterpret_cast<const float4*>(&s_splat[j].o);   // o, r, g, b
      const int pos = (int)(b0 - start) + j + 1;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        if (!pass[k]) continue;
        const float alpha = fminf(kAlphaMax, col.x * splat_gauss(p2[k]));
        const float Tn = T[k] * (1.0f - alpha);
        const bool stop = Tn < kTMin;
        fyk[k] = stop ? __builtin_nanf("") : fyk[k];
        if (stop) continue;
        if (WITH_COLOR) {
          const float w = alpha * T[k];
          C[k][0] = fmaf(col.y, w, C[k][0]);
          C[k][1] = fmaf(col.z, w, C[k][1]);
          C[k][2] = fmaf(col.w, w, C[k][2]);
        }
        if (CHUNKED) {
          const float wl = alpha * Tl[k];
          Lc[k][0] = fmaf(col.y, wl, Lc[k][0]);
          Lc[k][1] = fmaf(col.z, wl, Lc[k][1]);
          Lc[k][2] = fmaf(col.w, wl, Lc[k][2]);
          Tl[k] = Tl[k] * (1.0f - alpha);
        }
        T[k] = Tn;
        last[k] = pos;
      }
    };
    // the skip-test words of the next entry are read from LDS while the
    // current one is composited; two register sets alternate
    if (hit_any) {
      int ja = (int)__builtin_ctzll(todo);
      todo &= todo - 1;
      float4 ga = *reinterpret_cast<const float4*>(&s_splat[ja]);     // mx, my, A, B
      float2 ha = *reinterpret_cast<const float2*>(&s_splat[ja].C);   // C, thr
      for (;;) {
        const bool more_a = todo != 0;
        const int jb = more_a ? (int)__builtin_ctzll(todo) : ja;
        const float4 gb = *reinterpret_cast<const float4*>(&s_splat[jb]);
        const float2 hb = *reinterpret_cast<const float2*>(&s_splat[jb].C);
        todo &= todo - 1;
        composite(ga, ha, ja);
        if (!more_a) break;
        const bool more_b = todo != 0;
        ja = more_b ? (int)__builtin_ctzll(todo) : jb;
        ga = *reinterpret_cast<const float4*>(&s_splat[ja]);
        ha = *reinterpret_cast<const float2*>(&s_splat[ja].C);
        todo &= todo - 1;
        composite(gb, hb, jb);
        if (!more_b) break;
      }
    }
    if (CHUNKED) {
      reached = b0 + (uint32_t)n - start;
      if (reached % (uint32_t)chunk == 0) {
        // chunk ce just ended: its local composite goes to slot ce-1
        const int ce = (int)(reached / chunk) - 1;
        if (ce >= 1) {
          float4* dst = ck + (int64_t)(ce - 1) * (TW * TH);
#pragma unroll
          for (int k = 0; k < PX; ++k)
            dst[q0 + k * kRasterWave] = make_float4(Tl[k], Lc[k][0], Lc[k][1], Lc[k][2]);
        }
#pragma unroll
        for (int k = 0; k < PX; ++k) {
          Tl[k] = 1.0f;
          Lc[k][0] = Lc[k][1] = Lc[k][2] = 0.0f;
        }
      }
    }
  }
  if (CHUNKED && reached > 0) {
    // the partly processed last chunk (if any) and the reverse recursion
    int clast = (int)((reached - 1) / chunk);          // last chunk touched
    if (reached % (uint32_t)chunk != 0 && clast >= 1) {
      float4* dst = ck + (int64_t)(clast - 1) * (TW * TH);
#pragma unroll
      for (int k = 0; k < PX; ++k)
        dst[q0 + k * kRasterWave] = make_float4(Tl[k], Lc[k][0], Lc[k][1], Lc[k][2]);
    }
    float Tn[PX], U[PX][3];
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      Tn[k] = T[k];
      U[k][0] = bg0;
      U[k][1] = bg1;
      U[k][2] = bg2;
    }
    for (int c = clast - 1; c >= 0; --c) {
      float4* slot = ck + (int64_t)c * (TW * TH);
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        const int q = q0 + k * kRasterWave;
        const float4 pl = slot[q];                          // (P, L) of chunk c+1
        const float Te = Tn[k] / pl.x;
        U[k][0] = fmaf(pl.x, U[k][0], pl.y);
        U[k][1] = fmaf(pl.x, U[k][1], pl.z);
        U[k][2] = fmaf(pl.x, U[k][2], pl.w);
        slot[q] = make_float4(Te, U[k][0], U[k][1], U[k][2]);
        Tn[k] = Te;
      }
    }
  }
}

// Per-call arguments shared by the forward and backward rasterisers.
struct RasterDev {
  const float* rec;
  const uint32_t* ids;
  const uint32_t* ranges;
  int W, H, tiles_x, tiles_per_slot;
  int64_t n_tiles;
  float bg0, bg1, bg2;
  // deterministic backward (NULL dup_grads: atomics into d_rec): emit[q]
  // is the emission index (gradient slot) of sorted entry q
  const uint32_t* emit;
  float* dup_grads;
  int64_t dup_cap;
};

// Deterministic mode: zero the gradient slots of list indices [lo, hi) of a
// tile (entries no pixel reaches), one entry per lane.
__device__ __forceinline__ void zero_dup_slots(const RasterDev& a, uint32_t start, int lo, int hi) {
  const int lane = threadIdx.x & (kRasterWave - 1);
  for (int q = lo + lane; q < hi; q += kRasterWave) {
    const uint32_t e = a.emit[start + q];
    if ((int64_t)e >= a.dup_cap) continue;
    float* g = a.dup_grads + (int64_t)e * GS_DREC_STRIDE;
#pragma unroll
    for (int c = 0; c < GS_DREC_STRIDE; ++c) g[c] = 0.0f;
  }
}

// Which tile a work-group processes: default XCD-aware order, a precomputed
// (longest-first) order, or a persistent grid pulling from an atomic queue.
struct TileSched {
  const uint32_t* order;   // NULL: XCD-aware default order
  uint32_t* queue;         // non-NULL: persistent launch, items pulled atomically
};

// Chunked backward: every tile list is cut into `chunk`-entry work items;
// offset[t] is the first item of tile t (offset[n_tiles] = item count),
// items[i] the tile of item i; ck the forward checkpoints (T_c, U_c), one
// TW*TH float4 block per item.
struct ChunkDev {
  int chunk;
  const uint32_t* offset;
  const uint32_t* items;
  float4* ck;
};

template <typename F>
__device__ __forceinline__ void for_each_tile(const TileSched& sch, int64_t n_tiles, F&& body) {
  if (sch.queue) {
    for (;;) {
      uint32_t item = 0;
      if (threadIdx.x == 0) item = atomicAdd(sch.queue, 1u);
      item = __builtin_amdgcn_readfirstlane(item);
      if ((int64_t)item >= n_tiles) break;
      body((int64_t)(sch.order ? sch.order[item] : item));
    }
  } else {
    const int64_t tile = sch.order ? ((int64_t)blockIdx.x < n_tiles ? (int64_t)sch.order[blockIdx.x] : n_tiles)
                                   : tile_of_block(n_tiles);
    if (tile < n_tiles) body(tile);
  }
}

// Forward of one tile by wave w = threadIdx.x / 64 of NW; PX = TW TH / (64 NW)
// pixels per lane.  With one pixel per lane the wave owns an 8x8 block of
// the tile (blocks in row-major order), the most compact box for the entry
// cull; otherwise the rows ty TH + (w PX + k) RSTEP + lane / TW of column
// lane % TW.
template <int TW, int TH, int NW>
__device__ __forceinline__ void fwd_tile(const RasterDev& a, const ChunkDev& ch, int64_t tile,
                                         Splat* s_splat, float* __restrict__ image,
                                         float* __restrict__ T_final,
                                         int32_t* __restrict__ n_contrib) {
  constexpr int PX = TileGeom<TW, TH>::PX / NW, RSTEP = TileGeom<TW, TH>::RSTEP;
  static_assert(PX >= 1 && TileGeom<TW, TH>::PX % NW == 0, "waves per tile");
  constexpr bool kBlock8 = PX == 1 && TW % 8 == 0 && TH % 8 == 0;
  const int W = a.W, H = a.H;
  const int slot = (int)(tile / a.tiles_per_slot);
  const int t = (int)(tile - (int64_t)slot * a.tiles_per_slot);
  const int ty = t / a.tiles_x, tx = t - ty * a.tiles_x;
  const int lane = threadIdx.x & (kRasterWave - 1);
  const int w = threadIdx.x / kRasterWave;
  // the lane's column and first row inside the tile, and the wave's box
  const int lx = kBlock8 ? (w % (TW / 8)) * 8 + lane % 8 : lane % TW;
  const int ly0 = kBlock8 ? (w / (TW / 8)) * 8 + lane / 8 : lane / TW + w * PX * RSTEP;
  const int bxo = kBlock8 ? (w % (TW / 8)) * 8 : 0, bw = kBlock8 ? 8 : TW;
  const int byo = kBlock8 ? (w / (TW / 8)) * 8 : w * PX * RSTEP, bh = kBlock8 ? 8 : PX * RSTEP;
  const PixBox box{(float)(tx * TW + bxo) + 0.5f, (float)(tx * TW + bxo + bw - 1) + 0.5f,
                   (float)(ty * TH + byo) + 0.5f, (float)(ty * TH + byo + bh - 1) + 0.5f};
  const int px = tx * TW + lx;
  const int py0 = ty * TH + ly0;
  const float fx = (float)px + 0.5f;
  float fy[PX];
  bool inside[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    const int py = py0 + k * RSTEP;
    fy[k] = (float)py + 0.5f;
    inside[k] = (px < W) && (py < H);
  }
  const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
  float T[PX], C[PX][3];
  int last[PX];
  if (ch.ck) {
    float4* ck = ch.ck + (int64_t)ch.offset[tile] * (TW * TH);
    tile_forward<TW, TH, PX, true, true>(a.rec, a.ids, start, end, fx, fy, inside, s_splat, T, C,
                                         last, box, ck, ch.chunk, a.bg0, a.bg1, a.bg2,
                                         ly0 * TW + lx);
  } else {
    tile_forward<TW, TH, PX, true>(a.rec, a.ids, start, end, fx, fy, inside, s_splat, T, C, last,
                                   box);
  }
  const int64_t HW = (int64_t)H * W;
  float* img = image + (int64_t)slot * 3 * HW;
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    if (!inside[k]) continue;
    const int64_t o = (int64_t)(py0 + k * RSTEP) * W + px;
    img[o] = C[k][0] + T[k] * a.bg0;
    img[HW + o] = C[k][1] + T[k] * a.bg1;
    img[2 * HW + o] = C[k][2] + T[k] * a.bg2;
    if (T_final) T_final[(int64_t)slot * HW + o] = T[k];
    if (n_contrib) n_contrib[(int64_t)slot * HW + o] = last[k];
  }
}

// Waves per SIMD that two 16x16 rasterisers are compiled for: 7 caps them at
// 72 VGPRs (80 unconstrained, i.e. 6 waves); the few spilled registers are
// reloaded at most once per 64-entry batch, never per entry.  Measured 2%
// faster for the forward on four waves (one pixel per lane) and for the
// chunked backward.  1 leaves the compiler free (other shapes spill heavily
// under the cap).
template <int TW, int TH, int NW>
constexpr int kFwdWavesPerEU = (TW == 16 && TH == 16 && NW == 4) ? 7 : 1;
template <int TW, int TH>
constexpr int kBwdWavesPerEU = (TW == 16 && TH == 16) ? 7 : 1;

template <int TW, int TH, int NW>
__global__ __launch_bounds__(kRasterWave * NW)
__attribute__((amdgpu_waves_per_eu(kFwdWavesPerEU<TW, TH, NW>)))
void k_raster_fwd(RasterDev a, TileSched sch,
                                                                 ChunkDev ch,
                                                                 float* __restrict__ image,
                                                                 float* __restrict__ T_final,
                                                                 int32_t* __restrict__ n_contrib) {
  __shared__ Splat s_splat[kRasterWave * NW];
  // wave-uniform base (scalar), so per-entry LDS addresses stay scalar too
  Splat* mine = s_splat + __builtin_amdgcn_readfirstlane(threadIdx.x / kRasterWave) * kRasterWave;
  for_each_tile(sch, a.n_tiles, [&](int64_t tile) {
    fwd_tile<TW, TH, NW>(a, ch, tile, mine, image, T_final, n_contrib);
  });
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
  return v;
}

// Reduce-scatter of the 9 gradient components of one list entry over the
// wave.  Stage 1 pairs lanes l and l ^ 32 with v_permlane32_swap, stage 2
// pairs l and l ^ 16 with v_permlane16_swap: swapping the halves of two
// component registers and adding gives, in every lane, one component summed
// over the lane pair, with no selects.  Stages 3-4 (partners l ^ 8 via
// row_ror:8, and l <-> 7 - (l mod 8) via row_half_mirror) keep one of two
// components per lane, and two quad_perm steps finish the sum.  Afterwards
// each group of 4 lanes holds the wave total of one component: 9 of the 16
// groups hold one each, and lanes 4k issue a single 9-lane atomic.
struct Scatter9 {
  int slot;       // component this lane's group holds (-1: none)
  float scale;    // its constant factor in d_rec
};

__device__ __forceinline__ Scatter9 scatter9_setup() {
  const int lane = threadIdx.x & (kRasterWave - 1);
  // which operand a lane keeps after each swap: push 0 / 1 through it
  const auto p32 = __builtin_amdgcn_permlane32_swap(0u, 1u, false, false);
  const auto p16 = __builtin_amdgcn_permlane16_swap(0u, 1u, false, false);
  const bool first32 = p32[0] == 0u, first16 = p16[0] == 0u;
  const int b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1;
  const int u = b2 == 0 ? (b3 ? 2 : 0) : (b3 ? -1 : 1);           // after stage 2
  const int w = u < 0 ? -1 : (first16 ? u : (u + 3 <= 4 ? u + 3 : -1));   // after stage 1
  const int v = w < 0 ? -1 : (first32 ? w : (w + 5 <= 8 ? w + 5 : -1));  // component
  // d mean2d (x2) carry -ln2, d Q11 and d Q22 -1/2, d Q12 -1 (log2-scaled
  // falloff); opacity and colour 1
  const float sc[9] = {-kLn2, -kLn2, -0.5f, -1.0f, -0.5f, 1.0f, 1.0f, 1.0f, 1.0f};
  Scatter9 r;
  r.slot = ((lane & 3) == 0) ? v : -1;
  r.scale = v >= 0 ? sc[v] : 0.0f;
  return r;
}

__device__ __forceinline__ float swap_add32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float swap_add16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// v[0..8]: this lane's partial components; returns the wave total of the
// component named by scatter9_setup().slot (valid in every lane of its group).
__device__ __forceinline__ float reduce_scatter9(const float (&v)[9]) {
  const int lane = threadIdx.x & (kRasterWave - 1);
  // stage 1: 9 -> 5 (pairs (i, i + 5), v[9] = 0)
  const float w0 = swap_add32(v[0], v[5]);
  const float w1 = swap_add32(v[1], v[6]);
  const float w2 = swap_add32(v[2], v[7]);
  const float w3 = swap_add32(v[3], v[8]);
  const float w4 = swap_add32(v[4], 0.0f);
  // stage 2: 5 -> 3 (pairs (i, i + 3), w[5] = 0)
  const float u0 = swap_add16(w0, w3);
  const float u1 = swap_add16(w1, w4);
  const float u2 = swap_add16(w2, 0.0f);
  // stage 3: 3 -> 2 across l ^ 8: bit 3 clear keeps (u0, u1), set keeps (u2, -)
  const bool b3 = (lane >> 3) & 1;
  const float k0 = b3 ? u2 : u0, s0 = b3 ? u0 : u2;
  const float k1 = b3 ? 0.0f : u1, s1 = b3 ? u1 : 0.0f;
  const float t0 = k0 + dpp_f<kDppRowRor8>(s0);
  const float t1 = k1 + dpp_f<kDppRowRor8>(s1);
  // stage 4: 2 -> 1 across l <-> 7 - (l mod 8): bit 2 clear keeps t0
  const bool b2 = (lane >> 2) & 1;
  const float kk = b2 ? t1 : t0, ss = b2 ? t0 : t1;
  float z = kk + dpp_f<kDppRowHalfMirror>(ss);
  // stages 5-6: sum over the quad
  z += dpp_f<kDppQuadSwap1>(z);
  z += dpp_f<kDppQuadSwap2>(z);
  return z;
}

// Reverse replay of list positions (lo, hi] of one tile (entries start+lo ..
// start+hi-1, last first).  Per pixel k on entry: T[k] = transmittance after
// position hi, dIacc[k] = dI . (colour blended behind position hi + bg T_final).
// With a.dup_grads the entry's components go to its emission slot (s_id then
// holds the slot index), else they are added atomically to d_rec.
template <int TW, int TH>
__device__ __forceinline__ void reverse_pass(const RasterDev& a, uint32_t start, int lo, int hi,
                                             const float fx, const float* fy, const int* last,
                                             float* T, float (*dI)[3], float* dIacc,
                                             Splat* s_splat, uint32_t* s_id,
                                             float* __restrict__ d_rec, const Scatter9& red) {
  constexpr int PX = TileGeom<TW, TH>::PX;
  const int lane = threadIdx.x;
  const bool det = a.dup_grads != nullptr;
  float* const gbase = det ? a.dup_grads : d_rec;
  // the tile's pixel box
  const float bx0 = fx - (float)(lane % TW), by0 = fy[0] - (float)(lane / TW);
  const float bx1 = bx0 + (float)(TW - 1), by1 = by0 + (float)(TH - 1);
  for (int top = hi; top > lo; top -= kRasterWave) {
    const int bot = max(lo, top - kRasterWave);
    const int n = top - bot;
    __syncthreads();
    bool hit = false;
    if (lane < n) {
      const uint32_t id = a.ids[start + bot + lane];
      const uint32_t e = det ? a.emit[start + bot + lane] : id;
      s_id[lane] = e;
      const Splat s = load_splat(a.rec, id);
      hit = splat_may_hit(s, bx0, bx1, by0, by1);
      s_splat[lane] = s;
      // an entry that cannot reach the tile gets zero gradients
      if (!hit && det && (int64_t)e < a.dup_cap) {
        float* g = gbase + (int64_t)e * GS_DREC_STRIDE;
#pragma unroll
        for (int c = 0; c < GS_DREC_STRIDE; ++c) g[c] = 0.0f;
      }
    }
    uint64_t todo = __ballot(hit);
    __syncthreads();
    while (todo) {
      const int j = 63 - (int)__builtin_clzll(todo);         // last first
      todo &= ~(1ull << j);
      const Splat sp = s_splat[j];
      const int pos = bot + j + 1;
      const float dx = __fsub_rn(fx, sp.mx);
      float p2[PX];
      splat_p2_column<PX>(sp, dx, fy, p2);
      bool pass[PX], any = false;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        pass[k] = (pos <= last[k]) && splat_pass(sp, p2[k]);
        any = any || pass[k];
      }
      if (!__any(any)) {
        if (det && red.slot >= 0 && (int64_t)s_id[j] < a.dup_cap)
          gbase[(int64_t)s_id[j] * GS_DREC_STRIDE + red.slot] = 0.0f;
        continue;
      }
      // per-lane sums over the lane's pixels; the geometric gradients of the
      // lane follow from sG = sum G, sGdy = sum G dy, sGdy2 = sum G dy^2 with
      // G = dL/d(power) (dx is shared by the lane's column)
      float sG = 0.f, sGdy = 0.f, sGdy2 = 0.f, so = 0.f, sr = 0.f, sg = 0.f, sb = 0.f;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        if (!pass[k]) continue;
        const float gss = splat_gauss(p2[k]);
        const float aa = sp.o * gss;
        const float alpha = fminf(kAlphaMax, aa);
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
        if (aa < kAlphaMax) {
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
      // geometric gradients of the lane (constant factors applied per
      // component after the reduction)
      const float comp[9] = {fmaf(2.0f * sp.A * dx, sG, sp.B * sGdy),   // d mx / -ln2
                             fmaf(2.0f * sp.C, sGdy, bdx * sG),         // d my / -ln2
                             dx * dx * sG,                              // d Q11 / -1/2
                             dx * sGdy,                                 // d Q12 / -1
                             sGdy2,                                     // d Q22 / -1/2
                             so, sr, sg, sb};
      const float tot = reduce_scatter9(comp);
      if (red.slot >= 0) {
        float* dst = gbase + (int64_t)s_id[j] * GS_DREC_STRIDE + red.slot;
        if (!det) atomicAdd(dst, red.scale * tot);
        else if ((int64_t)s_id[j] < a.dup_cap) *dst = red.scale * tot;
      }
    }
  }
}

// Pixel geometry of one tile for the calling lane.
template <int TW, int TH>
struct LanePixels {
  static constexpr int PX = TileGeom<TW, TH>::PX, RSTEP = TileGeom<TW, TH>::RSTEP;
  int slot, px, py0, tx, ty;
  float fx, fy[PX];
  bool inside[PX];
  __device__ __forceinline__ LanePixels(const RasterDev& a, int64_t tile) {
    slot = (int)(tile / a.tiles_per_slot);
    const int t = (int)(tile - (int64_t)slot * a.tiles_per_slot);
    ty = t / a.tiles_x;
    tx = t - ty * a.tiles_x;
    const int lane = threadIdx.x;
    px = tx * TW + (lane % TW);
    py0 = ty * TH + lane / TW;
    fx = (float)px + 0.5f;
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      const int py = py0 + k * RSTEP;
      fy[k] = (float)py + 0.5f;
      inside[k] = (px < a.W) && (py < a.H);
    }
  }
  __device__ __forceinline__ int64_t offset(const RasterDev& a, int k) const {
    return (int64_t)(py0 + k * RSTEP) * a.W + px;
  }
};

template <int TW, int TH, bool RECOMPUTE>
__device__ __forceinline__ void bwd_tile(const RasterDev& a, int64_t tile, Splat* s_splat,
                                         uint32_t* s_id, const float* __restrict__ T_final,
                                         const int32_t* __restrict__ n_contrib,
                                         const float* __restrict__ d_image,
                                         float* __restrict__ d_rec) {
  constexpr int PX = TileGeom<TW, TH>::PX;
  const LanePixels<TW, TH> L(a, tile);
  const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
  if (start >= end) return;
  const int64_t HW = (int64_t)a.H * a.W;
  float T[PX];
  int last[PX];
  if (RECOMPUTE) {
    const PixBox box{(float)(L.tx * TW) + 0.5f, (float)(L.tx * TW + TW - 1) + 0.5f,
                     (float)(L.ty * TH) + 0.5f, (float)(L.ty * TH + TH - 1) + 0.5f};
    tile_forward<TW, TH, PX, false>(a.rec, a.ids, start, end, L.fx, L.fy, L.inside, s_splat, T,
                                    nullptr, last, box);
  } else {
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      const int64_t o = (int64_t)L.slot * HW + L.offset(a, k);
      T[k] = L.inside[k] ? T_final[o] : 1.0f;
      last[k] = L.inside[k] ? n_contrib[o] : 0;
    }
  }
  // dIacc = dI . (sum of the colour blended behind + bg T_final), per pixel
  float dI[PX][3], dIacc[PX];
  const float* dimg = d_image + (int64_t)L.slot * 3 * HW;
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    const int64_t o = L.offset(a, k);
    dI[k][0] = L.inside[k] ? dimg[o] : 0.0f;
    dI[k][1] = L.inside[k] ? dimg[HW + o] : 0.0f;
    dI[k][2] = L.inside[k] ? dimg[2 * HW + o] : 0.0f;
    dIacc[k] = T[k] * (dI[k][0] * a.bg0 + dI[k][1] * a.bg1 + dI[k][2] * a.bg2);
    // a pixel with a zero image gradient (a masked one) adds exactly zero
    // to every gradient: it takes no part in the reverse pass
    if (dI[k][0] == 0.0f && dI[k][1] == 0.0f && dI[k][2] == 0.0f) last[k] = 0;
  }
  int lmax = 0;
#pragma unroll
  for (int k = 0; k < PX; ++k) lmax = max(lmax, last[k]);
  lmax = min(wave_max_int(lmax), (int)(end - start));
  reverse_pass<TW, TH>(a, start, 0, lmax, L.fx, L.fy, last, T, dI, dIacc, s_splat, s_id, d_rec,
                       scatter9_setup());
  if (a.dup_grads) zero_dup_slots(a, start, lmax, (int)(end - start));
}

template <int TW, int TH, bool RECOMPUTE>
__global__ __launch_bounds__(kRasterWave) void k_raster_bwd(RasterDev a, TileSched sch,
                                                            const float* __restrict__ T_final,
                                                            const int32_t* __restrict__ n_contrib,
                                                            const float* __restrict__ d_image,
                                                            float* __restrict__ d_rec) {
  __shared__ Splat s_splat[kRasterWave];
  __shared__ uint32_t s_id[kRasterWave];
  for_each_tile(sch, a.n_tiles, [&](int64_t tile) {
    bwd_tile<TW, TH, RECOMPUTE>(a, tile, s_splat, s_id, T_final, n_contrib, d_image, d_rec);
  });
}

// Chunked backward: one work-group per (tile, chunk) item.  Chunk c covers
// list positions (c*chunk, min((c+1)*chunk, len)]; the state after its last
// position is the forward's final state for pixels whose last blended entry
// lies at or before it, else the checkpoint (T_c, U_c) the forward stored
// there (dI . acc = T_c dI . U_c).
template <int TW, int TH>
__global__ __launch_bounds__(kRasterWave)
__attribute__((amdgpu_waves_per_eu(kBwdWavesPerEU<TW, TH>)))
void k_raster_bwd_chunked(
    RasterDev a, ChunkDev ch, const float* __restrict__ T_final,
    const int32_t* __restrict__ n_contrib, const float* __restrict__ d_image,
    float* __restrict__ d_rec) {
  constexpr int PX = TileGeom<TW, TH>::PX;
  __shared__ Splat s_splat[kRasterWave];
  __shared__ uint32_t s_id[kRasterWave];
  const uint32_t item = blockIdx.x;
  if (item >= ch.offset[a.n_tiles]) return;
  const int64_t tile = ch.items[item];
  const int c = (int)(item - ch.offset[tile]);
  const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
  const int len = (int)(end - start);
  const int lo = c * ch.chunk, hi_pos = min(lo + ch.chunk, len);
  const LanePixels<TW, TH> L(a, tile);
  const int64_t HW = (int64_t)a.H * a.W;
  int last[PX];
  float T[PX], dI[PX][3], dIacc[PX];
  const float* dimg = d_image + (int64_t)L.slot * 3 * HW;
  int lmax = 0;
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    const int64_t o = L.offset(a, k);
    last[k] = L.inside[k] ? n_contrib[(int64_t)L.slot * HW + o] : 0;
    dI[k][0] = L.inside[k] ? dimg[o] : 0.0f;
    dI[k][1] = L.inside[k] ? dimg[HW + o] : 0.0f;
    dI[k][2] = L.inside[k] ? dimg[2 * HW + o] : 0.0f;
    // a pixel with a zero image gradient (a masked one) adds exactly zero
    // to every gradient: it takes no part in the reverse pass
    if (dI[k][0] == 0.0f && dI[k][1] == 0.0f && dI[k][2] == 0.0f) last[k] = 0;
    lmax = max(lmax, last[k]);
  }
  const int hi = min(wave_max_int(lmax), hi_pos);
  if (hi <= lo) {
    if (a.dup_grads) zero_dup_slots(a, start, lo, hi_pos);
    return;
  }
  const float4* ck = ch.ck + ((int64_t)ch.offset[tile] + c) * (TW * TH);
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    const int64_t o = L.offset(a, k);
    if (!L.inside[k] || last[k] <= hi_pos) {
      // nothing blended after this chunk: final state, I - C_final = bg T_final
      T[k] = L.inside[k] ? T_final[(int64_t)L.slot * HW + o] : 1.0f;
      dIacc[k] = T[k] * (dI[k][0] * a.bg0 + dI[k][1] * a.bg1 + dI[k][2] * a.bg2);
    } else {
      const float4 s = ck[threadIdx.x + k * kRasterWave];   // (T_c, U_c)
      T[k] = s.x;
      dIacc[k] = s.x * (dI[k][0] * s.y + dI[k][1] * s.z + dI[k][2] * s.w);
    }
  }
  reverse_pass<TW, TH>(a, start, lo, hi, L.fx, L.fy, last, T, dI, dIacc, s_splat, s_id, d_rec,
                       scatter9_setup());
  if (a.dup_grads) zero_dup_slots(a, start, hi, hi_pos);
}

// ---------------------------------------------------------------- quadrant groups

// Reduce-scatter of the 9 gradient components over each 16-lane row of the
// wave (the rows work on different entries): row_ror:8 pairs l and l ^ 8,
// row_half_mirror l and 7 - l, and two quad_perm steps l ^ 2 and l ^ 1;
// each step keeps, per lane, about half of the components summed over the
// lane pair.  Afterwards 9 lanes of every row hold the row total of one
// component each (row_slot9 names which).
template <int CTRL>
__device__ __forceinline__ float keep_add(bool hi, float lo_v, float hi_v) {
  const float mine = hi ? hi_v : lo_v, other = hi ? lo_v : hi_v;
  return mine + dpp_f<CTRL>(other);
}

__device__ __forceinline__ float reduce_scatter9_row(const float (&v)[9]) {
  const int l = threadIdx.x & 15;
  const bool b3 = (l >> 3) & 1, b2 = (l >> 2) & 1, b1 = (l >> 1) & 1, b0 = l & 1;
  // 9 -> 5: bit 3 clear keeps 0..4, set keeps 5..8
  const float w0 = keep_add<kDppRowRor8>(b3, v[0], v[5]);
  const float w1 = keep_add<kDppRowRor8>(b3, v[1], v[6]);
  const float w2 = keep_add<kDppRowRor8>(b3, v[2], v[7]);
  const float w3 = keep_add<kDppRowRor8>(b3, v[3], v[8]);
  const float w4 = keep_add<kDppRowRor8>(b3, v[4], 0.0f);
  // 5 -> 3: bit 2 clear keeps w0..w2, set keeps w3, w4
  const float u0 = keep_add<kDppRowHalfMirror>(b2, w0, w3);
  const float u1 = keep_add<kDppRowHalfMirror>(b2, w1, w4);
  const float u2 = keep_add<kDppRowHalfMirror>(b2, w2, 0.0f);
  // 3 -> 2: bit 1 clear keeps u0, u1, set keeps u2
  const float t0 = keep_add<kDppQuadSwap2>(b1, u0, u2);
  const float t1 = keep_add<kDppQuadSwap2>(b1, u1, 0.0f);
  // 2 -> 1: bit 0 clear keeps t0, set keeps t1
  return keep_add<kDppQuadSwap1>(b0, t0, t1);
}

// Component (0-8) whose row total reduce_scatter9_row leaves in row lane l,
// or -1.
__device__ __forceinline__ int row_slot9(int l) {
  const int b3 = (l >> 3) & 1, b2 = (l >> 2) & 1, b1 = (l >> 1) & 1, b0 = l & 1;
  int L1[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) L1[k] = b3 ? (k < 4 ? 5 + k : -1) : k;
  const int L2[3] = {b2 ? L1[3] : L1[0], b2 ? L1[4] : L1[1], b2 ? -1 : L1[2]};
  const int L3[2] = {b1 ? L2[2] : L2[0], b1 ? -1 : L2[1]};
  return b0 ? L3[1] : L3[0];
}

// Chunked backward on quadrant lane groups: row q of the wave (lanes 16q ..
// 16q+15) owns the (TW/2) x (TH/2) quadrant (q mod 2, q / 2) of the tile,
// PXQ pixels of one column per lane (column r mod QW, rows r / QW + k RS),
// and walks in reverse list order only the entries of the chunk that may
// reach its quadrant (the staging cull against each quadrant's box); the
// four rows work on different entries at once, and an entry's 9 components
// are reduced over its row and added atomically.  Splats that reach part of
// a tile then cost their fixed share (the reduction) on 16 lanes instead of
// 64.  Per pixel the arithmetic and the skip and stop decisions are those of
// reverse_pass.  Atomic gradient sums only.
template <int TW, int TH>
__global__ __launch_bounds__(kRasterWave) void k_raster_bwd_chunked_q(
    RasterDev a, ChunkDev ch, const float* __restrict__ T_final,
    const int32_t* __restrict__ n_contrib, const float* __restrict__ d_image,
    float* __restrict__ d_rec) {
  constexpr int QW = TW / 2, QH = TH / 2, PXQ = QW * QH / 16, RS = 16 / QW;
  static_assert(QW * QH % 16 == 0 && 16 % QW == 0, "quadrant shape");
  __shared__ Splat s_splat[kRasterWave];
  __shared__ uint32_t s_id[kRasterWave];
  const uint32_t item = blockIdx.x;
  if (item >= ch.offset[a.n_tiles]) return;
  const int64_t tile = ch.items[item];
  const int c = (int)(item - ch.offset[tile]);
  const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
  const int len = (int)(end - start);
  const int lo = c * ch.chunk, hi_pos = min(lo + ch.chunk, len);
  const int lane = threadIdx.x, q = lane >> 4, r = lane & 15;
  const int slot = (int)(tile / a.tiles_per_slot);
  const int tt = (int)(tile - (int64_t)slot * a.tiles_per_slot);
  const int ty = tt / a.tiles_x, tx = tt - ty * a.tiles_x;
  const int lx = (q & 1) * QW + r % QW, ly0 = (q >> 1) * QH + r / QW;   // in the tile
  const int px = tx * TW + lx;
  const float fx = (float)px + 0.5f;
  const int64_t HW = (int64_t)a.H * a.W;
  const float* dimg = d_image + (int64_t)slot * 3 * HW;
  float fy[PXQ], T[PXQ], dI[PXQ][3], dIacc[PXQ];
  int last[PXQ];
  bool inside[PXQ];
  int lmax = 0;
#pragma unroll
  for (int k = 0; k < PXQ; ++k) {
    const int py = ty * TH + ly0 + k * RS;
    fy[k] = (float)py + 0.5f;
    inside[k] = (px < a.W) && (py < a.H);
    const int64_t o = (int64_t)py * a.W + px;
    last[k] = inside[k] ? n_contrib[(int64_t)slot * HW + o] : 0;
    dI[k][0] = inside[k] ? dimg[o] : 0.0f;
    dI[k][1] = inside[k] ? dimg[HW + o] : 0.0f;
    dI[k][2] = inside[k] ? dimg[2 * HW + o] : 0.0f;
    // a pixel with a zero image gradient (a masked one) adds exactly zero
    if (dI[k][0] == 0.0f && dI[k][1] == 0.0f && dI[k][2] == 0.0f) last[k] = 0;
    lmax = max(lmax, last[k]);
  }
  const int hi = min(wave_max_int(lmax), hi_pos);
  if (hi <= lo) return;
  const float4* ck = ch.ck + ((int64_t)ch.offset[tile] + c) * (TW * TH);
#pragma unroll
  for (int k = 0; k < PXQ; ++k) {
    if (!inside[k] || last[k] <= hi_pos) {
      // nothing blended after this chunk: final state, I - C_final = bg T_final
      const int64_t o = (int64_t)(ty * TH + ly0 + k * RS) * a.W + px;
      T[k] = inside[k] ? T_final[(int64_t)slot * HW + o] : 1.0f;
      dIacc[k] = T[k] * (dI[k][0] * a.bg0 + dI[k][1] * a.bg1 + dI[k][2] * a.bg2);
    } else {
      const float4 sck = ck[(ly0 + k * RS) * TW + lx];   // (T_c, U_c)
      T[k] = sck.x;
      dIacc[k] = sck.x * (dI[k][0] * sck.y + dI[k][1] * sck.z + dI[k][2] * sck.w);
    }
  }
  const int rslot = row_slot9(r);
  // d mean2d (x2) carry -ln2, d Q11 and d Q22 -1/2, d Q12 -1 (log2-scaled
  // falloff); opacity and colour 1
  const float sc[9] = {-kLn2, -kLn2, -0.5f, -1.0f, -0.5f, 1.0f, 1.0f, 1.0f, 1.0f};
  const float rscale = rslot >= 0 ? sc[rslot] : 0.0f;
  const float qx0 = (float)(tx * TW) + 0.5f, qy0 = (float)(ty * TH) + 0.5f;
  for (int top = hi; top > lo; top -= kRasterWave) {
    const int bot = max(lo, top - kRasterWave);
    const int n = top - bot;
    wave_sync();
    uint32_t qm = 0;
    if (lane < n) {
      const uint32_t id = a.ids[start + bot + lane];
      s_id[lane] = id;
      const Splat sp = load_splat(a.rec, id);
      s_splat[lane] = sp;
      // which quadrants' pixel-centre boxes the entry may reach
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float x0 = qx0 + (float)((g & 1) * QW), y0 = qy0 + (float)((g >> 1) * QH);
        if (splat_may_hit(sp, x0, x0 + (float)(QW - 1), y0, y0 + (float)(QH - 1)))
          qm |= 1u << g;
      }
    }
    const uint64_t m0 = __ballot(qm & 1u), m1 = __ballot(qm & 2u), m2 = __ballot(qm & 4u),
                   m3 = __ballot(qm & 8u);
    wave_sync();
    uint64_t todo = q == 0 ? m0 : (q == 1 ? m1 : (q == 2 ? m2 : m3));
    while (__any(todo != 0)) {
      const bool act = todo != 0;
      const int j = act ? 63 - (int)__builtin_clzll(todo) : 0;     // last first
      if (act) todo &= ~(1ull << j);
      const Splat sp = s_splat[j];
      const int pos = bot + j + 1;
      const float dx = __fsub_rn(fx, sp.mx);
      float p2[PXQ];
      splat_p2_column<PXQ>(sp, dx, fy, p2);
      bool pass[PXQ], any = false;
#pragma unroll
      for (int k = 0; k < PXQ; ++k) {
        pass[k] = act && (pos <= last[k]) && splat_pass(sp, p2[k]);
        any = any || pass[k];
      }
      if (!__any(any)) continue;
      // per-lane sums over the lane's pixels (dx is shared by its column)
      float sG = 0.f, sGdy = 0.f, sGdy2 = 0.f, so = 0.f, sr = 0.f, sg = 0.f, sb = 0.f;
#pragma unroll
      for (int k = 0; k < PXQ; ++k) {
        if (!pass[k]) continue;
        const float gss = splat_gauss(p2[k]);
        const float aa = sp.o * gss;
        const float alpha = fminf(kAlphaMax, aa);
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
        if (aa < kAlphaMax) {
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
      const float comp[9] = {fmaf(2.0f * sp.A * dx, sG, sp.B * sGdy),   // d mx / -ln2
                             fmaf(2.0f * sp.C, sGdy, bdx * sG),         // d my / -ln2
                             dx * dx * sG,                              // d Q11 / -1/2
                             dx * sGdy,                                 // d Q12 / -1
                             sGdy2,                                     // d Q22 / -1/2
                             so, sr, sg, sb};
      const float tot = reduce_scatter9_row(comp);
      // rows whose entry no pixel of theirs passed add nothing
      const uint64_t rows = __ballot(any);
      if (rslot >= 0 && ((rows >> (16 * q)) & 0xffffull) != 0)
        atomicAdd(d_rec + (int64_t)s_id[j] * GS_DREC_STRIDE + rslot, rscale * tot);
    }
  }
}

// ---------------------------------------------------------------- split forward

// Forward of long tile lists in parallel (stored mode with chunk items).
// Part 1: one wave per chunk item (tile, c) composites the chunk's entries
// for the tile's pixels from a local transmittance of 1, ignoring the stop
// rule: P = prod(1 - alpha) and L = sum rgb alpha T_local over the chunk
// (the arithmetic of the sequential forward's chunk composites), and the
// chunk-local position of the last blend.  The (P, L) of chunk c >= 1 go to
// checkpoint slot c - 1, those of chunk 0 to slot nc - 1 (nc = the tile's
// chunks; the backward never reads that slot, the last chunk starting from
// the final state).
template <int TW, int TH>
__global__ __launch_bounds__(kRasterWave) void k_raster_fwd_part(RasterDev a, ChunkDev ch,
                                                                uint16_t* __restrict__ clast) {
  constexpr int PX = TileGeom<TW, TH>::PX;
  __shared__ Splat s_splat[kRasterWave];
  const uint32_t item = blockIdx.x;
  if (item >= ch.offset[a.n_tiles]) return;
  const int64_t tile = ch.items[item];
  const uint32_t c0 = ch.offset[tile];
  const int c = (int)(item - c0), nc = (int)(ch.offset[tile + 1] - c0);
  const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
  const int len = (int)(end - start);
  const int lo = c * ch.chunk, hi_pos = min(lo + ch.chunk, len);
  const LanePixels<TW, TH> L(a, tile);
  const PixBox box{(float)(L.tx * TW) + 0.5f, (float)(L.tx * TW + TW - 1) + 0.5f,
                   (float)(L.ty * TH) + 0.5f, (float)(L.ty * TH + TH - 1) + 0.5f};
  const int lane = threadIdx.x;
  float fyk[PX], Tl[PX], Lc[PX][3];
  int lastl[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    fyk[k] = L.inside[k] ? L.fy[k] : __builtin_nanf("");
    Tl[k] = 1.0f;
    Lc[k][0] = Lc[k][1] = Lc[k][2] = 0.0f;
    lastl[k] = 0;
  }
  for (int b0 = lo; b0 < hi_pos; b0 += kRasterWave) {
    const int n = min(kRasterWave, hi_pos - b0);
    wave_sync();
    bool hit = false;
    if (lane < n) {
      const Splat s = load_splat(a.rec, a.ids[start + b0 + lane]);
      hit = splat_may_hit(s, box.x0, box.x1, box.y0, box.y1);
      s_splat[lane] = s;
    }
    uint64_t todo = __ballot(hit);
    wave_sync();
    while (todo) {
      const int j = (int)__builtin_ctzll(todo);
      todo &= todo - 1;
      const Splat sp = s_splat[j];
      const float dx = __fsub_rn(L.fx, sp.mx);
      float p2[PX];
      splat_p2_column<PX>(sp, dx, fyk, p2);
      bool pass[PX], any = false;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        pass[k] = splat_pass(sp, p2[k]);
        any = any || pass[k];
      }
      if (!__any(any)) continue;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        if (!pass[k]) continue;
        const float alpha = fminf(kAlphaMax, sp.o * splat_gauss(p2[k]));
        const float wl = alpha * Tl[k];
        Lc[k][0] = fmaf(sp.r, wl, Lc[k][0]);
        Lc[k][1] = fmaf(sp.g, wl, Lc[k][1]);
        Lc[k][2] = fmaf(sp.b, wl, Lc[k][2]);
        Tl[k] = Tl[k] * (1.0f - alpha);
        lastl[k] = b0 - lo + j + 1;
      }
    }
  }
  float4* ck = ch.ck + ((int64_t)c0 + (c >= 1 ? c - 1 : nc - 1)) * (TW * TH);
  uint16_t* cl = clast + ((int64_t)c0 + c) * (TW * TH);
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    ck[lane + k * kRasterWave] = make_float4(Tl[k], Lc[k][0], Lc[k][1], Lc[k][2]);
    cl[lane + k * kRasterWave] = (uint16_t)lastl[k];
  }
}

// Part 2: one wave per tile joins its chunks in list order.  A pixel whose
// transmittance stays at or above the cut-off through chunk c (T P_c >=
// T_min: the partial products only fall, so no entry of the chunk stops
// it) takes C += T L_c, T = T P_c; where T P_c < T_min the chunk is
// composited again entry by entry from T with the stop rule (all lanes stage
// it, the pixels concerned composite), and the pixel ends there.  Then the
// image, T_final and n_contrib are written, and the checkpoints become the
// (T_c, U_c) the backward reads, by the recursion of the sequential forward
// over the chunks' (P, L) (identity after a pixel's stop, the partial
// composite up to it in the stopping chunk).  Both walks over the chunks
// keep D chunks' loads in flight: a long list's join is a chain of
// dependent loads otherwise.
template <int TW, int TH>
__global__ __launch_bounds__(kRasterWave) void k_raster_fwd_join(
    RasterDev a, TileSched sch, ChunkDev ch, const uint16_t* __restrict__ clast,
    float* __restrict__ image, float* __restrict__ T_final, int32_t* __restrict__ n_contrib) {
  constexpr int PX = TileGeom<TW, TH>::PX, NP = TW * TH;
  constexpr int D = PX >= 4 ? 1 : 4 / PX;
  __shared__ Splat s_splat[kRasterWave];
  for_each_tile(sch, a.n_tiles, [&](int64_t tile) {
    const LanePixels<TW, TH> L(a, tile);
    const int lane = threadIdx.x;
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const int len = (int)(end - start);
    const uint32_t c0 = ch.offset[tile];
    const int nc = (int)(ch.offset[tile + 1] - c0);
    float4* ck = ch.ck + (int64_t)c0 * NP;
    const uint16_t* cl = clast + (int64_t)c0 * NP;
    const PixBox box{(float)(L.tx * TW) + 0.5f, (float)(L.tx * TW + TW - 1) + 0.5f,
                     (float)(L.ty * TH) + 0.5f, (float)(L.ty * TH + TH - 1) + 0.5f};
    float T[PX], C[PX][3], Ps[PX], Ls[PX][3];
    int last[PX], cs[PX];
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      T[k] = 1.0f;
      C[k][0] = C[k][1] = C[k][2] = 0.0f;
      last[k] = 0;
      cs[k] = nc;                       // chunk of the stop (nc: none)
      Ps[k] = 1.0f;
      Ls[k][0] = Ls[k][1] = Ls[k][2] = 0.0f;
    }
    // chunk c's (P, L) sit in slot c - 1, chunk 0's in slot nc - 1
    auto load_chunk = [&](int c, float4 (&pl)[PX], int (&ll)[PX]) {
      const int sl = c >= 1 ? c - 1 : nc - 1;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        pl[k] = ck[(int64_t)sl * NP + lane + k * kRasterWave];
        ll[k] = cl[(int64_t)c * NP + lane + k * kRasterWave];
      }
    };
    auto join_chunk = [&](int c, const float4 (&pl)[PX], const int (&ll)[PX]) {
      bool fix[PX], any_fix = false;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        fix[k] = false;
        if (cs[k] < nc || !L.inside[k]) continue;
        const float Tn = T[k] * pl[k].x;
        if (Tn < kTMin) {
          fix[k] = true;
          any_fix = true;
          continue;
        }
        C[k][0] = fmaf(T[k], pl[k].y, C[k][0]);
        C[k][1] = fmaf(T[k], pl[k].z, C[k][1]);
        C[k][2] = fmaf(T[k], pl[k].w, C[k][2]);
        T[k] = Tn;
        if (ll[k]) last[k] = c * ch.chunk + ll[k];
      }
      if (!__any(any_fix)) return;
      // composite chunk c again, entry by entry with the stop rule, for the
      // pixels whose transmittance reaches the cut-off inside it
      float fyk[PX], Tl[PX], Lc[PX][3];
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        fyk[k] = fix[k] ? L.fy[k] : __builtin_nanf("");
        Tl[k] = 1.0f;
        Lc[k][0] = Lc[k][1] = Lc[k][2] = 0.0f;
      }
      const int lo = c * ch.chunk, hi_pos = min(lo + ch.chunk, len);
      for (int b0 = lo; b0 < hi_pos; b0 += kRasterWave) {
        const int n = min(kRasterWave, hi_pos - b0);
        wave_sync();
        bool hit = false;
        if (lane < n) {
          const Splat s = load_splat(a.rec, a.ids[start + b0 + lane]);
          hit = splat_may_hit(s, box.x0, box.x1, box.y0, box.y1);
          s_splat[lane] = s;
        }
        uint64_t todo = __ballot(hit);
        wave_sync();
        while (todo) {
          const int j = (int)__builtin_ctzll(todo);
          todo &= todo - 1;
          const Splat sp = s_splat[j];
          const float dx = __fsub_rn(L.fx, sp.mx);
          float p2[PX];
          splat_p2_column<PX>(sp, dx, fyk, p2);
          bool pass[PX], any = false;
#pragma unroll
          for (int k = 0; k < PX; ++k) {
            pass[k] = splat_pass(sp, p2[k]);
            any = any || pass[k];
          }
          if (!__any(any)) continue;
#pragma unroll
          for (int k = 0; k < PX; ++k) {
            if (!pass[k]) continue;
            const float alpha = fminf(kAlphaMax, sp.o * splat_gauss(p2[k]));
            const float Tn = T[k] * (1.0f - alpha);
            if (Tn < kTMin) {              // the pixel stops; this entry is not blended
              fyk[k] = __builtin_nanf("");
              cs[k] = c;
              continue;
            }
            const float w = alpha * T[k];
            C[k][0] = fmaf(sp.r, w, C[k][0]);
            C[k][1] = fmaf(sp.g, w, C[k][1]);
            C[k][2] = fmaf(sp.b, w, C[k][2]);
            const float wl = alpha * Tl[k];
            Lc[k][0] = fmaf(sp.r, wl, Lc[k][0]);
            Lc[k][1] = fmaf(sp.g, wl, Lc[k][1]);
            Lc[k][2] = fmaf(sp.b, wl, Lc[k][2]);
            Tl[k] = Tl[k] * (1.0f - alpha);
            T[k] = Tn;
            last[k] = b0 + j + 1;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        if (cs[k] != c) continue;
        Ps[k] = Tl[k];
        Ls[k][0] = Lc[k][0];
        Ls[k][1] = Lc[k][1];
        Ls[k][2] = Lc[k][2];
      }
    };
    float4 buf[D][PX];
    int lbuf[D][PX];
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (d < nc) load_chunk(d, buf[d], lbuf[d]);
    for (int cb = 0; cb < nc; cb += D) {
      // every pixel stopped (or outside the image): the rest blends nothing
      bool done = true;
#pragma unroll
      for (int k = 0; k < PX; ++k) done = done && (cs[k] < nc || !L.inside[k]);
      if (__all(done)) break;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int c = cb + d;
        if (c >= nc) break;
        float4 pl[PX];
        int ll[PX];
#pragma unroll
        for (int k = 0; k < PX; ++k) {
          pl[k] = buf[d][k];
          ll[k] = lbuf[d][k];
        }
        if (c + D < nc) load_chunk(c + D, buf[d], lbuf[d]);
        join_chunk(c, pl, ll);
      }
    }
    const int64_t HW = (int64_t)a.H * a.W;
    float* img = image + (int64_t)L.slot * 3 * HW;
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      if (!L.inside[k]) continue;
      const int64_t o = L.offset(a, k);
      img[o] = C[k][0] + T[k] * a.bg0;
      img[HW + o] = C[k][1] + T[k] * a.bg1;
      img[2 * HW + o] = C[k][2] + T[k] * a.bg2;
      T_final[(int64_t)L.slot * HW + o] = T[k];
      n_contrib[(int64_t)L.slot * HW + o] = last[k];
    }
    // checkpoints: slot c <- (T_c, U_c) from chunk c+1's (P, L), last first.
    // The backward reads slot c only for pixels that blend after chunk c, so
    // the walk starts below the last chunk holding a blend of any pixel
    // (after it T_c = T_final and U_c = bg exactly).
    int lc = 0;
#pragma unroll
    for (int k = 0; k < PX; ++k) lc = max(lc, (last[k] + ch.chunk - 1) / ch.chunk);
    const int c_top = min(nc - 2, wave_max_int(lc) - 2);
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      float Tn = T[k], U[3] = {a.bg0, a.bg1, a.bg2};
      float4* col = ck + lane + k * kRasterWave;
      for (int cb = c_top; cb >= 0; cb -= D) {
        float4 v[D];
#pragma unroll
        for (int d = 0; d < D; ++d)
          if (cb - d >= 0) v[d] = col[(int64_t)(cb - d) * NP];
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int c = cb - d;
          if (c < 0) break;
          const int e = c + 1;
          const float4 pl = e > cs[k] ? make_float4(1.0f, 0.0f, 0.0f, 0.0f)
                                      : (e == cs[k] ? make_float4(Ps[k], Ls[k][0], Ls[k][1],
                                                                  Ls[k][2])
                                                    : v[d]);
          const float Te = Tn / pl.x;
          U[0] = fmaf(pl.x, U[0], pl.y);
          U[1] = fmaf(pl.x, U[1], pl.z);
          U[2] = fmaf(pl.x, U[2], pl.w);
          col[(int64_t)c * NP] = make_float4(Te, U[0], U[1], U[2]);
          Tn = Te;
        }
      }
    }
  });
}

// ---------------------------------------------------------------- support count

// Per pixel, the number of list entries it blends (alpha test passed,
// transmittance still at or above the cut-off), with the forward's
// decisions: one work-group of 256 threads per tile, up to 2 pixels per
// thread, entries staged 256 at a time.  A measurement of the method's work
// (the pairs an exact rasteriser must composite), not part of the training
// step.
constexpr int kCountThreads = 256;

__global__ __launch_bounds__(kCountThreads) void k_raster_count(RasterDev a, int TW, int TH,
                                                                int32_t* __restrict__ n_blend) {
  __shared__ Splat s_sp[kCountThreads];
  const int64_t tile = blockIdx.x;
  const int slot = (int)(tile / a.tiles_per_slot);
  const int tt = (int)(tile - (int64_t)slot * a.tiles_per_slot);
  const int ty = tt / a.tiles_x, tx = tt - ty * a.tiles_x;
  const int t = threadIdx.x;
  float fx[2], fy[2], T[2];
  int cnt[2];
  bool live[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int p = t + k * kCountThreads;
    const int px = tx * TW + p % TW, py = ty * TH + p / TW;
    fx[k] = (float)px + 0.5f;
    fy[k] = (float)py + 0.5f;
    live[k] = p < TW * TH && px < a.W && py < a.H;
    T[k] = 1.0f;
    cnt[k] = 0;
  }
  const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
  for (uint32_t b0 = start; b0 < end; b0 += kCountThreads) {
    if (__syncthreads_count(live[0] || live[1]) == 0) break;
    if (b0 + t < end) s_sp[t] = load_splat(a.rec, a.ids[b0 + t]);
    __syncthreads();
    const int n = (int)min((uint32_t)kCountThreads, end - b0);
    for (int j = 0; j < n; ++j) {
      const Splat sp = s_sp[j];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (!live[k]) continue;
        float p2;
        splat_p2_column<1>(sp, __fsub_rn(fx[k], sp.mx), &fy[k], &p2);
        if (!splat_pass(sp, p2)) continue;
        const float alpha = fminf(kAlphaMax, sp.o * splat_gauss(p2));
        const float Tn = T[k] * (1.0f - alpha);
        if (Tn < kTMin) {
          live[k] = false;
          continue;
        }
        T[k] = Tn;
        ++cnt[k];
      }
    }
    __syncthreads();
  }
  const int64_t HW = (int64_t)a.H * a.W;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int p = t + k * kCountThreads;
    const int px = tx * TW + p % TW, py = ty * TH + p / TW;
    if (p < TW * TH && px < a.W && py < a.H)
      n_blend[(int64_t)slot * HW + (int64_t)py * a.W + px] = cnt[k];
  }
}

__global__ void k_reset_queue(uint32_t* q) {
  if (threadIdx.x == 0) q[0] = 0u;
}

// ---------------------------------------------------------------- deterministic sum

// d_rec[p][c] += sum over pair p's emission slots of component c, in
// emission order; one thread per (pair, component), so the 9 threads of a
// pair read its slots' 36-byte records together.  pair_first [m][2] holds
// each pair's first emission index and its entry count.
__global__ __launch_bounds__(256) void k_dup_reduce(const uint32_t* __restrict__ pair_first,
                                                    int64_t m, const float* __restrict__ dup,
                                                    int64_t dup_cap, float* __restrict__ d_rec) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t p = i / GS_DREC_STRIDE;
  const int c = (int)(i - p * GS_DREC_STRIDE);
  if (p >= m) return;
  const int64_t nt = pair_first[2 * p + 1];
  if (nt <= 0) return;
  const int64_t e0 = pair_first[2 * p];
  if (e0 + nt > dup_cap) return;
  const float* g = dup + e0 * GS_DREC_STRIDE + c;
  float acc = 0.0f;
  for (int k = 0; k < nt; ++k) acc += g[k * GS_DREC_STRIDE];
  d_rec[p * GS_DREC_STRIDE + c] += acc;
}

// ---------------------------------------------------------------- dispatch

struct Launch {
  unsigned blocks;
  TileSched sch;
  ChunkDev ch;
  int64_t max_items;
  int fwd_waves;
};

static Launch make_launch(const RasterDev& a, const gs_raster_plan* plan) {
  Launch L;
  L.sch.order = plan ? plan->tile_order : nullptr;
  L.sch.queue = plan ? plan->queue : nullptr;
  L.ch.chunk = plan ? plan->chunk : 0;
  L.ch.offset = plan ? plan->chunk_offset : nullptr;
  L.ch.items = plan ? plan->chunk_items : nullptr;
  L.ch.ck = plan && plan->chunk > 0 ? reinterpret_cast<float4*>(plan->checkpoints) : nullptr;
  L.max_items = plan ? plan->max_items : 0;
  L.fwd_waves = plan && plan->fwd_waves > 1 ? plan->fwd_waves : 1;
  if (L.sch.queue) {
    int64_t w = plan->persistent_waves > 0 ? plan->persistent_waves : (int64_t)device_cu_count() * 16;
    L.blocks = (unsigned)std::min<int64_t>(w, std::max<int64_t>(a.n_tiles, 1));
  } else if (L.sch.order) {
    L.blocks = (unsigned)std::max<int64_t>(a.n_tiles, 1);
  } else {
    L.blocks = (unsigned)(8 * ((a.n_tiles + 7) / 8));
  }
  return L;
}

template <int TW, int TH>
static void launch_fwd(const RasterDev& a, const Launch& L, float* image, float* T_final,
                       int32_t* n_contrib, hipStream_t s) {
  constexpr int PXT = TileGeom<TW, TH>::PX;
  if constexpr (PXT % 4 == 0) {
    if (L.fwd_waves == 4) {
      hipLaunchKernelGGL((k_raster_fwd<TW, TH, 4>), dim3(L.blocks), dim3(4 * kRasterWave), 0, s,
                         a, L.sch, L.ch, image, T_final, n_contrib);
      return;
    }
  }
  if constexpr (PXT % 2 == 0) {
    if (L.fwd_waves == 2) {
      hipLaunchKernelGGL((k_raster_fwd<TW, TH, 2>), dim3(L.blocks), dim3(2 * kRasterWave), 0, s,
                         a, L.sch, L.ch, image, T_final, n_contrib);
      return;
    }
  }
  hipLaunchKernelGGL((k_raster_fwd<TW, TH, 1>), dim3(L.blocks), dim3(kRasterWave), 0, s, a, L.sch,
                     L.ch, image, T_final, n_contrib);
}

template <int TW, int TH>
static void launch_fwd_split(const RasterDev& a, const Launch& L, uint16_t* chunk_last,
                             float* image, float* T_final, int32_t* n_contrib, hipStream_t s) {
  hipLaunchKernelGGL((k_raster_fwd_part<TW, TH>), dim3((unsigned)L.max_items), dim3(kRasterWave),
                     0, s, a, L.ch, chunk_last);
  hipLaunchKernelGGL((k_raster_fwd_join<TW, TH>), dim3(L.blocks), dim3(kRasterWave), 0, s, a,
                     L.sch, L.ch, chunk_last, image, T_final, n_contrib);
}

template <int TW, int TH>
static void launch_bwd(const RasterDev& a, const Launch& L, const float* T_final,
                       const int32_t* n_contrib, const float* d_image, int mode, float* d_rec,
                       hipStream_t s) {
  // quadrant groups pay off for the small footprints of 8x8 tiles (the 4K
  // octant: 2.34 -> 1.98 ms); at 16x16 they measured the same as one wave
  // per item (0.421 vs 0.424 ms at 1080p)
  constexpr bool kQuad = TW == 8 && TH == 8;
  if (kQuad && mode == GS_BWD_STORED && L.ch.chunk > 0 && !a.dup_grads)
    hipLaunchKernelGGL((k_raster_bwd_chunked_q<kQuad ? TW : 8, kQuad ? TH : 8>),
                       dim3((unsigned)L.max_items), dim3(kRasterWave), 0, s, a, L.ch, T_final,
                       n_contrib, d_image, d_rec);
  else if (mode == GS_BWD_STORED && L.ch.chunk > 0)
    hipLaunchKernelGGL((k_raster_bwd_chunked<TW, TH>), dim3((unsigned)L.max_items),
                       dim3(kRasterWave), 0, s, a, L.ch, T_final, n_contrib, d_image, d_rec);
  else if (mode == GS_BWD_RECOMPUTE)
    hipLaunchKernelGGL((k_raster_bwd<TW, TH, true>), dim3(L.blocks), dim3(kRasterWave), 0, s, a,
                       L.sch, T_final, n_contrib, d_image, d_rec);
  else
    hipLaunchKernelGGL((k_raster_bwd<TW, TH, false>), dim3(L.blocks), dim3(kRasterWave), 0, s, a,
                       L.sch, T_final, n_contrib, d_image, d_rec);
}

// Tile shapes with a compiled rasteriser.
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
                                RasterDev& a) {
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
  a.bg0 = bg[0];
  a.bg1 = bg[1];
  a.bg2 = bg[2];
  a.emit = nullptr;
  a.dup_grads = nullptr;
  a.dup_cap = 0;
  return GS_OK;
}

static gs_status plan_prepare(const gs_raster_plan* plan, const gs_tiling* tiling, hipStream_t s,
                              const char* who) {
  if (!plan) return GS_OK;
  GS_REQUIRE(plan->persistent_waves >= 0, "%s: persistent_waves < 0", who);
  const int nw = plan->fwd_waves;
  GS_REQUIRE(nw == 0 || nw == 1 || nw == 2 || nw == 4, "%s: fwd_waves %d not in {0, 1, 2, 4}",
             who, nw);
  GS_REQUIRE(nw <= 1 || (tiling->tile_w * tiling->tile_h / kRasterWave) % nw == 0,
             "%s: fwd_waves %d does not divide the %dx%d tile's %d pixels per lane", who, nw,
             tiling->tile_w, tiling->tile_h, tiling->tile_w * tiling->tile_h / kRasterWave);
  GS_REQUIRE(nw <= 1 || plan->queue == nullptr, "%s: fwd_waves > 1 needs a non-persistent plan",
             who);
  if (plan->chunk > 0) {
    GS_REQUIRE(plan->chunk % kRasterWave == 0, "%s: chunk %d is not a multiple of 64", who,
               plan->chunk);
    GS_REQUIRE(plan->chunk_offset && plan->chunk_items && plan->checkpoints &&
                   plan->max_items > 0 && plan->max_items < (int64_t(1) << 31),
               "%s: chunked plan needs chunk_offset, chunk_items, checkpoints, max_items", who);
  }
  if (plan->queue) {
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, s, plan->queue);
    GS_LAUNCH_CHECK(who);
  }
  return GS_OK;
}

}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_raster_fwd(const gs_projected* proj, const gs_views* views, const gs_tiling* tiling,
                        const uint32_t* ids, const uint32_t* tile_ranges, const float bg[3],
                        float* image, float* T_final, int32_t* n_contrib,
                        const gs_raster_plan* plan, void* stream) {
  clear_error();
  RasterDev a;
  gs_status st = raster_prepare(proj, views, tiling, ids, tile_ranges, bg, "gs_raster_fwd", a);
  if (st != GS_OK) return st;
  GS_REQUIRE(image != nullptr, "gs_raster_fwd: NULL image");
  GS_REQUIRE((T_final == nullptr) == (n_contrib == nullptr),
             "gs_raster_fwd: T_final and n_contrib must both be set or both be NULL");
  hipStream_t s = as_stream(stream);
  st = plan_prepare(plan, tiling, s, "gs_raster_fwd");
  if (st != GS_OK) return st;
  const Launch L = make_launch(a, plan);
  const bool split = plan && plan->fwd_split && L.ch.ck != nullptr;
  GS_REQUIRE(!split || (plan->chunk_last && T_final),
             "gs_raster_fwd: fwd_split needs chunk_last and the stored state (T_final, n_contrib)");
#define GS_FWD_CASE(a_, b_)                                                          \
  if (tiling->tile_w == a_ && tiling->tile_h == b_) {                                \
    if (split)                                                                       \
      launch_fwd_split<a_, b_>(a, L, plan->chunk_last, image, T_final, n_contrib, s); \
    else                                                                             \
      launch_fwd<a_, b_>(a, L, image, T_final, n_contrib, s);                        \
  } else
  GS_RASTER_SHAPES(GS_FWD_CASE) {}
#undef GS_FWD_CASE
  GS_LAUNCH_CHECK("gs_raster_fwd");
  return GS_OK;
}

gs_status gs_raster_bwd(const gs_projected* proj, const gs_views* views, const gs_tiling* tiling,
                        const uint32_t* ids, const uint32_t* tile_ranges, const float bg[3],
                        const float* T_final, const int32_t* n_contrib, const float* d_image,
                        int32_t mode, float* d_rec, const gs_raster_plan* plan, void* stream) {
  clear_error();
  RasterDev a;
  gs_status st = raster_prepare(proj, views, tiling, ids, tile_ranges, bg, "gs_raster_bwd", a);
  if (st != GS_OK) return st;
  GS_REQUIRE(mode == GS_BWD_STORED || mode == GS_BWD_RECOMPUTE, "gs_raster_bwd: bad mode %d",
             mode);
  GS_REQUIRE(d_image && d_rec, "gs_raster_bwd: NULL d_image/d_rec");
  GS_REQUIRE(mode == GS_BWD_RECOMPUTE || (T_final && n_contrib),
             "gs_raster_bwd: STORED mode needs T_final and n_contrib");
  hipStream_t s = as_stream(stream);
  const bool det = plan && plan->dup_grads;
  if (det) {
    GS_REQUIRE(plan->pair_first && plan->emit_idx && plan->dup_capacity > 0,
               "gs_raster_bwd: deterministic mode needs pair_first, emit_idx, dup_capacity");
    a.emit = plan->emit_idx;
    a.dup_grads = plan->dup_grads;
    a.dup_cap = plan->dup_capacity;
  }
  st = plan_prepare(plan, tiling, s, "gs_raster_bwd");
  if (st != GS_OK) return st;
  const Launch L = make_launch(a, plan);
#define GS_BWD_CASE(a_, b_)                                                   \
  if (tiling->tile_w == a_ && tiling->tile_h == b_)                           \
    launch_bwd<a_, b_>(a, L, T_final, n_contrib, d_image, mode, d_rec, s);    \
  else
  GS_RASTER_SHAPES(GS_BWD_CASE) {}
#undef GS_BWD_CASE
  GS_LAUNCH_CHECK("gs_raster_bwd");
  if (det && proj->m > 0) {
    hipLaunchKernelGGL(k_dup_reduce, dim3((unsigned)ceil_div(proj->m * GS_DREC_STRIDE, 256)),
                       dim3(256), 0, s,
                       plan->pair_first, proj->m, plan->dup_grads,
                       plan->dup_capacity, d_rec);
    GS_LAUNCH_CHECK("gs_raster_bwd/reduce");
  }
  return GS_OK;
}

gs_status gs_raster_count(const gs_projected* proj, const gs_views* views,
                          const gs_tiling* tiling, const uint32_t* ids,
                          const uint32_t* tile_ranges, int32_t* n_blend, void* stream) {
  clear_error();
  RasterDev a;
  const float bg[3] = {0.f, 0.f, 0.f};
  gs_status st = raster_prepare(proj, views, tiling, ids, tile_ranges, bg, "gs_raster_count", a);
  if (st != GS_OK) return st;
  GS_REQUIRE(n_blend != nullptr, "gs_raster_count: NULL n_blend");
  GS_REQUIRE(tiling->tile_w * tiling->tile_h <= 2 * kCountThreads,
             "gs_raster_count: tile of %d pixels (at most %d)", tiling->tile_w * tiling->tile_h,
             2 * kCountThreads);
  if (a.n_tiles == 0) return GS_OK;
  hipLaunchKernelGGL(k_raster_count, dim3((unsigned)a.n_tiles), dim3(kCountThreads), 0,
                     as_stream(stream), a, tiling->tile_w, tiling->tile_h, n_blend);
  GS_LAUNCH_CHECK("gs_raster_count");
  return GS_OK;
}

}  // extern "C"
