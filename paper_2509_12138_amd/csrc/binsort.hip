// binsort.hip — tile binning and stable sort on (slot*tiles + tile, depth)
// keys for the 3D-GS rasteriser (the per-tile, depth-ordered Gaussian lists
// of the method the paper's Sec. II trains with).
//
// Pipeline (all sizes that depend on data stay on the device, so the whole
// call can be captured in a HIP graph):
//   k_depth_keys + 4 radix passes   the m pairs sorted stably by depth bits
//                  (ties by pair index): the depth order is sorted once per
//                  pair instead of once per duplicate; k_depth_keys also
//                  decides which tiles of each pair's bbox meet its support
//                  (a 64-bit row-major mask over bboxes of up to 64 tiles)
//   k_scan_reduce  per-block sums of the pairs' tile counts, in depth order
//   k_scan_top     exclusive scan of the block sums, total -> status[1],
//                  overflow flag, clamped count
//   k_emit         per block of depth-ordered pairs: local scan of the tile
//                  counts, an LDS map from duplicate to pair, then one
//                  thread per duplicate (coalesced writes) finds its tile as
//                  the k-th set bit of the pair's mask and writes key / pair
//                  index
//   k_radix_hist / k_radix_rowscan / k_radix_scatter   LSD radix passes on
//                  8-bit digits (9-bit when that saves a pass: 17-18 tile
//                  bits) over the tile bits of the keys only (the
//                  emission is already in (depth, pair) order and the passes
//                  are stable); the scatter ranks stably with wave64 ballots
//                  and stages the block in LDS so global writes are runs per
//                  digit
//   k_ranges       [start, end) per tile from the sorted keys
// When the caller does not ask for the sorted (tile, depth) keys, the tile
// phase (emission, tile passes, ranges) carries 32-bit tile indices as keys
// instead of 64-bit keys.
#include "gs_device.h"

namespace gsmi {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanItems = kScanThreads * kScanPer;   // pairs per scan/emit block
constexpr int kEmitRound = 2048;   // duplicates a k_emit block expands at a time
constexpr int kSortThreads = 256;
constexpr int kSortPer = 8;
constexpr int kSortItems = kSortThreads * kSortPer;   // keys per radix block
constexpr int kRadixBits = 8;      // digit width of the depth passes and of most tile passes
constexpr int kRadixBitsMax = 9;   // tile keys of 17-18 bits: two 9-bit passes instead of three
// emission record word 1: bbox width in tiles, and this flag when the whole
// bbox is listed (word 2 then holds the tile count instead of a mask)
constexpr uint32_t kWholeBbox = 1u << 31;
// per-pair tile counts kept as one byte; kNtEscape: look the count up in the
// emission record
constexpr uint32_t kNtEscape = 255;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kRadixMax = 1 << kRadixBitsMax;

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Stages src[0, n) into LDS at dst[at(i)] with 256 threads, kStageBatch
// loads per thread in flight at a time (a plain loop waits for each load
// before its LDS store).
constexpr int kStageBatch = 8;

template <typename T, typename At>
__device__ __forceinline__ void stage_to_lds(const T* __restrict__ src, int n, T* dst, At at) {
  for (int i0 = threadIdx.x; i0 < n; i0 += 256 * kStageBatch) {
    T v[kStageBatch];
#pragma unroll
    for (int q = 0; q < kStageBatch; ++q) {
      const int i = i0 + q * 256;
      v[q] = i < n ? src[i] : T(0);
    }
#pragma unroll
    for (int q = 0; q < kStageBatch; ++q) {
      const int i = i0 + q * 256;
      if (i < n) dst[at(i)] = v[q];
    }
  }
}

struct BinSortLayout {
  int64_t nb_scan, nb_sort, nb_pairs;
  size_t off_block_sums, off_count, off_keys_alt, off_vals_alt, off_emit_alt, off_hist, off_rowtot,
      off_erec;
  size_t off_pkeys[2], off_pvals[2], off_nt8, total;
};

static BinSortLayout layout(int64_t m, int64_t cap) {
  BinSortLayout L;
  const size_t mm = (size_t)(m > 0 ? m : 1);
  L.nb_scan = ceil_div(m > 0 ? m : 1, kScanItems);
  L.nb_sort = ceil_div(cap > 0 ? cap : 1, kSortItems);
  L.nb_pairs = ceil_div(m > 0 ? m : 1, kSortItems);
  const int64_t nb_hist = L.nb_sort > L.nb_pairs ? L.nb_sort : L.nb_pairs;
  size_t o = 0;
  L.off_block_sums = o; o += align256(sizeof(int64_t) * (size_t)L.nb_scan);
  L.off_count = o; o += align256(sizeof(int64_t) * 2);
  // 64-bit keys, or two 32-bit key arrays each starting 256-byte aligned
  L.off_keys_alt = o; o += 2 * align256(sizeof(uint32_t) * (size_t)(cap > 0 ? cap : 1));
  L.off_vals_alt = o; o += align256(sizeof(uint32_t) * (size_t)(cap > 0 ? cap : 1));
  L.off_emit_alt = o; o += align256(sizeof(uint32_t) * (size_t)(cap > 0 ? cap : 1));
  L.off_hist = o; o += align256(sizeof(uint32_t) * (size_t)kRadixMax * (size_t)nb_hist);
  L.off_rowtot = o; o += align256(sizeof(uint32_t) * kRadixMax);
  L.off_erec = o; o += align256(sizeof(uint32_t) * 4 * mm);
  for (int b = 0; b < 2; ++b) {
    L.off_pkeys[b] = o; o += align256(sizeof(uint32_t) * mm);
    L.off_pvals[b] = o; o += align256(sizeof(uint32_t) * mm);
  }
  L.off_nt8 = o; o += align256(mm);
  L.total = o;
  return L;
}

// ------------------------------------------------------------ tile listing

constexpr int kMaskTiles = 64;   // bboxes of more tiles are listed whole

// Tiles of one pair's tile bbox (tx0, ty0)-(tx1, ty1) whose pixel-centre
// rectangle [tx tw + 1/2, tx tw + tw - 1/2] x [ty th + 1/2, ty th + th - 1/2]
// meets the pair's support (alpha >= 1/255, d^T Q d <= 2 ln(255 o)) widened
// by 0.02 + 1e-5 M, M = a X^2 + 2|b| X Y + c Y^2 over the bbox's pixel-centre
// extents: no pixel centre outside it passes the alpha test, and the margin
// exceeds the single-precision rounding of this test and of the per-pixel
// one.  The support is convex, so inside one tile row's pixel-centre band
// its x-extent is an interval [L, R]: the rightmost point of the whole
// ellipse (dx = xmax at dy = -b xmax / c) when that dy lies in the band, else
// the larger of the two band edges' right ends (the right boundary is
// concave in dy), and the same for the left end.  Bit (ty - ty0) * span +
// (tx - tx0) of the result is set for each tile column meeting [L, R].
// Call only for bboxes of at most kMaskTiles tiles.
__device__ __forceinline__ uint64_t support_tile_mask(const float* __restrict__ r, int tx0,
                                                      int ty0, int tx1, int ty1, int tw, int th) {
  const float mx = r[0], my = r[1], a = r[2], b = r[3], c = r[4], o = r[5];
  const int span = tx1 - tx0 + 1, rows = ty1 - ty0 + 1;
  const float X = fmaxf(fabsf((float)(tx0 * tw) + 0.5f - mx),
                        fabsf((float)(tx1 * tw + tw) - 0.5f - mx));
  const float Y = fmaxf(fabsf((float)(ty0 * th) + 0.5f - my),
                        fabsf((float)(ty1 * th + th) - 0.5f - my));
  const float M = fmaf(a * X, X, fmaf(2.0f * fabsf(b) * X, Y, c * Y * Y));
  const float thr = fmaf(1e-5f, M, fmaf(2.0f, logf(255.0f * o), 0.02f));
  // det = a c - b^2 with the rounding error of b^2 carried (thin supports
  // have det << a c)
  const float bb = b * b;
  const float det = fmaf(a, c, -bb) - fmaf(b, b, -bb);
  const int area = span * rows;
  const uint64_t all = area >= 64 ? ~0ull : ((1ull << area) - 1ull);
  if (!(det > 0.0f) || !(thr > 0.0f)) return all;         // degenerate form: list all
  const float ymax = sqrtf(a * thr / det), xmax = sqrtf(c * thr / det);
  const float dyr = -b * xmax / c;                         // dy of the rightmost point
  const float at = a * thr;
  uint64_t mask = 0;
  for (int ty = ty0; ty <= ty1; ++ty) {
    const float y0 = (float)(ty * th) + 0.5f - my;
    const float u0 = fmaxf(y0, -ymax), u1 = fminf(y0 + (float)(th - 1), ymax);
    if (!(u0 <= u1)) continue;
    const float h0 = sqrtf(fmaxf(fmaf(-det * u0, u0, at), 0.0f));
    const float h1 = sqrtf(fmaxf(fmaf(-det * u1, u1, at), 0.0f));
    const float R = (u0 <= dyr && dyr <= u1) ? xmax : fmaxf(fmaf(-b, u0, h0), fmaf(-b, u1, h1)) / a;
    const float L = (u0 <= -dyr && -dyr <= u1) ? -xmax
                                                 : fminf(fmaf(-b, u0, -h0), fmaf(-b, u1, -h1)) / a;
    // columns with tx tw + tw - 1/2 >= mx + L and tx tw + 1/2 <= mx + R
    const float f0 = fmaxf(ceilf((mx + L + 0.5f) / (float)tw - 1.0f), (float)tx0);
    const float f1 = fminf(floorf((mx + R - 0.5f) / (float)tw), (float)tx1);
    if (!(f0 <= f1)) continue;
    const int c0 = (int)f0, n = (int)f1 - c0 + 1;
    const uint64_t run = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
    mask |= run << ((ty - ty0) * span + (c0 - tx0));
  }
  return mask;
}

// Position of the k-th set bit (from 0) of v, which has more than k.
__device__ __forceinline__ int select_bit(uint64_t v, uint32_t k) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    const uint64_t low = v & ((1ull << w) - 1ull);
    const uint32_t cnt = (uint32_t)__popcll(low);
    if (k >= cnt) {
      k -= cnt;
      v >>= w;
      pos += w;
    }
  }
  return pos;
}

// ------------------------------------------------------------ block scans

// Inclusive prefix sum over a wave64 with cross-lane shuffles.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Exclusive prefix sum over a 256-thread block; `total` receives the sum.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* sm_waves /*[4]*/, T& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T inc = wave_inclusive_scan(v);
  if (lane == 63) sm_waves[wave] = inc;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    T x = sm_waves[w];
    if (w < wave) base += x;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return base + inc - v;
}

// ------------------------------------------------------------ scan of n_tiles

// Pairs in depth order (perm: pair index at each depth-ordered position):
// their tile counts from the one-byte copies (a random gather from a small
// array), the emission record for the rare count of kNtEscape or more.
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ perm,
                                                              const uint8_t* __restrict__ nt8,
                                                              const uint4* __restrict__ erec,
                                                              int64_t m,
                                                              int64_t* __restrict__ block_sums) {
  __shared__ int64_t sm[4];
  int64_t base = (int64_t)blockIdx.x * kScanItems;
  int64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    int64_t i = base + k * kScanThreads + threadIdx.x;
    if (i < m) {
      const uint32_t p = perm[i];
      uint32_t c = nt8[p];
      if (c == kNtEscape) c = erec[p].z;
      sum += (int64_t)c;
    }
  }
  int64_t total;
  block_exclusive_scan<int64_t>(sum, sm, total);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Single workgroup: exclusive scan of nb block sums in place; writes the
// true total to status[1] and min(total, cap) to count[0].  The sums are
// staged in LDS kTopLds at a time with coalesced loads (one padding slot
// after every 32, so the per-thread runs below start in different banks),
// thread t scans its run of consecutive sums there, and the prefixes go back
// with coalesced stores; the running total carries from segment to segment.
constexpr int kTopLds = 8192;

__global__ __launch_bounds__(kScanThreads) void k_scan_top(int64_t* __restrict__ block_sums,
                                                           int64_t nb, int64_t cap,
                                                           int64_t* __restrict__ status,
                                                           int64_t* __restrict__ count) {
  __shared__ int64_t r[kTopLds + kTopLds / 32];
  __shared__ int64_t sm[4];
  auto at = [](int i) { return i + (i >> 5); };
  int64_t carry = 0;
  for (int64_t s0 = 0; s0 < nb; s0 += kTopLds) {
    const int n = (int)min((int64_t)kTopLds, nb - s0);
    int64_t* seg = block_sums + s0;
    stage_to_lds(seg, n, r, at);
    __syncthreads();
    const int per = (n + kScanThreads - 1) / kScanThreads;
    const int b0 = min((int)threadIdx.x * per, n), b1 = min(b0 + per, n);
    int64_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += r[at(b)];
    int64_t total;
    int64_t ex = carry + block_exclusive_scan<int64_t>(sum, sm, total);
    for (int b = b0; b < b1; ++b) {
      const int64_t x = r[at(b)];
      r[at(b)] = ex;
      ex += x;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kScanThreads) seg[i] = r[at(i)];
    carry += total;
    __syncthreads();                                 // LDS reused by the next segment
  }
  if (threadIdx.x == 0) {
    if (status) {
      status[1] = carry;
      if (carry > cap) status[0] |= GS_FLAG_CAPACITY;
    }
    count[0] = carry < cap ? carry : cap;
  }
}

// ------------------------------------------------------------ emit

// Block b handles depth-ordered positions b*kScanItems ...: pair perm[i]
// with depth bits pkey[i] and emission record erec[perm[i]] (k_depth_keys),
// which also gives its tile count: one 16-byte gather per pair.
// pair_first (optional) is [m][2]: word 0 of a pair with tiles > 0 receives
// the emission index of its first entry.
// The block's duplicates are expanded kEmitRound at a time: each thread
// marks, in an LDS owner map, the duplicates of its own pairs that fall in
// the round, then one thread per duplicate reads its pair from the map
// (coalesced key and value writes, no search).
template <typename K>
__global__ __launch_bounds__(kScanThreads) void k_emit(
    const uint4* __restrict__ erec, const uint32_t* __restrict__ pkey,
    const uint32_t* __restrict__ perm, int64_t m,
    const int64_t* __restrict__ block_offsets, int64_t cap, int tiles_x, int tiles_per_slot,
    K* __restrict__ keys, uint32_t* __restrict__ vals, uint32_t* __restrict__ pair_first,
    uint32_t* __restrict__ emit) {
  __shared__ uint32_t s_off[kScanItems + 1];
  __shared__ uint32_t s_base[kScanItems];     // tile index of the bbox's first tile
  __shared__ uint32_t s_span[kScanItems];     // bbox width in tiles
  __shared__ uint64_t s_mask[kScanItems];
  __shared__ uint32_t s_depth[sizeof(K) == 8 ? kScanItems : 1];   // only 64-bit keys use it
  __shared__ uint32_t s_pair[kScanItems];
  __shared__ uint16_t s_owner[kEmitRound];
  __shared__ uint32_t s_w[4];
  static_assert(kScanItems <= 65536, "owner map holds 16-bit pair slots");
  (void)tiles_per_slot;
  const int64_t base = (int64_t)blockIdx.x * kScanItems;
  const int t = threadIdx.x;
  // stage the block's pairs (striped, coalesced) ...
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    int li = k * kScanThreads + t;
    int64_t i = base + li;
    int nt = 0;
    if (i < m) {
      const uint32_t p = perm[i];
      const uint4 e = erec[p];
      const bool whole = (e.y & kWholeBbox) != 0u;
      const uint64_t mask = whole ? 0ull : (((uint64_t)e.w << 32) | e.z);
      nt = whole ? (int)e.z : __popcll(mask);
      if (nt > 0) {
        s_base[li] = e.x;
        s_span[li] = e.y & ~kWholeBbox;
        s_mask[li] = mask;
        if constexpr (sizeof(K) == 8) s_depth[li] = pkey[i];   // only 64-bit keys hold it
        s_pair[li] = p;
      }
    }
    s_off[li] = (uint32_t)nt;
  }
  __syncthreads();
  // ... then scan them in blocked order (thread t owns items t*kScanPer ...)
  uint32_t v[kScanPer], run = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = s_off[t * kScanPer + k];
    run += v[k];
  }
  uint32_t total;
  uint32_t ex = block_exclusive_scan<uint32_t>(run, s_w, total);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    s_off[t * kScanPer + k] = ex;
    ex += v[k];
  }
  if (t == 0) s_off[kScanItems] = total;
  __syncthreads();
  const int64_t gbase = block_offsets[blockIdx.x];
  if (pair_first) {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const int li = k * kScanThreads + t;
      const int64_t i = base + li;
      if (i < m && s_off[li + 1] > s_off[li])
        pair_first[2 * (int64_t)s_pair[li]] = (uint32_t)(gbase + s_off[li]);
    }
  }
  for (uint32_t r0 = 0; r0 < total; r0 += kEmitRound) {
    const uint32_t r1 = min(total, r0 + (uint32_t)kEmitRound);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const int li = t * kScanPer + k;
      const uint32_t q0 = max(s_off[li], r0), q1 = min(s_off[li + 1], r1);
      for (uint32_t q = q0; q < q1; ++q) s_owner[q - r0] = (uint16_t)li;
    }
    __syncthreads();
    for (uint32_t j = r0 + t; j < r1; j += kScanThreads) {
      const int64_t dst = gbase + j;
      if (dst >= cap) break;
      const int li = s_owner[j - r0];
      uint32_t k = j - s_off[li];
      // the k-th listed tile: k-th set bit of the mask, or the k-th bbox tile
      const uint64_t mk = s_mask[li];
      if (mk) k = (uint32_t)select_bit(mk, k);
      const uint32_t span = s_span[li];
      const uint32_t ky = k / span;
      const uint64_t tile = (uint64_t)(s_base[li] + ky * (uint32_t)tiles_x + (k - ky * span));
      if constexpr (sizeof(K) == 8)
        keys[dst] = (tile << 32) | (uint64_t)s_depth[li];
      else
        keys[dst] = (K)tile;
      vals[dst] = s_pair[li];
      if (emit) emit[dst] = (uint32_t)dst;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ depth presort

// key = depth bits (the first radix pass takes the pair index i as its
// value); count[0] = m.  Depths of visible pairs are positive, so their bits
// order as the floats.  Every pair gets its emission record erec[i] =
// (index of its bbox's first tile: slot * tiles_per_slot + ty0 * tiles_x +
// tx0, bbox width, mask low and high words): the listed tiles are the set
// bits of support_tile_mask for a bbox of up to kMaskTiles tiles; a larger
// bbox is listed whole (width | kWholeBbox, tile count, 0); a pair that lists
// no tile gets zeros.  nt8[i] = min(tile count, kNtEscape); pair_count
// (optional) receives the count.
// Also clears the n_range_words words of the tile ranges (grid-stride), so
// the bin/sort needs no separate fill before k_ranges writes them.
__global__ __launch_bounds__(256) void k_depth_keys(const float* __restrict__ rec,
                                                   const int32_t* __restrict__ n_tiles,
                                                   const uint2* __restrict__ tile_bbox, int tw,
                                                   int th, int tiles_x, int tiles_per_slot,
                                                   int64_t m,
                                                   uint32_t* __restrict__ keys,
                                                   uint8_t* __restrict__ nt8,
                                                   uint4* __restrict__ erec,
                                                   uint32_t* __restrict__ pair_count,
                                                   int64_t* __restrict__ count,
                                                   uint32_t* __restrict__ ranges,
                                                   int64_t n_range_words) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t w = i; w < n_range_words; w += (int64_t)gridDim.x * 256) ranges[w] = 0u;
  if (i == 0) count[0] = m;
  if (i >= m) return;
  const float* r = rec + i * GS_REC_STRIDE;
  uint32_t nt = (uint32_t)max(n_tiles[i], 0);
  uint4 e = make_uint4(0u, 0u, 0u, 0u);
  if (nt > 0) {
    const uint32_t slot = __float_as_uint(r[10]);
    const uint2 bb = tile_bbox[i];
    const int tx0 = (int)(bb.x & 0xffff), ty0 = (int)(bb.x >> 16), tx1 = (int)(bb.y & 0xffff);
    const uint32_t first = slot * (uint32_t)tiles_per_slot + (uint32_t)(ty0 * tiles_x + tx0);
    const uint32_t span = (uint32_t)(tx1 - tx0 + 1);
    if (nt <= (uint32_t)kMaskTiles) {
      const uint64_t mask = support_tile_mask(r, tx0, ty0, tx1, (int)(bb.y >> 16), tw, th);
      nt = (uint32_t)__popcll(mask);
      if (nt > 0) e = make_uint4(first, span, (uint32_t)mask, (uint32_t)(mask >> 32));
    } else {
      e = make_uint4(first, span | kWholeBbox, nt, 0u);
    }
  }
  erec[i] = e;
  nt8[i] = (uint8_t)min(nt, kNtEscape);
  if (pair_count) pair_count[2 * i + 1] = nt;
  keys[i] = __float_as_uint(r[9]);
}

// ------------------------------------------------------------ radix sort

// Adds the RB-bit digits (key >> shift) of the keys [b0, min(b0 + kSortItems,
// n)) to the LDS counts h (256 threads).  The counts do not depend on which
// thread reads which key, so a 16-byte aligned array is read in whole
// 16-byte words, all of a thread's loads issued before its first count.
template <int RB, typename K>
__device__ __forceinline__ void count_block(const K* __restrict__ keys, int64_t b0, int64_t n,
                                            int shift, uint32_t* h) {
  constexpr int KP = 16 / (int)sizeof(K);                  // keys per word
  constexpr int WPT = kSortItems / KP / kSortThreads;     // words per thread
  constexpr uint32_t R = 1u << RB;
  const int t = threadIdx.x;
  union Word {
    uint4 v;
    K k[KP];
  };
  if ((reinterpret_cast<uintptr_t>(keys) & 15) == 0) {
    Word w[WPT];
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const int64_t e0 = b0 + (int64_t)(q * kSortThreads + t) * KP;
      if (e0 + KP <= n) {
        w[q].v = *reinterpret_cast<const uint4*>(keys + e0);
      } else {
#pragma unroll
        for (int k = 0; k < KP; ++k) w[q].k[k] = e0 + k < n ? keys[e0 + k] : K(0);
      }
    }
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const int64_t e0 = b0 + (int64_t)(q * kSortThreads + t) * KP;
#pragma unroll
      for (int k = 0; k < KP; ++k)
        if (e0 + k < n) atomicAdd(&h[(uint32_t)(w[q].k[k] >> shift) & (R - 1)], 1u);
    }
  } else {
#pragma unroll 4
    for (int k = 0; k < kSortPer; ++k) {
      const int64_t i = b0 + k * kSortThreads + t;
      if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & (R - 1)], 1u);
    }
  }
}

// Digit counts of one block of keys: hist[digit][block].  RB-bit digits,
// 1 << RB of them (each thread owns 1 << RB / 256).
template <int RB, typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const K* __restrict__ keys,
                                                             const int64_t* __restrict__ count,
                                                             int shift, int64_t nb,
                                                             uint32_t* __restrict__ hist) {
  constexpr int R = 1 << RB, DPT = R / kSortThreads;
  __shared__ uint32_t h[R];
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < DPT; ++q) h[t + q * kSortThreads] = 0;
  __syncthreads();
  const int64_t n = count[0];
  const int64_t base = (int64_t)blockIdx.x * kSortItems;
  // blocks past the count are never read (the row scans and the scatter
  // stop at the last block that holds keys)
  if (base >= n) return;
  count_block<RB>(keys, base, n, shift, h);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int d = t + q * kSortThreads;
    hist[(int64_t)d * nb + blockIdx.x] = h[d];
  }
}

// The same counts for G consecutive blocks per work-group: the G counts of
// one digit are adjacent in the digit-major table, so the writes go out in
// G-word runs instead of one scattered word per (block, digit).  For large
// sorts, where the scattered writes of k_radix_hist dominate its time.
template <int RB, int G, typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist_g(const K* __restrict__ keys,
                                                               const int64_t* __restrict__ count,
                                                               int shift, int64_t nb,
                                                               uint32_t* __restrict__ hist) {
  constexpr int R = 1 << RB, RP = R + 1;               // padded rows: no bank conflicts below
  __shared__ uint32_t h[G * RP];
  const int t = threadIdx.x;
  for (int i = t; i < G * RP; i += kSortThreads) h[i] = 0;
  __syncthreads();
  const int64_t n = count[0];
  const int64_t b0 = (int64_t)blockIdx.x * G;
  const int64_t nb_used = min(nb, (n + kSortItems - 1) / kSortItems);
  if (b0 >= nb_used) return;
  for (int g = 0; g < G; ++g) {
    const int64_t base = (b0 + g) * kSortItems;
    if (base >= n) break;
    count_block<RB>(keys, base, n, shift, h + g * RP);
  }
  __syncthreads();
  for (int idx = t; idx < G * R; idx += kSortThreads) {
    const int d = idx / G, g = idx - d * G;
    if (b0 + g < nb_used) hist[(int64_t)d * nb + b0 + g] = h[g * RP + d];
  }
}

// Launch the digit counts of one pass: grouped blocks for large sorts.
template <int RB, typename K>
static void launch_hist(const K* keys, const int64_t* count, int shift, int64_t nb,
                        uint32_t* hist, hipStream_t s) {
  constexpr int G = 8;
  // (grouped from 2048 blocks: with the 16-byte key loads also for 8-bit
  // digits, 4 passes over 13.3M depth keys 0.121 -> 0.105 ms; 9-bit digits
  // over 20.7M keys 0.164 -> 0.084 ms before those loads)
  if (nb >= 2048)
    hipLaunchKernelGGL((k_radix_hist_g<RB, G, K>), dim3((unsigned)((nb + G - 1) / G)),
                       dim3(kSortThreads), 0, s, keys, count, shift, nb, hist);
  else
    hipLaunchKernelGGL((k_radix_hist<RB, K>), dim3((unsigned)nb), dim3(kSortThreads), 0, s, keys,
                       count, shift, nb, hist);
}

// The row of a digit's block counts is scanned in segments of up to kRowLds
// counts staged in LDS with coalesced loads (each thread scans its part
// there) and written back with coalesced stores, the running total carried
// from segment to segment; one padding slot after every 32 counts starts the
// threads' runs in different LDS banks.  (Scanning per-thread segments in global memory
// instead, every access of a wave touched 64 lines: 43 us per pass at 17K
// blocks, 475 us at 50K.)
constexpr int kRowLds = 32768;                      // 132 KB of LDS with the padding

__global__ __launch_bounds__(256) void k_radix_rowscan_lds(uint32_t* __restrict__ hist, int64_t nb,
                                                           const int64_t* __restrict__ count,
                                                           uint32_t* __restrict__ row_tot) {
  __shared__ uint32_t r[kRowLds + kRowLds / 32];   // one padding slot after every 32
  auto at = [](int i) { return i + (i >> 5); };
  __shared__ uint32_t sm[4];
  uint32_t* row = hist + (int64_t)blockIdx.x * nb;
  // the row's first nb_used counts: the blocks that hold keys
  const int64_t nb_used = min(nb, (count[0] + kSortItems - 1) / kSortItems);
  uint32_t carry = 0;
  for (int64_t s0 = 0; s0 < nb_used; s0 += kRowLds) {
    const int n = (int)min((int64_t)kRowLds, nb_used - s0);
    uint32_t* seg = row + s0;
    stage_to_lds(seg, n, r, at);
    __syncthreads();
    const int per = (n + 255) / 256;
    const int b0 = min((int)threadIdx.x * per, n), b1 = min(b0 + per, n);
    uint32_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += r[at(b)];
    uint32_t total;
    uint32_t ex = carry + block_exclusive_scan<uint32_t>(sum, sm, total);
    for (int b = b0; b < b1; ++b) {
      const uint32_t x = r[at(b)];
      r[at(b)] = ex;
      ex += x;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 256) seg[i] = r[at(i)];
    carry += total;
    __syncthreads();                                 // LDS reused by the next segment
  }
  if (threadIdx.x == 0) row_tot[blockIdx.x] = carry;
}

static void launch_rowscan(uint32_t* hist, int64_t nb, const int64_t* count, uint32_t* row_tot,
                           int digits, hipStream_t s) {
  hipLaunchKernelGGL(k_radix_rowscan_lds, dim3(digits), dim3(256), 0, s, hist, nb, count,
                     row_tot);
}

// One stable LSD pass over RB-bit digits (1 << RB of them; each thread owns
// 1 << RB / 256 consecutive digits).  vin NULL: the value of item i is i.
// TWO: a second value vin2 -> vout2 is carried along.  The block's 2048 items are ranked in 8 rounds of 256 (item
// base + r * 256 + t in round r): within a wave by ballots over the digit
// bits, then per round the owner of each digit turns the 4 waves' counts
// into offsets after the items of earlier rounds and waves, so the LDS holds
// one round's counts (double-buffered) instead of all 32 (round, wave) rows
// and more blocks fit on a CU.
template <int RB, bool TWO, typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const K* __restrict__ kin, const uint32_t* __restrict__ vin,
    K* __restrict__ kout, uint32_t* __restrict__ vout, const int64_t* __restrict__ count,
    int shift, int64_t nb, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ row_tot,
    const uint32_t* __restrict__ vin2, uint32_t* __restrict__ vout2) {
  constexpr int R = 1 << RB, DPT = R / kSortThreads;
  static_assert(DPT >= 1 && R % kSortThreads == 0, "digits per thread");
  __shared__ uint16_t s_cnt[2][4][R];               // one round's (wave, digit) counts
  __shared__ uint32_t s_run[R];                     // items of earlier rounds per digit
  __shared__ K s_key[kSortItems];                   // 16 KB (64-bit keys), 8 KB
  __shared__ uint32_t s_val[kSortItems];            // 8 KB
  __shared__ uint32_t s_val2[TWO ? kSortItems : 1];
  __shared__ uint32_t s_dstart[R];                  // local digit starts
  __shared__ uint32_t s_gbase[R];                   // global digit base of this block
  __shared__ uint32_t s_w[4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t n = count[0];
  const int64_t base = (int64_t)blockIdx.x * kSortItems;
  if (base >= n) return;
  // global base per digit = sum of all row totals of smaller digits + this
  // block's exclusive prefix within the digit's row
  {
    uint32_t rt[DPT], sum = 0;
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      rt[q] = row_tot[t * DPT + q];
      sum += rt[q];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan<uint32_t>(sum, s_w, tot);
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int d = t * DPT + q;
      s_gbase[d] = ex + hist[(int64_t)d * nb + blockIdx.x];
      ex += rt[q];
    }
  }
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int d = t * DPT + q;
    s_run[d] = 0u;
#pragma unroll
    for (int w = 0; w < 4; ++w) s_cnt[0][w][d] = 0;
  }
  __syncthreads();
  K key[kSortPer];
  uint32_t val[kSortPer], val2[kSortPer];
  uint32_t rank[kSortPer];                 // position among the block's items of its digit
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // all rounds' loads first: the barriers of the ranking below would
  // otherwise hold each round's load until the round before it is ranked
#pragma unroll
  for (int r = 0; r < kSortPer; ++r) {
    const int64_t i = base + r * kSortThreads + t;
    const bool valid = i < n;
    key[r] = valid ? kin[i] : (K)0;
    val[r] = valid ? (vin ? vin[i] : (uint32_t)i) : 0u;
    if (TWO) val2[r] = valid ? vin2[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kSortPer; ++r) {
    const int b = r & 1;
    const bool valid = base + r * kSortThreads + t < n;
    const uint32_t d = (uint32_t)(key[r] >> shift) & (R - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < RB; ++bit) {
      const uint64_t m = __ballot((d >> bit) & 1u);
      peers &= ((d >> bit) & 1u) ? m : ~m;
    }
    const uint32_t wrank = (uint32_t)__popcll(peers & lt_mask);
    if (valid && wrank == 0) s_cnt[b][wave][d] = (uint16_t)__popcll(peers);
    __syncthreads();
    // digit owners: counts -> offsets; clear the other buffer for round r + 1
    // (its offsets of round r - 1 were read before the barrier above)
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int dd = t * DPT + q;
      uint32_t run = s_run[dd];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint32_t c = s_cnt[b][w][dd];
        s_cnt[b][w][dd] = (uint16_t)run;
        run += c;
        s_cnt[b ^ 1][w][dd] = 0;
      }
      s_run[dd] = run;
    }
    __syncthreads();
    rank[r] = (uint32_t)s_cnt[b][wave][d] + wrank;
  }
  // s_run: the block's count per digit; exclusive scan over digits
  {
    uint32_t run[DPT], sum = 0;
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      run[q] = s_run[t * DPT + q];
      sum += run[q];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan<uint32_t>(sum, s_w, tot);
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      s_dstart[t * DPT + q] = ex;
      ex += run[q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortPer; ++r) {
    const int64_t i = base + r * kSortThreads + t;
    if (i < n) {
      const uint32_t d = (uint32_t)(key[r] >> shift) & (R - 1);
      const uint32_t pos = s_dstart[d] + rank[r];
      s_key[pos] = key[r];
      s_val[pos] = val[r];
      if (TWO) s_val2[pos] = val2[r];
    }
  }
  __syncthreads();
  const int64_t nloc = min((int64_t)kSortItems, n - base);
#pragma unroll 4
  for (int r = 0; r < kSortPer; ++r) {
    const int li = r * kSortThreads + t;
    if (li < nloc) {
      const K k = s_key[li];
      const uint32_t d = (uint32_t)(k >> shift) & (R - 1);
      const int64_t dst = (int64_t)s_gbase[d] + (li - (int64_t)s_dstart[d]);
      kout[dst] = k;
      vout[dst] = s_val[li];
      if (TWO) vout2[dst] = s_val2[li];
    }
  }
}

// One scatter pass, one block per work-group.
template <int RB, typename K>
static void launch_scatter(const K* kin, const uint32_t* vin, K* kout,
                           uint32_t* vout, const int64_t* count, int shift, int64_t nb,
                           const uint32_t* hist, const uint32_t* row_tot, const uint32_t* vin2,
                           uint32_t* vout2, hipStream_t s) {
  // (G consecutive blocks per work-group, so that their prefixes within a
  // digit's row share a cache line, measured slower: 162 vs 127 us for an
  // 8-bit pass over 13.3M keys at G = 4)
  if (vin2 != nullptr)
    hipLaunchKernelGGL((k_radix_scatter<RB, true, K>), dim3((unsigned)nb), dim3(kSortThreads), 0, s,
                       kin, vin, kout, vout, count, shift, nb, hist, row_tot, vin2, vout2);
  else
    hipLaunchKernelGGL((k_radix_scatter<RB, false, K>), dim3((unsigned)nb), dim3(kSortThreads), 0,
                       s, kin, vin, kout, vout, count, shift, nb, hist, row_tot, vin2, vout2);
}

// Tile index of a sorted key: the high word of a 64-bit (tile, depth) key, or
// the whole 32-bit tile key.
template <typename K>
__device__ __forceinline__ uint32_t key_tile(K k) {
  if constexpr (sizeof(K) == 8)
    return (uint32_t)(k >> 32);
  else
    return (uint32_t)k;
}

// Each thread takes kRangePer consecutive sorted keys and the one before
// them, and marks the tile boundaries among them.
constexpr int kRangePer = 4;

template <typename K>
__global__ __launch_bounds__(256) void k_ranges(const K* __restrict__ keys,
                                                const int64_t* __restrict__ count,
                                                uint32_t* __restrict__ ranges) {
  const int64_t n = count[0];
  const int64_t j0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * kRangePer;
  if (j0 >= n) return;
  uint32_t prev = j0 > 0 ? key_tile(keys[j0 - 1]) : 0u;
  uint32_t tk[kRangePer];
#pragma unroll
  for (int q = 0; q < kRangePer; ++q) tk[q] = j0 + q < n ? key_tile(keys[j0 + q]) : 0u;
#pragma unroll
  for (int q = 0; q < kRangePer; ++q) {
    const int64_t j = j0 + q;
    if (j >= n) break;
    if (j == 0 || prev != tk[q]) {
      ranges[2 * (int64_t)tk[q]] = (uint32_t)j;
      if (j > 0) ranges[2 * (int64_t)prev + 1] = (uint32_t)j;
    }
    if (j == n - 1) ranges[2 * (int64_t)tk[q] + 1] = (uint32_t)n;
    prev = tk[q];
  }
}

// The tile phase after the depth presort: emission of the duplicates in
// (depth, pair) order into (k0, v0, e0), `passes` stable passes of rb-bit
// digits over the tile bits (from bit key_shift) ping-ponging with
// (k1, v1, e1), and the tile ranges.  K = uint64_t: (tile << 32) | depth
// keys; K = uint32_t: the tile index only (half the key traffic).
template <typename K>
static gs_status tile_phase(K* k0, K* k1, uint32_t* v0, uint32_t* v1, uint32_t* e0, uint32_t* e1,
                            int key_shift, int rb, int passes, const uint4* erec,
                            const uint32_t* pkey, const uint32_t* pval, int64_t m,
                            const int64_t* block_sums, int64_t cap, int tiles_x,
                            int tiles_per_slot, uint32_t* pair_first, const int64_t* count,
                            const BinSortLayout& L, uint32_t* hist, uint32_t* rowtot,
                            uint32_t* tile_ranges, hipStream_t s) {
  hipLaunchKernelGGL(k_emit<K>, dim3((unsigned)L.nb_scan), dim3(kScanThreads), 0, s, erec, pkey,
                     pval, m, block_sums, cap, tiles_x, tiles_per_slot, k0, v0, pair_first, e0);
  GS_LAUNCH_CHECK("gs_bin_sort/emit");
  for (int p = 0; p < passes; ++p) {
    const int shift = key_shift + p * rb;
    const K* kin = (p % 2 == 0) ? k0 : k1;
    const uint32_t* vin = (p % 2 == 0) ? v0 : v1;
    K* kout = (p % 2 == 0) ? k1 : k0;
    uint32_t* vout = (p % 2 == 0) ? v1 : v0;
    const uint32_t* ein = (p % 2 == 0) ? e0 : e1;
    uint32_t* eout = (p % 2 == 0) ? e1 : e0;
    if (rb == kRadixBitsMax)
      launch_hist<kRadixBitsMax>(kin, count, shift, L.nb_sort, hist, s);
    else
      launch_hist<kRadixBits>(kin, count, shift, L.nb_sort, hist, s);
    GS_LAUNCH_CHECK("gs_bin_sort/radix_hist");
    launch_rowscan(hist, L.nb_sort, count, rowtot, 1 << rb, s);
    GS_LAUNCH_CHECK("gs_bin_sort/radix_rowscan");
    if (rb == kRadixBitsMax)
      launch_scatter<kRadixBitsMax>(kin, vin, kout, vout, count, shift, L.nb_sort, hist, rowtot,
                                    ein, eout, s);
    else
      launch_scatter<kRadixBits>(kin, vin, kout, vout, count, shift, L.nb_sort, hist, rowtot, ein,
                                 eout, s);
    GS_LAUNCH_CHECK("gs_bin_sort/radix_scatter");
  }
  const K* sorted = (passes % 2 == 0) ? k0 : k1;
  hipLaunchKernelGGL(k_ranges<K>, dim3((unsigned)ceil_div(ceil_div(cap, kRangePer), 256)),
                     dim3(256), 0, s, sorted, count, tile_ranges);
  GS_LAUNCH_CHECK("gs_bin_sort/ranges");
  return GS_OK;
}

}  // namespace gsmi

using namespace gsmi;

extern "C" {

size_t gs_bin_sort_workspace_bytes(int64_t m, int64_t dup_capacity, const gs_tiling* tiling,
                                   int32_t n_slots) {
  (void)tiling;
  (void)n_slots;
  if (m < 0 || dup_capacity < 0) return 0;
  return layout(m, dup_capacity).total;
}

gs_status gs_bin_sort(const gs_projected* proj, const gs_views* views, const gs_tiling* tiling,
                      int64_t dup_capacity, void* ws, size_t ws_bytes, uint64_t* keys_out,
                      uint32_t* ids_out, uint32_t* tile_ranges, uint32_t* pair_first,
                      uint32_t* emit_out, int64_t* status, void* stream) {
  clear_error();
  GS_REQUIRE(proj != nullptr, "gs_bin_sort: NULL proj");
  gs_status st = check_views(views, tiling, "gs_bin_sort");
  if (st != GS_OK) return st;
  GS_REQUIRE(proj->m == views->total_pairs, "gs_bin_sort: proj->m != total_pairs");
  GS_REQUIRE(dup_capacity >= 1 && dup_capacity <= (int64_t)0xFFFFFFFFll,
             "gs_bin_sort: dup_capacity=%lld outside [1, 2^32-1]", (long long)dup_capacity);
  GS_REQUIRE(ids_out && tile_ranges && ws, "gs_bin_sort: NULL output/workspace");
  const int64_t m = proj->m;
  GS_REQUIRE(m == 0 || (proj->rec && proj->tile_bbox && proj->n_tiles),
             "gs_bin_sort: NULL projected arrays");
  BinSortLayout L = layout(m, dup_capacity);
  GS_REQUIRE(ws_bytes >= L.total, "gs_bin_sort: workspace %zu < required %zu", ws_bytes, L.total);
  GS_REQUIRE(((uintptr_t)ws & 255) == 0, "gs_bin_sort: workspace must be 256-byte aligned");
  hipStream_t s = as_stream(stream);
  char* w = (char*)ws;
  int64_t* block_sums = (int64_t*)(w + L.off_block_sums);
  int64_t* count = (int64_t*)(w + L.off_count);
  uint64_t* keys_alt = (uint64_t*)(w + L.off_keys_alt);
  uint32_t* vals_alt = (uint32_t*)(w + L.off_vals_alt);
  uint32_t* hist = (uint32_t*)(w + L.off_hist);
  uint32_t* rowtot = (uint32_t*)(w + L.off_rowtot);
  const int tiles_x = (int)ceil_div(tiling->width, tiling->tile_w);
  const int tiles_y = (int)ceil_div(tiling->height, tiling->tile_h);
  const int64_t tiles_per_slot = (int64_t)tiles_x * tiles_y;
  const int64_t n_tiles_all = tiles_per_slot * views->n_slots;
  GS_REQUIRE(n_tiles_all <= (int64_t)0xFFFFFFFFll,
             "gs_bin_sort: %lld tiles per slot x %d slots exceed 32-bit tile indices",
             (long long)tiles_per_slot, views->n_slots);
  // passes over the tile bits of the keys (the depth order comes from the
  // presort of the pairs)
  int tile_bits = 0;
  while ((int64_t(1) << tile_bits) < n_tiles_all) ++tile_bits;
  // 17-18 tile bits (e.g. 8x8 tiles of one 3840x2160 image): two 9-bit passes
  // instead of three 8-bit ones
  const int rb = (tile_bits > 2 * kRadixBits && tile_bits <= 2 * kRadixBitsMax) ? kRadixBitsMax
                                                                                : kRadixBits;
  const int passes = (tile_bits + rb - 1) / rb;
  // emit into the buffer that the last pass will not overwrite
  uint32_t* v0 = (passes % 2 == 0) ? ids_out : vals_alt;
  uint32_t* v1 = (passes % 2 == 0) ? vals_alt : ids_out;
  uint32_t* emit_alt = (uint32_t*)(w + L.off_emit_alt);
  uint32_t* e0 = emit_out ? ((passes % 2 == 0) ? emit_out : emit_alt) : nullptr;
  uint32_t* e1 = emit_out ? ((passes % 2 == 0) ? emit_alt : emit_out) : nullptr;

  if (m == 0) {
    st = gs_zero(tile_ranges, sizeof(uint32_t) * 2 * (size_t)n_tiles_all, stream);
    if (st != GS_OK) return st;
    st = gs_zero(count, sizeof(int64_t) * 2, stream);
    if (st != GS_OK) return st;
    if (status) {
      // status[1] = 0 duplicates; flags untouched
      st = gs_zero(status + 1, sizeof(int64_t), stream);
      if (st != GS_OK) return st;
    }
    return GS_OK;
  }
  // depth presort of the m pairs: 4 stable passes over the depth bits,
  // ping-pong ending in buffer 0
  uint32_t* pk[2] = {(uint32_t*)(w + L.off_pkeys[0]), (uint32_t*)(w + L.off_pkeys[1])};
  uint8_t* nt8 = (uint8_t*)(w + L.off_nt8);
  uint32_t* pv[2] = {(uint32_t*)(w + L.off_pvals[0]), (uint32_t*)(w + L.off_pvals[1])};
  int64_t* count_pairs = count + 1;
  uint4* erec = (uint4*)(w + L.off_erec);
  hipLaunchKernelGGL(k_depth_keys, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, s, proj->rec,
                     proj->n_tiles, (const uint2*)proj->tile_bbox, tiling->tile_w,
                     tiling->tile_h, tiles_x, (int)tiles_per_slot, m, pk[0], nt8, erec,
                     pair_first, count_pairs, tile_ranges, 2 * n_tiles_all);
  GS_LAUNCH_CHECK("gs_bin_sort/depth_keys");
  for (int p = 0; p < 4; ++p) {
    const int shift = p * kRadixBits;
    const int a = p & 1, b = a ^ 1;
    launch_hist<kRadixBits>(pk[a], count_pairs, shift, L.nb_pairs, hist, s);
    GS_LAUNCH_CHECK("gs_bin_sort/depth_hist");
    launch_rowscan(hist, L.nb_pairs, count_pairs, rowtot, kRadix, s);
    GS_LAUNCH_CHECK("gs_bin_sort/depth_rowscan");
    // (the first pass numbers the pairs itself: values in = NULL)
    launch_scatter<kRadixBits>(pk[a], p == 0 ? nullptr : pv[a], pk[b], pv[b], count_pairs, shift,
                               L.nb_pairs, hist, rowtot, (const uint32_t*)nullptr,
                               (uint32_t*)nullptr, s);
    GS_LAUNCH_CHECK("gs_bin_sort/depth_scatter");
  }
  // duplicates in depth order, then stable passes over the tile bits only
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)L.nb_scan), dim3(kScanThreads), 0, s, pv[0],
                     (const uint8_t*)nt8, (const uint4*)erec, m, block_sums);
  GS_LAUNCH_CHECK("gs_bin_sort/scan_reduce");
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, block_sums, L.nb_scan,
                     dup_capacity, status, count);
  GS_LAUNCH_CHECK("gs_bin_sort/scan_top");
  if (keys_out) {
    uint64_t* k0 = (passes % 2 == 0) ? keys_out : keys_alt;
    uint64_t* k1 = (passes % 2 == 0) ? keys_alt : keys_out;
    return tile_phase<uint64_t>(k0, k1, v0, v1, e0, e1, 32, rb, passes, erec, pk[0], pv[0], m,
                                block_sums, dup_capacity, tiles_x, (int)tiles_per_slot,
                                pair_first, count, L, hist, rowtot, tile_ranges, s);
  }
  // no keys asked for: 32-bit tile keys in the two halves of keys_alt
  uint32_t* t0 = reinterpret_cast<uint32_t*>(keys_alt);
  uint32_t* t1 = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(keys_alt) +
                                             align256(sizeof(uint32_t) * (size_t)dup_capacity));
  return tile_phase<uint32_t>(t0, t1, v0, v1, e0, e1, 0, rb, passes, erec, pk[0], pv[0], m,
                              block_sums, dup_capacity, tiles_x, (int)tiles_per_slot, pair_first,
                              count, L, hist, rowtot, tile_ranges, s);
}

}  // extern "C"
