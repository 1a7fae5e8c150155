// mlp.hip — learned initialisation: a 96 -> 64 -> 64 -> 8 ReLU network that
// maps 16-nearest-neighbour features of an isosurface point (the points of
// Sec. II "Isosurface Extraction") to the initial log-scale, rotation and
// opacity of its Gaussian.  BF16 weights and activations on the MFMA matrix
// cores, FP32 accumulation and biases; the FP32 master weights are rounded to
// bf16 when a work-group stages them in LDS.
//
// Products whose K runs over features or hidden units (the layers, and the
// backward's dZ W^T) use v_mfma_f32_16x16x32_bf16, lane l, j = 0..7:
//   A[m][k]: m = l % 16, k = 8 (l / 16) + j      (8 consecutive k per lane)
//   B[k][n]: n = l % 16, k = 8 (l / 16) + j
// The weight gradients, whose K runs over a tile's 16 points, and dY W3^T
// (K = 8 outputs) use v_mfma_f32_16x16x16_bf16, lane l, j = 0..3:
//   A[m][k]: m = l % 16, k = 4 (l / 16) + j      (4 consecutive k per lane)
//   B[k][n]: n = l % 16, k = 4 (l / 16) + j
// Both write C[m][n]: n = l % 16, m = 4 (l / 16) + j.  A C-layout fragment
// over 16 points is therefore, unchanged, the A operand of the transposed
// matrix with K = those 16 points, and also a B operand with K = those
// points: the weight-gradient products H^T dZ take both operands straight
// from registers; only the layer-to-layer hand-offs go through LDS.  One
// wave owns one 16-point tile at a time.
//
//   gs_mlp_features  16-NN offsets (divided by their mean distance) and
//                    neighbour normals in the point's local frame -> bf16 x
//   gs_mlp_fwd       y = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3
//   gs_mlp_bwd       parameter gradients (+ optional dx)
//   gs_mlp_targets   fitted Gaussians -> network targets (same frame/scale)
//   gs_mlp_loss      per-point loss against the targets and dL/dy
//   gs_mlp_apply     network output -> initial Gaussian parameters
#include <math.h>

#include "gs_device.h"

namespace gsmi {

constexpr int kIn = 96, kHid = 64, kOut = 8;
constexpr int kMlpWaves = 4;                       // waves per work-group
constexpr int kMlpThreads = 64 * kMlpWaves;
constexpr int kWSize = kIn * kHid + kHid * kHid + kHid * kOut;     // weight floats
constexpr int kBSize = kHid + kHid + kOut;                          // bias floats
constexpr int kPartial = kWSize + kBSize;                           // 10888
constexpr int kBwdBlockCap = 512;                  // bwd work-groups (partials)

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);                 // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Eight consecutive bf16 of row (row0 + l%16), columns k0 + 8(l/16) .. +7 of
// a row-major bf16 matrix in LDS with `stride` elements per row (16-B loads:
// stride and k0 are multiples of 8).
__device__ __forceinline__ bf16x8 frag8(const uint16_t* m, int stride, int row0, int k0) {
  const int l = threadIdx.x & 63;
  return *reinterpret_cast<const bf16x8*>(m + (row0 + (l & 15)) * stride + k0 + 8 * (l >> 4));
}

// Four consecutive bf16 of row (row0 + l%16), columns k0 + 4(l/16) .. +3 of a
// row-major bf16 matrix in LDS with `stride` elements per row.
__device__ __forceinline__ bf16x4 frag(const uint16_t* m, int stride, int row0, int k0) {
  const int l = threadIdx.x & 63;
  return *reinterpret_cast<const bf16x4*>(m + (row0 + (l & 15)) * stride + k0 + 4 * (l >> 4));
}

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
  bf16x4 r;
  r[0] = (short)f2bf(a);
  r[1] = (short)f2bf(b);
  r[2] = (short)f2bf(c);
  r[3] = (short)f2bf(d);
  return r;
}

// Orders this wave's LDS accesses (one wave reads what its other lanes wrote).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct MlpW {
  const float* w1;   // [96][64]  (input x output, row-major)
  const float* w2;   // [64][64]
  const float* w3;   // [64][8]
  const float* b1;
  const float* b2;
  const float* b3;
};

// Weights staged in LDS as bf16, in the layouts the fragments read:
//   w1t [64][96]  W1 transposed (B operand of layer 1)
//   w2t [64][64]  W2 transposed (B operand of layer 2)
//   w2n [64][64]  W2 as is       (B operand of dH1 = dZ2 W2^T)
//   w3t [16][64]  W3 transposed, rows >= 8 zero (B operand of layer 3)
//   w3n [64][16]  W3 as is, columns >= 8 zero (B operand of dH2 = dY W3^T)
struct MlpLds {
  uint16_t w1t[kHid * kIn];
  uint16_t w2t[kHid * kHid];
  uint16_t w2n[kHid * kHid];
  uint16_t w3t[16 * kHid];
  uint16_t w3n[kHid * 16];
  float b1[kHid], b2[kHid], b3[16];
};

// Per-wave scratch: the point tile's x, H1 (reused for dZ1), H2 and dZ2 as
// row-major bf16.
struct WaveLds {
  uint16_t x[16 * kIn];
  uint16_t h1[16 * kHid];
  uint16_t h2[16 * kHid];
  uint16_t dz2[16 * kHid];
};

constexpr int kSmemBytes = (int)(sizeof(MlpLds) + kMlpWaves * sizeof(WaveLds));
static_assert(kSmemBytes >= kPartial * 4, "block gradient reduction reuses the LDS");

__device__ void stage_weights(const MlpW& w, MlpLds& L) {
  for (int i = threadIdx.x; i < kIn * kHid; i += blockDim.x) {
    const int k = i / kHid, n = i % kHid;
    L.w1t[n * kIn + k] = f2bf(w.w1[i]);
  }
  for (int i = threadIdx.x; i < kHid * kHid; i += blockDim.x) {
    const int k = i / kHid, n = i % kHid;
    const uint16_t v = f2bf(w.w2[i]);
    L.w2t[n * kHid + k] = v;
    L.w2n[i] = v;
  }
  for (int i = threadIdx.x; i < 16 * kHid; i += blockDim.x) {
    const int n = i / kHid, k = i % kHid;      // w3t[n][k] = W3[k][n]
    L.w3t[i] = n < kOut ? f2bf(w.w3[k * kOut + n]) : (uint16_t)0;
    const int k2 = i / 16, n2 = i % 16;        // w3n[k2][n2] = W3[k2][n2]
    L.w3n[i] = n2 < kOut ? f2bf(w.w3[k2 * kOut + n2]) : (uint16_t)0;
  }
  for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
    L.b1[i] = w.b1[i];
    L.b2[i] = w.b2[i];
  }
  for (int i = threadIdx.x; i < 16; i += blockDim.x) L.b3[i] = i < kOut ? w.b3[i] : 0.0f;
  __syncthreads();
}

// x rows of one 16-point tile: 16 x 192 B = 192 x 16 B, three per lane
// (zero past the end), loaded into registers one tile ahead.
struct XRegs {
  uint4 v[3];
};

__device__ __forceinline__ void load_x(XRegs& r, const uint16_t* __restrict__ x, int64_t p0,
                                       int64_t n) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int i = l + 64 * s, row = i / 12, c = i % 12;
    r.v[s] = make_uint4(0u, 0u, 0u, 0u);
    if (p0 + row < n) r.v[s] = *reinterpret_cast<const uint4*>(x + (p0 + row) * kIn + 8 * c);
  }
}

__device__ __forceinline__ void store_x(const XRegs& r, uint16_t* xs) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int i = l + 64 * s;
    *reinterpret_cast<uint4*>(xs + (i / 12) * kIn + 8 * (i % 12)) = r.v[s];
  }
}

// Forward of the tile staged in Wv.x; z1/z2 keep the pre-activations (C
// layout), the bf16 activations are left in Wv.h1 / Wv.h2.
__device__ __forceinline__ void tile_forward(const MlpLds& L, WaveLds& Wv, f32x4 (&z1)[4],
                                             f32x4 (&z2)[4], f32x4& y) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) z1[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < kIn / 32; ++kt) {
    const bf16x8 a = frag8(Wv.x, kIn, 0, 32 * kt);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) z1[nt] = mfma32(a, frag8(L.w1t, kIn, 16 * nt, 32 * kt), z1[nt]);
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int col = 16 * nt + (l & 15);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      z1[nt][j] += L.b1[col];
      Wv.h1[(4 * (l >> 4) + j) * kHid + col] = f2bf(fmaxf(z1[nt][j], 0.0f));
    }
  }
  wave_lds_sync();
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) z2[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < kHid / 32; ++kt) {
    const bf16x8 a = frag8(Wv.h1, kHid, 0, 32 * kt);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) z2[nt] = mfma32(a, frag8(L.w2t, kHid, 16 * nt, 32 * kt), z2[nt]);
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int col = 16 * nt + (l & 15);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      z2[nt][j] += L.b2[col];
      Wv.h2[(4 * (l >> 4) + j) * kHid + col] = f2bf(fmaxf(z2[nt][j], 0.0f));
    }
  }
  wave_lds_sync();
  y = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < kHid / 32; ++kt)
    y = mfma32(frag8(Wv.h2, kHid, 0, 32 * kt), frag8(L.w3t, kHid, 0, 32 * kt), y);
#pragma unroll
  for (int j = 0; j < 4; ++j) y[j] += L.b3[l & 15];
}

__global__ __launch_bounds__(kMlpThreads) void k_mlp_fwd(const uint16_t* __restrict__ x, int64_t n,
                                                         MlpW w, float* __restrict__ y) {
  __shared__ __align__(16) unsigned char smem[kSmemBytes];
  MlpLds& L = *reinterpret_cast<MlpLds*>(smem);
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  WaveLds& S = reinterpret_cast<WaveLds*>(smem + sizeof(MlpLds))[wave];
  stage_weights(w, L);
  const int64_t tiles = (n + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * kMlpWaves;
  int64_t t = (int64_t)blockIdx.x * kMlpWaves + wave;
  XRegs nx;
  if (t < tiles) load_x(nx, x, t * 16, n);
  for (; t < tiles; t += stride) {
    store_x(nx, S.x);
    if (t + stride < tiles) load_x(nx, x, (t + stride) * 16, n);
    wave_lds_sync();
    f32x4 z1[4], z2[4], yy;
    tile_forward(L, S, z1, z2, yy);
    const int col = l & 15;
    if (col < kOut) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t p = t * 16 + 4 * (l >> 4) + j;
        if (p < n) y[p * kOut + col] = yy[j];
      }
    }
    wave_lds_sync();
  }
}

// Backward.  Each wave accumulates all parameter gradients over its tiles in
// registers (C layout); the block sums its waves in LDS in a fixed order and
// writes one partial per block to part[block][kPartial] in the order
// dW1 [96][64], dW2 [64][64], dW3 [64][8], db1, db2, db3.  With dx != NULL
// also dx = dZ1 W1^T [n][96] fp32.
template <bool WITH_DX>
__global__ __launch_bounds__(kMlpThreads) void k_mlp_bwd(const uint16_t* __restrict__ x, int64_t n,
                                                         MlpW w, const float* __restrict__ dy,
                                                         float* __restrict__ part,
                                                         float* __restrict__ dx) {
  __shared__ __align__(16) unsigned char smem[kSmemBytes];
  MlpLds& L = *reinterpret_cast<MlpLds*>(smem);
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  WaveLds& S = reinterpret_cast<WaveLds*>(smem + sizeof(MlpLds))[wave];
  stage_weights(w, L);
  f32x4 gw1[6][4], gw2[4][4], gw3[4];
  float gb1[4] = {0.f, 0.f, 0.f, 0.f}, gb2[4] = {0.f, 0.f, 0.f, 0.f}, gb3 = 0.f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    gw3[a] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 4; ++b) gw2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) gw1[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t tiles = (n + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * kMlpWaves;
  int64_t t = (int64_t)blockIdx.x * kMlpWaves + wave;
  XRegs nx;
  if (t < tiles) load_x(nx, x, t * 16, n);
  for (; t < tiles; t += stride) {
    const int64_t p0 = t * 16;
    store_x(nx, S.x);
    if (t + stride < tiles) load_x(nx, x, (t + stride) * 16, n);
    wave_lds_sync();
    f32x4 z1[4], z2[4], yy;
    tile_forward(L, S, z1, z2, yy);
    // dY rounded to bf16, as the A operand (points x outputs, K padded to 16)
    // and as the B operand (points x outputs) of dW3 = H2^T dY
    float da[4], db[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 4 * (l >> 4) + j;
      const int64_t pa = p0 + (l & 15);
      da[j] = (k < kOut && pa < n) ? dy[pa * kOut + k] : 0.0f;
      const int64_t pb = p0 + 4 * (l >> 4) + j;
      db[j] = ((l & 15) < kOut && pb < n) ? dy[pb * kOut + (l & 15)] : 0.0f;
    }
    const bf16x4 dyA = pack4(da[0], da[1], da[2], da[3]);
    const bf16x4 dyB = pack4(db[0], db[1], db[2], db[3]);
#pragma unroll
    for (int j = 0; j < 4; ++j) gb3 += bf2f((uint16_t)dyB[j]);
    // H2 and H1 in C layout, bf16: A operands of the transposed products
    bf16x4 h2c[4], h1c[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      h2c[nt] = pack4(fmaxf(z2[nt][0], 0.f), fmaxf(z2[nt][1], 0.f), fmaxf(z2[nt][2], 0.f),
                      fmaxf(z2[nt][3], 0.f));
      h1c[nt] = pack4(fmaxf(z1[nt][0], 0.f), fmaxf(z1[nt][1], 0.f), fmaxf(z1[nt][2], 0.f),
                      fmaxf(z1[nt][3], 0.f));
    }
    // dW3 += H2^T dY
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) gw3[mt] = mfma(h2c[mt], dyB, gw3[mt]);
    // dZ2 = (dY W3^T) * [z2 > 0]  (C layout), bf16
    bf16x4 dz2c[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const f32x4 d = mfma(dyA, frag(L.w3n, 16, 16 * nt, 0), f32x4{0.f, 0.f, 0.f, 0.f});
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = z2[nt][j] > 0.f ? d[j] : 0.f;
      dz2c[nt] = pack4(v[0], v[1], v[2], v[3]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        S.dz2[(4 * (l >> 4) + j) * kHid + 16 * nt + (l & 15)] = (uint16_t)dz2c[nt][j];
        gb2[nt] += bf2f((uint16_t)dz2c[nt][j]);
      }
    }
    // dW2 += H1^T dZ2
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) gw2[mt][nt] = mfma(h1c[mt], dz2c[nt], gw2[mt][nt]);
    wave_lds_sync();
    // dZ1 = (dZ2 W2^T) * [z1 > 0]
    bf16x4 dz1c[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 d = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kt = 0; kt < kHid / 32; ++kt)
        d = mfma32(frag8(S.dz2, kHid, 0, 32 * kt), frag8(L.w2n, kHid, 16 * nt, 32 * kt), d);
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = z1[nt][j] > 0.f ? d[j] : 0.f;
      dz1c[nt] = pack4(v[0], v[1], v[2], v[3]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        gb1[nt] += bf2f((uint16_t)dz1c[nt][j]);
        if (WITH_DX) S.h1[(4 * (l >> 4) + j) * kHid + 16 * nt + (l & 15)] = (uint16_t)dz1c[nt][j];
      }
    }
    // dW1 += X^T dZ1; X^T fragments: rows = inputs, k = the tile's points
#pragma unroll
    for (int mt = 0; mt < 6; ++mt) {
      const int col = 16 * mt + (l & 15);
      bf16x4 xa;
#pragma unroll
      for (int j = 0; j < 4; ++j) xa[j] = (short)S.x[(4 * (l >> 4) + j) * kIn + col];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) gw1[mt][nt] = mfma(xa, dz1c[nt], gw1[mt][nt]);
    }
    if (WITH_DX) {
      wave_lds_sync();
      // dX = dZ1 W1^T: B[k = hidden][n = input] = W1[n][k] = w1t[k][n]
#pragma unroll
      for (int nt = 0; nt < 6; ++nt) {
        f32x4 d = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < kHid / 32; ++kt) {
          bf16x8 b;
#pragma unroll
          for (int j = 0; j < 8; ++j)
            b[j] = __builtin_bit_cast(
                __bf16, L.w1t[(32 * kt + 8 * (l >> 4) + j) * kIn + 16 * nt + (l & 15)]);
          d = mfma32(frag8(S.h1, kHid, 0, 32 * kt), b, d);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t p = p0 + 4 * (l >> 4) + j;
          if (p < n) dx[p * kIn + 16 * nt + (l & 15)] = d[j];
        }
      }
    }
    wave_lds_sync();
  }
  // block sum in LDS, waves in a fixed order (deterministic)
  __syncthreads();
  float* acc = reinterpret_cast<float*>(smem);
  const int c = l & 15, r0 = 4 * (l >> 4);
  for (int wv = 0; wv < kMlpWaves; ++wv) {
    if (wave == wv) {
      const bool first = wv == 0;
#pragma unroll
      for (int mt = 0; mt < 6; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            float& a = acc[(16 * mt + r0 + j) * kHid + 16 * nt + c];
            a = first ? gw1[mt][nt][j] : a + gw1[mt][nt][j];
          }
      float* a2 = acc + kIn * kHid;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            float& a = a2[(16 * mt + r0 + j) * kHid + 16 * nt + c];
            a = first ? gw2[mt][nt][j] : a + gw2[mt][nt][j];
          }
      float* a3 = a2 + kHid * kHid;
      if (c < kOut)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            float& a = a3[(16 * mt + r0 + j) * kOut + c];
            a = first ? gw3[mt][j] : a + gw3[mt][j];
          }
      // biases: the four lane groups (l/16) of each column, then across waves
      float b1v[4], b2v[4], b3v = gb3;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        b1v[nt] = gb1[nt] + __shfl_xor(gb1[nt], 16, 64);
        b1v[nt] += __shfl_xor(b1v[nt], 32, 64);
        b2v[nt] = gb2[nt] + __shfl_xor(gb2[nt], 16, 64);
        b2v[nt] += __shfl_xor(b2v[nt], 32, 64);
      }
      b3v += __shfl_xor(b3v, 16, 64);
      b3v += __shfl_xor(b3v, 32, 64);
      float* ab = a3 + kHid * kOut;
      if (l < 16) {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          ab[16 * nt + l] = first ? b1v[nt] : ab[16 * nt + l] + b1v[nt];
          ab[kHid + 16 * nt + l] = first ? b2v[nt] : ab[kHid + 16 * nt + l] + b2v[nt];
        }
        if (l < kOut) ab[2 * kHid + l] = first ? b3v : ab[2 * kHid + l] + b3v;
      }
    }
    __syncthreads();
  }
  float* out = part + (int64_t)blockIdx.x * kPartial;
  for (int i = threadIdx.x; i < kPartial; i += kMlpThreads) out[i] = acc[i];
}

// Sum of the block partials, in block order, added into the caller's gradients.
struct MlpG {
  float* dw1;
  float* dw2;
  float* dw3;
  float* db1;
  float* db2;
  float* db3;
};

__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ part, int nparts,
                                                    MlpG g) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kPartial) return;
  float s = 0.f;
  for (int w = 0; w < nparts; ++w) s += part[(int64_t)w * kPartial + i];
  int o = i;
  if (o < kIn * kHid) { g.dw1[o] += s; return; }
  o -= kIn * kHid;
  if (o < kHid * kHid) { g.dw2[o] += s; return; }
  o -= kHid * kHid;
  if (o < kHid * kOut) { g.dw3[o] += s; return; }
  o -= kHid * kOut;
  if (o < kHid) { g.db1[o] += s; return; }
  o -= kHid;
  if (o < kHid) { g.db2[o] += s; return; }
  o -= kHid;
  g.db3[o] += s;
}

// ---------------------------------------------------------------- geometry

// Local frame of a point: z = unit normal, x = normal x (least aligned world
// axis, lowest index on ties), normalised, y = z x x.  Rows of F are the
// frame axes (world -> local).
__device__ __forceinline__ void local_frame(float nx, float ny, float nz, float F[9]) {
  const float inv = rsqrtf(fmaxf(nx * nx + ny * ny + nz * nz, 1e-30f));
  nx *= inv; ny *= inv; nz *= inv;
  const float ax = fabsf(nx), ay = fabsf(ny), az = fabsf(nz);
  float e0 = 0.f, e1 = 0.f, e2 = 0.f;
  if (ax <= ay && ax <= az) e0 = 1.f;
  else if (ay <= az) e1 = 1.f;
  else e2 = 1.f;
  float tx = ny * e2 - nz * e1, ty = nz * e0 - nx * e2, tz = nx * e1 - ny * e0;
  const float it = rsqrtf(tx * tx + ty * ty + tz * tz);
  tx *= it; ty *= it; tz *= it;
  F[0] = tx; F[1] = ty; F[2] = tz;
  F[3] = ny * tz - nz * ty; F[4] = nz * tx - nx * tz; F[5] = nx * ty - ny * tx;
  F[6] = nx; F[7] = ny; F[8] = nz;
}

__device__ __forceinline__ void quat_to_rotm(float w, float x, float y, float z, float R[9]) {
  const float qn = rsqrtf(fmaxf(w * w + x * x + y * y + z * z, 1e-30f));
  w *= qn; x *= qn; y *= qn; z *= qn;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

// Rotation matrix -> unit quaternion (w, x, y, z) with w >= 0, branching on
// the largest of the trace and the diagonal (Shepperd's method).
__device__ __forceinline__ void rotm_to_quat(const float R[9], float q[4]) {
  const float tr = R[0] + R[4] + R[8];
  float w, x, y, z;
  if (tr > 0.f) {
    const float s = 2.f * sqrtf(tr + 1.f);
    w = 0.25f * s; x = (R[7] - R[5]) / s; y = (R[2] - R[6]) / s; z = (R[3] - R[1]) / s;
  } else if (R[0] > R[4] && R[0] > R[8]) {
    const float s = 2.f * sqrtf(1.f + R[0] - R[4] - R[8]);
    w = (R[7] - R[5]) / s; x = 0.25f * s; y = (R[1] + R[3]) / s; z = (R[2] + R[6]) / s;
  } else if (R[4] > R[8]) {
    const float s = 2.f * sqrtf(1.f + R[4] - R[0] - R[8]);
    w = (R[2] - R[6]) / s; x = (R[1] + R[3]) / s; y = 0.25f * s; z = (R[5] + R[7]) / s;
  } else {
    const float s = 2.f * sqrtf(1.f + R[8] - R[0] - R[4]);
    w = (R[3] - R[1]) / s; x = (R[2] + R[6]) / s; y = (R[5] + R[7]) / s; z = 0.25f * s;
  }
  const float sg = w < 0.f ? -1.f : 1.f;
  const float qn = sg * rsqrtf(w * w + x * x + y * y + z * z);
  q[0] = w * qn; q[1] = x * qn; q[2] = y * qn; q[3] = z * qn;
}

// ---------------------------------------------------------------- features

// One thread per point.  Neighbour k (sorted by distance, index) fills
// x[6k .. 6k+2] = F (p_j - p) / dbar and x[6k+3 .. 6k+5] = F n_j; missing
// neighbours (index -1) are zero.  dbar = mean distance over the present
// neighbours (1 when there are none).
__global__ __launch_bounds__(256) void k_mlp_features(const float* __restrict__ pts,
                                                      const float* __restrict__ nrm, int64_t n,
                                                      const int32_t* __restrict__ idx,
                                                      const float* __restrict__ dist,
                                                      uint16_t* __restrict__ x,
                                                      float* __restrict__ dbar) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float F[9];
  local_frame(nrm[i], nrm[n + i], nrm[2 * n + i], F);
  float dm = 0.f;
  int cnt = 0;
  for (int k = 0; k < 16; ++k)
    if (idx[i * 16 + k] >= 0) {
      dm += dist[i * 16 + k];
      ++cnt;
    }
  dm = cnt > 0 ? dm / (float)cnt : 1.0f;
  dm = fmaxf(dm, 1e-30f);
  dbar[i] = dm;
  const float inv = 1.0f / dm;
  const float px = pts[i], py = pts[n + i], pz = pts[2 * n + i];
  uint4* xr = reinterpret_cast<uint4*>(x + i * kIn);
  // four neighbours = 24 bf16 = 48 B = 3 x 16 B
  for (int k4 = 0; k4 < 4; ++k4) {
    uint32_t wds[12];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int j = idx[i * 16 + 4 * k4 + kk];
      float f[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (j >= 0) {
        const float dx = (pts[j] - px) * inv, dy = (pts[n + j] - py) * inv,
                    dz = (pts[2 * n + j] - pz) * inv;
        const float mx = nrm[j], my = nrm[n + j], mz = nrm[2 * n + j];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          f[a] = F[3 * a] * dx + F[3 * a + 1] * dy + F[3 * a + 2] * dz;
          f[3 + a] = F[3 * a] * mx + F[3 * a + 1] * my + F[3 * a + 2] * mz;
        }
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
        wds[3 * kk + a] = (uint32_t)f2bf(f[2 * a]) | ((uint32_t)f2bf(f[2 * a + 1]) << 16);
    }
    xr[3 * k4 + 0] = make_uint4(wds[0], wds[1], wds[2], wds[3]);
    xr[3 * k4 + 1] = make_uint4(wds[4], wds[5], wds[6], wds[7]);
    xr[3 * k4 + 2] = make_uint4(wds[8], wds[9], wds[10], wds[11]);
  }
}

// ---------------------------------------------------------------- targets

// Fitted Gaussian -> network target in the point's frame and scale:
// t[0:3] = log s - log dbar, t[3:7] = quaternion of F R_fit (w >= 0),
// t[7] = opacity logit.
__global__ __launch_bounds__(256) void k_mlp_targets(const float* __restrict__ log_scale,
                                                     const float* __restrict__ quat,
                                                     const float* __restrict__ logit,
                                                     const float* __restrict__ nrm,
                                                     const float* __restrict__ dbar, int64_t n,
                                                     float* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float* ti = t + i * kOut;
  const float ld = logf(dbar[i]);
#pragma unroll
  for (int a = 0; a < 3; ++a) ti[a] = log_scale[a * n + i] - ld;
  ti[7] = logit[i];
  float F[9], Rg[9], Rl[9], q[4];
  local_frame(nrm[i], nrm[n + i], nrm[2 * n + i], F);
  quat_to_rotm(quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i], Rg);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      Rl[3 * r + c] = F[3 * r] * Rg[c] + F[3 * r + 1] * Rg[3 + c] + F[3 * r + 2] * Rg[6 + c];
  rotm_to_quat(Rl, q);
#pragma unroll
  for (int a = 0; a < 4; ++a) ti[3 + a] = q[a];
}

// ---------------------------------------------------------------- loss

// Per point: squared error of the 3 log-scale entries and the opacity logit,
// plus 1 - |<q/|q|, q*>| for the rotation (q* the unit target); the loss is
// the mean over points.  dy = dL/dy; block partial sums in part.
__global__ __launch_bounds__(256) void k_mlp_loss(const float* __restrict__ y,
                                                  const float* __restrict__ t, int64_t n,
                                                  float* __restrict__ dy,
                                                  float* __restrict__ part) {
  __shared__ float sm[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float L = 0.f;
  if (i < n) {
    const float* yi = y + i * kOut;
    const float* ti = t + i * kOut;
    float* di = dy + i * kOut;
    const float inv_n = 1.0f / (float)n;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float r = yi[a] - ti[a];
      L += r * r;
      di[a] = 2.f * r * inv_n;
    }
    const float r7 = yi[7] - ti[7];
    L += r7 * r7;
    di[7] = 2.f * r7 * inv_n;
    const float q0 = yi[3], q1 = yi[4], q2 = yi[5], q3 = yi[6];
    const float iq = 1.0f / fmaxf(sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3), 1e-12f);
    const float d = (q0 * ti[3] + q1 * ti[4] + q2 * ti[5] + q3 * ti[6]) * iq;   // <q^, q*>
    L += 1.f - fabsf(d);
    const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
    // d<q^,q*>/dq = (q* - q^ <q^,q*>) / |q|
    di[3] = -sg * (ti[3] - q0 * iq * d) * iq * inv_n;
    di[4] = -sg * (ti[4] - q1 * iq * d) * iq * inv_n;
    di[5] = -sg * (ti[5] - q2 * iq * d) * iq * inv_n;
    di[6] = -sg * (ti[6] - q3 * iq * d) * iq * inv_n;
  }
  L = wave_sum(L);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = L;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
}

__global__ __launch_bounds__(256) void k_mlp_loss_final(const float* __restrict__ part, int64_t nb,
                                                        int64_t n, float* __restrict__ loss) {
  __shared__ double sm[256];
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += 256) s += part[b];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) sm[threadIdx.x] += sm[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(sm[0] / (double)n);
}

// ---------------------------------------------------------------- apply

// Network output -> Gaussian: log s = log dbar + y[0:3], rotation F^T R(y[3:7])
// (the frame's axes as columns times the local rotation), quaternion with
// w >= 0, opacity logit y[7].  Planar SoA outputs.
__global__ __launch_bounds__(256) void k_mlp_apply(const float* __restrict__ y,
                                                   const float* __restrict__ nrm,
                                                   const float* __restrict__ dbar, int64_t n,
                                                   float* __restrict__ log_scale,
                                                   float* __restrict__ quat,
                                                   float* __restrict__ logit) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float* yi = y + i * kOut;
  const float ld = logf(dbar[i]);
#pragma unroll
  for (int a = 0; a < 3; ++a) log_scale[a * n + i] = ld + yi[a];
  logit[i] = yi[7];
  float F[9], Rl[9], R[9], q[4];
  local_frame(nrm[i], nrm[n + i], nrm[2 * n + i], F);
  quat_to_rotm(yi[3], yi[4], yi[5], yi[6], Rl);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      R[3 * r + c] = F[r] * Rl[c] + F[3 + r] * Rl[3 + c] + F[6 + r] * Rl[6 + c];
  rotm_to_quat(R, q);
#pragma unroll
  for (int a = 0; a < 4; ++a) quat[a * n + i] = q[a];
}

static unsigned mlp_blocks(int64_t n, int64_t cap) {
  const int64_t tiles = (n + 15) / 16;
  const int64_t b = (tiles + kMlpWaves - 1) / kMlpWaves;
  return (unsigned)(b < cap ? (b > 0 ? b : 1) : cap);
}

static gs_status mlp_check(const gs_mlp* w, const char* who) {
  GS_REQUIRE(w && w->w1 && w->w2 && w->w3 && w->b1 && w->b2 && w->b3, "%s: NULL weights", who);
  return GS_OK;
}

}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_mlp_features(const float* pts, const float* normals, int64_t n, const int32_t* knn_idx,
                          const float* knn_dist, uint16_t* x_bf16, float* dbar, void* stream) {
  clear_error();
  GS_REQUIRE(n >= 0 && n < (int64_t(1) << 31), "gs_mlp_features: n=%lld outside [0, 2^31)",
             (long long)n);
  if (n == 0) return GS_OK;
  GS_REQUIRE(pts && normals && knn_idx && knn_dist && x_bf16 && dbar,
             "gs_mlp_features: NULL argument");
  GS_REQUIRE(((uintptr_t)x_bf16 & 15) == 0, "gs_mlp_features: x must be 16-byte aligned");
  hipLaunchKernelGGL(k_mlp_features, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0,
                     as_stream(stream), pts, normals, n, knn_idx, knn_dist, x_bf16, dbar);
  GS_LAUNCH_CHECK("gs_mlp_features");
  return GS_OK;
}

gs_status gs_mlp_fwd(const uint16_t* x_bf16, int64_t n, const gs_mlp* w, float* y, void* stream) {
  clear_error();
  gs_status st = mlp_check(w, "gs_mlp_fwd");
  if (st != GS_OK) return st;
  GS_REQUIRE(n >= 0, "gs_mlp_fwd: n < 0");
  if (n == 0) return GS_OK;
  GS_REQUIRE(x_bf16 && y, "gs_mlp_fwd: NULL x/y");
  GS_REQUIRE(((uintptr_t)x_bf16 & 15) == 0, "gs_mlp_fwd: x must be 16-byte aligned");
  MlpW W{w->w1, w->w2, w->w3, w->b1, w->b2, w->b3};
  hipLaunchKernelGGL(k_mlp_fwd, dim3(mlp_blocks(n, (int64_t)device_cu_count() * 8)),
                     dim3(kMlpThreads), 0, as_stream(stream), x_bf16, n, W, y);
  GS_LAUNCH_CHECK("gs_mlp_fwd");
  return GS_OK;
}

size_t gs_mlp_bwd_workspace_bytes(int64_t n) {
  return sizeof(float) * (size_t)kPartial * (size_t)mlp_blocks(n > 0 ? n : 1, kBwdBlockCap);
}

gs_status gs_mlp_bwd(const uint16_t* x_bf16, int64_t n, const gs_mlp* w, const float* dy,
                     gs_mlp_grads* g, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  gs_status st = mlp_check(w, "gs_mlp_bwd");
  if (st != GS_OK) return st;
  GS_REQUIRE(n >= 0, "gs_mlp_bwd: n < 0");
  GS_REQUIRE(g && g->dw1 && g->dw2 && g->dw3 && g->db1 && g->db2 && g->db3,
             "gs_mlp_bwd: NULL gradient");
  if (n == 0) return GS_OK;
  GS_REQUIRE(x_bf16 && dy && ws, "gs_mlp_bwd: NULL argument");
  GS_REQUIRE(((uintptr_t)x_bf16 & 15) == 0, "gs_mlp_bwd: x must be 16-byte aligned");
  GS_REQUIRE(ws_bytes >= gs_mlp_bwd_workspace_bytes(n), "gs_mlp_bwd: workspace %zu < %zu bytes",
             ws_bytes, gs_mlp_bwd_workspace_bytes(n));
  const unsigned blocks = mlp_blocks(n, kBwdBlockCap);
  MlpW W{w->w1, w->w2, w->w3, w->b1, w->b2, w->b3};
  hipStream_t s = as_stream(stream);
  if (g->dx)
    hipLaunchKernelGGL(k_mlp_bwd<true>, dim3(blocks), dim3(kMlpThreads), 0, s, x_bf16, n, W, dy,
                       (float*)ws, g->dx);
  else
    hipLaunchKernelGGL(k_mlp_bwd<false>, dim3(blocks), dim3(kMlpThreads), 0, s, x_bf16, n, W, dy,
                       (float*)ws, (float*)nullptr);
  GS_LAUNCH_CHECK("gs_mlp_bwd");
  MlpG G{g->dw1, g->dw2, g->dw3, g->db1, g->db2, g->db3};
  hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)ceil_div(kPartial, 256)), dim3(256), 0, s,
                     (const float*)ws, (int)blocks, G);
  GS_LAUNCH_CHECK("gs_mlp_bwd/reduce");
  return GS_OK;
}

gs_status gs_mlp_targets(const float* log_scale, const float* quat, const float* opacity_logit,
                         const float* normals, const float* dbar, int64_t n, float* target,
                         void* stream) {
  clear_error();
  GS_REQUIRE(n >= 0, "gs_mlp_targets: n < 0");
  if (n == 0) return GS_OK;
  GS_REQUIRE(log_scale && quat && opacity_logit && normals && dbar && target,
             "gs_mlp_targets: NULL argument");
  hipLaunchKernelGGL(k_mlp_targets, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0,
                     as_stream(stream), log_scale, quat, opacity_logit, normals, dbar, n, target);
  GS_LAUNCH_CHECK("gs_mlp_targets");
  return GS_OK;
}

size_t gs_mlp_loss_workspace_bytes(int64_t n) {
  return sizeof(float) * (size_t)ceil_div(n > 0 ? n : 1, 256);
}

gs_status gs_mlp_loss(const float* y, const float* target, int64_t n, float* dy, void* ws,
                      size_t ws_bytes, float* loss_out, void* stream) {
  clear_error();
  GS_REQUIRE(n >= 1, "gs_mlp_loss: n < 1");
  GS_REQUIRE(y && target && dy && ws && loss_out, "gs_mlp_loss: NULL argument");
  GS_REQUIRE(ws_bytes >= gs_mlp_loss_workspace_bytes(n), "gs_mlp_loss: workspace too small");
  const int64_t nb = ceil_div(n, 256);
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(k_mlp_loss, dim3((unsigned)nb), dim3(256), 0, s, y, target, n, dy, (float*)ws);
  GS_LAUNCH_CHECK("gs_mlp_loss");
  hipLaunchKernelGGL(k_mlp_loss_final, dim3(1), dim3(256), 0, s, (const float*)ws, nb, n, loss_out);
  GS_LAUNCH_CHECK("gs_mlp_loss/final");
  return GS_OK;
}

gs_status gs_mlp_apply(const float* y, const float* normals, const float* dbar, int64_t n,
                       float* log_scale, float* quat, float* opacity_logit, void* stream) {
  clear_error();
  GS_REQUIRE(n >= 0, "gs_mlp_apply: n < 0");
  if (n == 0) return GS_OK;
  GS_REQUIRE(y && normals && dbar && log_scale && quat && opacity_logit,
             "gs_mlp_apply: NULL argument");
  hipLaunchKernelGGL(k_mlp_apply, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0,
                     as_stream(stream), y, normals, dbar, n, log_scale, quat, opacity_logit);
  GS_LAUNCH_CHECK("gs_mlp_apply");
  return GS_OK;
}

}  // extern "C"
