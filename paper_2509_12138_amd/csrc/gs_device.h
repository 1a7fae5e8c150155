// gs_device.h — internal helpers of libgsmi (gfx950 / CDNA4, wave64).
//
// Host side: thread-local error text, argument checks, launch checks.
// Device side: wave64 DPP reductions, the splat evaluation shared by the
// forward and backward rasterisers (so both take bit-identical decisions),
// and the method's constants in FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include "gs.h"

namespace gsmi {

// ----------------------------------------------------------------- host side

void set_error(const char* fmt, ...);
void clear_error();

#define GS_REQUIRE(cond, ...)            \
  do {                                   \
    if (!(cond)) {                       \
      ::gsmi::set_error(__VA_ARGS__);    \
      return GS_ERR_ARG;                 \
    }                                    \
  } while (0)

#define GS_LAUNCH_CHECK(what)                                                   \
  do {                                                                          \
    hipError_t _e = hipGetLastError();                                          \
    if (_e != hipSuccess) {                                                     \
      ::gsmi::set_error("%s: %s", (what), hipGetErrorString(_e));               \
      return GS_ERR_HIP;                                                        \
    }                                                                           \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Validates a gs_views / gs_tiling pair; returns GS_OK or GS_ERR_ARG.
gs_status check_views(const gs_views* v, const gs_tiling* t, const char* who);

// Number of compute units of the current device (cached per device).
int device_cu_count();

// ----------------------------------------------------------------- constants

constexpr float kC0 = 0.28209479177387814f;      // degree-0 SH basis 1/(2 sqrt(pi))
constexpr float kDilate = 0.3f;                  // 2D covariance low-pass (px^2)
constexpr float kFrustum = 1.3f;                 // Jacobian clamp factor
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// ----------------------------------------------------------------- device side

// DPP lane moves within a wave64 (GFX9 DPP controls).  Lanes that read an
// invalid source or whose row is masked off receive 0.
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK,
                                         BANK_MASK, false));
}

constexpr int kDppQuadSwap1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppQuadSwap2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppRowRor4 = 0x124;    // row_ror:4
constexpr int kDppRowRor8 = 0x128;    // row_ror:8
constexpr int kDppRowHalfMirror = 0x141;  // row_half_mirror (l <-> 7 - l in 8 lanes)
constexpr int kDppRowBcast15 = 0x142; // row_bcast:15
constexpr int kDppRowBcast31 = 0x143; // row_bcast:31

// Sum over the 64 lanes of a wave; the total is valid in lane 63.
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
  v += dpp_f<kDppQuadSwap1>(v);
  v += dpp_f<kDppQuadSwap2>(v);
  v += dpp_f<kDppRowRor4>(v);
  v += dpp_f<kDppRowRor8>(v);
  v += dpp_f<kDppRowBcast15, 0xa>(v);
  v += dpp_f<kDppRowBcast31, 0xc>(v);
  return v;
}

__device__ __forceinline__ float lane63(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

__device__ __forceinline__ float wave_sum(float v) { return lane63(wave_sum_to_lane63(v)); }

// A Gaussian as staged in LDS for the rasterisers: mean, log2-scaled conic
// (A, B, C) so that log2 of the Gaussian falloff is A dx^2 + B dx dy + C dy^2,
// opacity, colour and the log2-domain skip threshold thr = -log2(255 o):
// o 2^p2 < 1/255 exactly when p2 < thr, so skipped entries never reach exp.
// The first six words are what the skip test reads.
struct alignas(16) Splat {
  float mx, my, A, B, C, thr, o, r, g, b, pad1, pad2;
};

// log2-domain falloff exponents of the PX pixels a lane owns in one column
// (same dx, rows fy[k]).  Explicit rounded operations keep the forward and
// backward kernels bit-identical, so their skip/stop decisions agree.
// Column terms of p2 shared by a lane's pixels: A dx^2 and B dx.
__device__ __forceinline__ float splat_adx2(const Splat& s, float dx) {
  return __fmul_rn(__fmul_rn(s.A, dx), dx);
}
__device__ __forceinline__ float splat_bdx(const Splat& s, float dx) { return __fmul_rn(s.B, dx); }

// p2 of one pixel of the column (row centre fy).
__device__ __forceinline__ float splat_p2_row(const Splat& s, float adx2, float bdx, float fy) {
  const float dy = __fsub_rn(fy, s.my);
  const float t = __fmaf_rn(s.C, dy, bdx);       // C dy + B dx
  return __fmaf_rn(dy, t, adx2);                 // A dx^2 + B dx dy + C dy^2
}

template <int PX>
__device__ __forceinline__ void splat_p2_column(const Splat& s, float dx, const float* fy,
                                                float* p2) {
  const float adx2 = splat_adx2(s, dx), bdx = splat_bdx(s, dx);
#pragma unroll
  for (int k = 0; k < PX; ++k) p2[k] = splat_p2_row(s, adx2, bdx, fy[k]);
}

// Entry passes the skip tests: falloff exponent <= 0 and alpha >= 1/255.
__device__ __forceinline__ bool splat_pass(const Splat& s, float p2) {
  return (p2 <= 0.0f) && (p2 >= s.thr);
}

// Conservative cull of a splat against the pixel centres of the box
// [x0, x1] x [y0, y1]: false only when every centre certainly fails the
// alpha test.  p2 is concave (A, C < 0), so its maximum over the box is 0
// when the mean lies inside, else the largest of the four edge maxima, each
// taken at the edge's stationary point clamped to the edge.  The margin
// 0.02 + 4e-6 M, with M bounding the magnitudes of the three terms of p2
// over the box, exceeds the FP32 rounding of this bound and of the
// per-pixel p2 together, so culling never changes a pixel's decision.
__device__ __forceinline__ bool splat_may_hit(const Splat& s, float x0, float x1, float y0,
                                              float y1) {
  const float dx0 = x0 - s.mx, dx1 = x1 - s.mx, dy0 = y0 - s.my, dy1 = y1 - s.my;
  if (dx0 <= 0.0f && dx1 >= 0.0f && dy0 <= 0.0f && dy1 >= 0.0f) return true;
  const float iA = -0.5f * __builtin_amdgcn_rcpf(s.A);    // -1 / (2A) > 0
  const float iC = -0.5f * __builtin_amdgcn_rcpf(s.C);
  float best = -INFINITY;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const float dy = e ? dy1 : dy0;                        // edge y = const
    const float dx = fminf(fmaxf(s.B * dy * iA, dx0), dx1);
    best = fmaxf(best, fmaf(fmaf(s.A, dx, s.B * dy), dx, s.C * dy * dy));
    const float ex = e ? dx1 : dx0;                        // edge x = const
    const float ey = fminf(fmaxf(s.B * ex * iC, dy0), dy1);
    best = fmaxf(best, fmaf(fmaf(s.C, ey, s.B * ex), ey, s.A * ex * ex));
  }
  const float X = fmaxf(fabsf(dx0), fabsf(dx1)), Y = fmaxf(fabsf(dy0), fabsf(dy1));
  const float M = fmaf(-s.A * X, X, fmaf(fabsf(s.B) * X, Y, -s.C * Y * Y));
  return best >= s.thr - fmaf(4e-6f, M, 0.02f);
}

// Unclamped alpha o * 2^p2; __builtin_amdgcn_exp2f is the hardware v_exp_f32.
__device__ __forceinline__ float splat_gauss(float p2) { return __builtin_amdgcn_exp2f(p2); }

// ----------------------------------------------------------------- Adam

// Learning rate and bias-correction factors of Adam step t (from 1): lr0
// decayed log-linearly towards lr_final over decay_steps when lr_final > 0
// (the 3D-GS position schedule).  Shared by every Adam kernel so that fused
// and separate updates agree bit for bit.
__device__ __forceinline__ void adam_schedule(int t, float b1, float b2, float lr0,
                                              float lr_final, int decay_steps, float& lr,
                                              float& ibc1, float& ibc2) {
  ibc1 = 1.0f / (1.0f - powf(b1, (float)t));
  ibc2 = 1.0f / (1.0f - powf(b2, (float)t));
  lr = lr0;
  if (lr_final > 0.0f && decay_steps > 0) {
    const float u = fminf((float)t / (float)decay_steps, 1.0f);
    lr = lr0 * expf(u * logf(lr_final / lr0));
  }
}

// One bias-corrected Adam update of a parameter p with gradient g.  No
// multiply-add contraction: which product a contraction would fuse depends
// on the surrounding code, and every kernel that steps Adam (the plain one
// and the fused projection backward) must round alike.
__device__ __forceinline__ void adam_update(float& p, float g, float& m, float& v, float lr,
                                            float ibc1, float ibc2, float b1, float b2,
                                            float eps) {
#pragma clang fp contract(off)
  m = b1 * m + (1.0f - b1) * g;
  v = b2 * v + (1.0f - b2) * g * g;
  const float mh = m * ibc1;
  const float vh = v * ibc2;
  p -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace gsmi
