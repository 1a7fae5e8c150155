// loss.hip — background-masked L1 + D-SSIM photometric loss and its image
// gradient (masks: the paper's Sec. II "Image Rendering and Masking" and
// Sec. III-A; L1 + D-SSIM: the 3D-GS training loss it trains with).
//
// One work-group per (image, channel, 32x32 output tile), one kernel for
// the loss terms and the gradient: the masked image and target are staged
// with a 10-pixel halo (zero outside the image); the five moment maps are
// blurred with the separable 11-tap window over the 42x42 positions whose
// SSIM terms reach the tile's pixels; the three per-position partials
// dS/dmu_x, dS/dE[x^2], dS/dE[xy] (zero outside the image) are blurred again
// with the same symmetric window, which is the adjoint of the forward blur,
// and combined with the L1 subgradient into d loss / d image.  The block
// sums of S and |x - y| over the tile go to a partials array;
// k_loss_final sums them per image in FP64.  Every blur pass keeps several
// outputs per thread in registers, so each staged value is read from LDS
// once per thread rather than once per tap.
#include <math.h>

#include <mutex>
#include <vector>

#include "gs_device.h"

namespace gsmi {

constexpr int kLT = 32;               // output tile edge
constexpr int kLR = 5;                // window radius
constexpr int kLTaps = 2 * kLR + 1;
constexpr int kLM = kLT + 2 * kLR;    // 42: positions with SSIM terms reaching the tile
constexpr int kLS = kLM + 2 * kLR;    // 52: staged edge
constexpr int kLThreads = 256;
// LDS row strides (odd: consecutive rows start in different banks)
constexpr int kLSs = kLS + 1;         // staged image / target
constexpr int kLMs = kLM + 1;         // horizontal moments, partials
constexpr int kLTs = kLT + 1;         // horizontal pass of the partials
// register blocking of the four passes
constexpr int kH1 = 3;                // moments, horizontal: 3 columns per item
constexpr int kV1 = 7;                // moments, vertical: 7 rows per item
constexpr int kH2 = 4;                // partials, horizontal: 4 columns per item
constexpr int kV2 = 4;                // partials, vertical: 4 rows per item
static_assert(kLM % kH1 == 0 && kLM % kV1 == 0 && kLT % kH2 == 0 && kLT % kV2 == 0, "blocking");
static_assert((kLM / kV1) * kLM <= kLThreads && (kLT / kV2) * kLT == kLThreads, "blocking");

struct Window {
  float w[kLTaps];
};

static Window ssim_window() {
  double w[kLTaps], s = 0;
  for (int k = 0; k < kLTaps; ++k) {
    double d = k - kLR;
    w[k] = exp(-d * d / (2.0 * 1.5 * 1.5));
    s += w[k];
  }
  Window W;
  for (int k = 0; k < kLTaps; ++k) W.w[k] = (float)(w[k] / s);
  return W;
}

struct LossLayout {
  int64_t tiles_x, tiles_y, blocks_per_img;
  size_t off_part, total;
};

static LossLayout loss_layout(int S, int H, int W) {
  LossLayout L;
  L.tiles_x = ceil_div(W, kLT);
  L.tiles_y = ceil_div(H, kLT);
  L.blocks_per_img = L.tiles_x * L.tiles_y;
  L.off_part = 0;
  size_t part = sizeof(float) * 2 * 3 * (size_t)S * L.blocks_per_img;
  L.total = (part + 255) & ~size_t(255);
  return L;
}

// LDS: region A holds the staged image and target, later the partials;
// region B the horizontal moment sums, later the horizontal pass of the
// partials.
constexpr int kLRegionA = (2 * kLS * kLSs > 3 * kLM * kLMs) ? 2 * kLS * kLSs : 3 * kLM * kLMs;
constexpr int kLMom = 6;              // blurred moments: x, y, xx, yy, xy, foreground
constexpr int kLRegionB = (kLMom * kLS * kLMs > 3 * kLM * kLTs) ? kLMom * kLS * kLMs
                                                                 : 3 * kLM * kLTs;

template <bool MASK>
__global__ __launch_bounds__(kLThreads) void k_ssim(
    const float* __restrict__ image, const float* __restrict__ target,
    const uint8_t* __restrict__ mask, int H, int W, int64_t tiles_x, int64_t blocks_per_img,
    Window win, float l1_coef, float ssim_coef, float* __restrict__ d_image,
    float* __restrict__ part) {
  __shared__ float sA[kLRegionA];
  __shared__ float sB[kLRegionB];
  __shared__ float s_red[3][kLThreads / 64];
  const int64_t ic = blockIdx.x / blocks_per_img;          // image * 3 + channel
  const int64_t img = ic / 3;
  const int64_t b = blockIdx.x - ic * blocks_per_img;
  const int ty = (int)(b / tiles_x), tx = (int)(b - (int64_t)ty * tiles_x);
  const int ox = tx * kLT, oy = ty * kLT;                  // tile origin
  const int t = threadIdx.x;
  const int64_t HW = (int64_t)H * W;
  const float* I = image + ic * HW;
  const float* G = target + ic * HW;
  const uint8_t* Mk = MASK ? mask + img * HW : nullptr;
  float* s_x = sA;                  // [kLS][kLSs], staged row r = image row oy - 10 + r
  float* s_y = sA + kLS * kLSs;
  float* s_h = sB;                  // [5][kLS][kLMs]
  float* s_p = sA;                  // [3][kLM][kLMs], position row r = image row oy - 5 + r
  float* s_g = sB;                  // [3][kLM][kLTs]

  // stage the masked image and target with their foreground pixels shifted
  // by the foreground means (x'' = M (x - sx)): variances and the covariance
  // follow from moments of the shifted values and the blurred mask without
  // the cancellation of E[x^2] - mu^2 where the images are smooth.  A
  // background pixel (mask 0 or outside the image: zero padding) is staged
  // as -0.0, a foreground one never is ((x - sx) + 0 is +0 when x = sx), so
  // the sign bit of a staged zero carries the mask.  Every load reads a
  // clamped, valid address and the value is dropped afterwards if it lies
  // outside, so all loads of a thread are in flight together.
  constexpr int kStage = kLS * kLS;
  constexpr int kStageQ = (kStage + kLThreads - 1) / kLThreads;
  bool fg = false;      // a foreground pixel among the inputs of the tile's SSIM terms
  float shx, shy;       // the shifts of image and target
  {
    float iv[kStageQ], gv[kStageQ];
    uint8_t mv[kStageQ];
    bool ok[kStageQ];
#pragma unroll
    for (int q = 0; q < kStageQ; ++q) {
      const int i = min(t + q * kLThreads, kStage - 1);
      const int r = i / kLS, c = i - r * kLS;
      const int y = oy - 2 * kLR + r, x = ox - 2 * kLR + c;
      ok[q] = x >= 0 && x < W && y >= 0 && y < H && t + q * kLThreads < kStage;
      const int64_t o = (int64_t)min(max(y, 0), H - 1) * W + min(max(x, 0), W - 1);
      mv[q] = MASK ? Mk[o] : (uint8_t)1;
      iv[q] = I[o];
      gv[q] = G[o];
    }
    float sx = 0.f, sy = 0.f, sn = 0.f;
#pragma unroll
    for (int q = 0; q < kStageQ; ++q) {
      const float mk = (ok[q] && mv[q] != 0) ? 1.0f : 0.0f;
      iv[q] *= mk;
      gv[q] *= mk;
      sx += iv[q];
      sy += gv[q];
      sn += mk;
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    sn = wave_sum(sn);
    if ((t & 63) == 0) {
      s_red[0][t >> 6] = sx;
      s_red[1][t >> 6] = sy;
      s_red[2][t >> 6] = sn;
    }
    __syncthreads();
    float tx_ = 0.f, ty_ = 0.f, tn = 0.f;
#pragma unroll
    for (int w = 0; w < kLThreads / 64; ++w) {
      tx_ += s_red[0][w];
      ty_ += s_red[1][w];
      tn += s_red[2][w];
    }
    shx = tn > 0.f ? tx_ / tn : 0.f;
    shy = tn > 0.f ? ty_ / tn : 0.f;
#pragma unroll
    for (int q = 0; q < kStageQ; ++q) {
      const int i = t + q * kLThreads;
      if (i >= kStage) continue;
      const int r = i / kLS, c = i - r * kLS;
      const bool f = ok[q] && mv[q] != 0;
      s_x[r * kLSs + c] = f ? (iv[q] - shx) + 0.0f : -0.0f;
      s_y[r * kLSs + c] = f ? (gv[q] - shy) + 0.0f : -0.0f;
      fg = fg || (f && r >= kLR && r < kLS - kLR && c >= kLR && c < kLS - kLR);
    }
  }
  if (!__syncthreads_or(fg)) {
    // background tile: the mask is zero over the 42x42 inputs of the tile's
    // SSIM terms, so both masked images are zero there: each term is 1 (the
    // blurs of zeros are zero), the L1 terms are 0 and so is the gradient
    // (the mask is zero at the tile's own pixels).  Write that directly.
    float* D = d_image + ic * HW;
    float cnt = 0.f;
    for (int i = t; i < kLT * kLT; i += kLThreads) {
      const int y = oy + i / kLT, x = ox + i % kLT;
      if (x < W && y < H) {
        D[(int64_t)y * W + x] = 0.0f;
        cnt += 1.0f;
      }
    }
    cnt = wave_sum(cnt);
    if ((t & 63) == 0) s_red[0][t >> 6] = cnt;
    __syncthreads();
    if (t == 0) {
      float a0 = 0.f;
#pragma unroll
      for (int w = 0; w < kLThreads / 64; ++w) a0 += s_red[0][w];
      part[2 * blockIdx.x] = a0;
      part[2 * blockIdx.x + 1] = 0.0f;
    }
    return;
  }

  // moments, horizontal: staged row r, positions c0 .. c0 + kH1 - 1
  constexpr int kItems1 = kLS * (kLM / kH1);
  for (int it = t; it < kItems1; it += kLThreads) {
    const int r = it / (kLM / kH1), c0 = (it - r * (kLM / kH1)) * kH1;
    float acc[kH1][kLMom];
#pragma unroll
    for (int u = 0; u < kH1; ++u)
#pragma unroll
      for (int q = 0; q < kLMom; ++q) acc[u][q] = 0.f;
#pragma unroll
    for (int j = 0; j < kH1 + 2 * kLR; ++j) {
      const float xv = s_x[r * kLSs + c0 + j], yv = s_y[r * kLSs + c0 + j];
      const float xx = xv * xv, yy = yv * yv, xy = xv * yv;
      const float mk = __float_as_uint(xv) == 0x80000000u ? 0.f : 1.f;
#pragma unroll
      for (int u = 0; u < kH1; ++u) {
        const int k = j - u;
        if (k < 0 || k > 2 * kLR) continue;
        const float w = win.w[k];
        acc[u][0] = fmaf(w, xv, acc[u][0]);
        acc[u][1] = fmaf(w, yv, acc[u][1]);
        acc[u][2] = fmaf(w, xx, acc[u][2]);
        acc[u][3] = fmaf(w, yy, acc[u][3]);
        acc[u][4] = fmaf(w, xy, acc[u][4]);
        acc[u][5] = fmaf(w, mk, acc[u][5]);
      }
    }
#pragma unroll
    for (int u = 0; u < kH1; ++u)
#pragma unroll
      for (int q = 0; q < kLMom; ++q) s_h[(q * kLS + r) * kLMs + c0 + u] = acc[u][q];
  }
  __syncthreads();

  // moments, vertical, then SSIM and its partials at positions (r0 + u, c)
  float ssum = 0.f;
  if (t < (kLM / kV1) * kLM) {
    const int c = t % kLM, r0 = (t / kLM) * kV1;
    float m[kV1][kLMom];
#pragma unroll
    for (int u = 0; u < kV1; ++u)
#pragma unroll
      for (int q = 0; q < kLMom; ++q) m[u][q] = 0.f;
#pragma unroll
    for (int j = 0; j < kV1 + 2 * kLR; ++j) {
      float h[kLMom];
#pragma unroll
      for (int q = 0; q < kLMom; ++q) h[q] = s_h[(q * kLS + r0 + j) * kLMs + c];
#pragma unroll
      for (int u = 0; u < kV1; ++u) {
        const int k = j - u;
        if (k < 0 || k > 2 * kLR) continue;
#pragma unroll
        for (int q = 0; q < kLMom; ++q) m[u][q] = fmaf(win.w[k], h[q], m[u][q]);
      }
    }
    const int x = ox - kLR + c;
    const bool colin = x >= 0 && x < W;
    const bool colc = c >= kLR && c < kLR + kLT;
    float P[kV1][3];
#pragma unroll
    for (int u = 0; u < kV1; ++u) {
      const int y = oy - kLR + r0 + u;
      const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
      // moments of the shifted values (mu', E') and the blurred mask wt,
      // om = 1 - wt (x = x'' + s M with M^2 = M and x'' M = x''):
      //   mu = mu' + s wt,  var = E'xx - mu'^2 + om (2 s mu' + s^2 wt),
      //   cov = E'xy - mu'x mu'y + om (sy mu'x + sx mu'y + sx sy wt)
      const float wt = m[u][5], om = 1.f - wt;
      const float ux = m[u][0], uy = m[u][1];
      const float mx = fmaf(shx, wt, ux), my = fmaf(shy, wt, uy);
      const float vx = (m[u][2] - ux * ux) + om * (2.f * shx * ux + shx * shx * wt);
      const float vy = (m[u][3] - uy * uy) + om * (2.f * shy * uy + shy * shy * wt);
      const float cv = (m[u][4] - ux * uy) + om * (shy * ux + shx * uy + shx * shy * wt);
      const float A1 = 2.f * mx * my + C1;
      const float A2 = 2.f * cv + C2;
      const float B1 = mx * mx + my * my + C1;
      const float B2 = vx + vy + C2;
      // B1, B2 >= C1, C2 > 0: hardware reciprocals (1 ulp) suffice
      const float iB1 = __builtin_amdgcn_rcpf(B1), iB2 = __builtin_amdgcn_rcpf(B2);
      const float iB = iB1 * iB2;
      const float S = A1 * A2 * iB;
      const bool in = colin && y >= 0 && y < H;
      if (in && colc && r0 + u >= kLR && r0 + u < kLR + kLT) ssum += S;
      // partials of S in (mu, var, cov), folded so that, at a foreground
      // pixel p, dS/dx_p = sum_q w_qp (Q0_q + 2 x''_p Q1_q + y''_p Q2_q)
      // since there x_p - mu_q = x''_p - mu'_q + sx om_q
      // dS/dmu_x = 2 A2 / (B1^2 B2) (my - mx) (my (mx + my) + C1), the
      // factored form of 2 my A2 / (B1 B2) - 2 mx A1 A2 / (B1^2 B2), whose
      // two terms cancel where the means agree; my - mx from the shifted means
      const float dm = (uy - ux) + (shy - shx) * wt;
      const float Pm = 2.f * A2 * iB2 * iB1 * iB1 * dm * fmaf(my, mx + my, C1);
      const float Pv = -S * iB2;                                  // dS/dvar_x
      const float Pc = 2.f * A1 * iB;                             // dS/dcov
      P[u][0] = in ? Pm + 2.f * (shx * om - ux) * Pv + (shy * om - uy) * Pc : 0.f;
      P[u][1] = in ? Pv : 0.f;
      P[u][2] = in ? Pc : 0.f;
    }
    // region A (the staged images) is free once every thread is past the
    // horizontal pass, which the barrier above guarantees
#pragma unroll
    for (int u = 0; u < kV1; ++u)
#pragma unroll
      for (int q = 0; q < 3; ++q) s_p[(q * kLM + r0 + u) * kLMs + c] = P[u][q];
  }
  __syncthreads();

  // this thread's output pixels (column cx, rows ry0 .. ry0 + kV2 - 1):
  // fetch image, target and mask now, consumed after two more passes
  const int cx = t % kLT, ry0 = (t / kLT) * kV2;
  float xo[kV2], yo[kV2], mo[kV2];
#pragma unroll
  for (int u = 0; u < kV2; ++u) {
    const int y = oy + ry0 + u, x = ox + cx;
    const int64_t o = (int64_t)min(y, H - 1) * W + min(x, W - 1);
    const uint8_t mb = MASK ? Mk[o] : (uint8_t)1;
    const float iv = I[o], gv = G[o];
    mo[u] = (x < W && y < H && mb != 0) ? 1.0f : 0.0f;
    xo[u] = mo[u] * iv;
    yo[u] = mo[u] * gv;
  }

  // partials, horizontal: position row r, output columns c0 .. c0 + kH2 - 1
  constexpr int kItems2 = kLM * (kLT / kH2);
  for (int it = t; it < kItems2; it += kLThreads) {
    const int r = it / (kLT / kH2), c0 = (it - r * (kLT / kH2)) * kH2;
    float acc[kH2][3];
#pragma unroll
    for (int u = 0; u < kH2; ++u)
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[u][q] = 0.f;
#pragma unroll
    for (int j = 0; j < kH2 + 2 * kLR; ++j) {
      float p[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) p[q] = s_p[(q * kLM + r) * kLMs + c0 + j];
#pragma unroll
      for (int u = 0; u < kH2; ++u) {
        const int k = j - u;
        if (k < 0 || k > 2 * kLR) continue;
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[u][q] = fmaf(win.w[k], p[q], acc[u][q]);
      }
    }
#pragma unroll
    for (int u = 0; u < kH2; ++u)
#pragma unroll
      for (int q = 0; q < 3; ++q) s_g[(q * kLM + r) * kLTs + c0 + u] = acc[u][q];
  }
  __syncthreads();

  // partials, vertical, and d loss / d image
  float g[kV2][3];
#pragma unroll
  for (int u = 0; u < kV2; ++u)
#pragma unroll
    for (int q = 0; q < 3; ++q) g[u][q] = 0.f;
#pragma unroll
  for (int j = 0; j < kV2 + 2 * kLR; ++j) {
    float h[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) h[q] = s_g[(q * kLM + ry0 + j) * kLTs + cx];
#pragma unroll
    for (int u = 0; u < kV2; ++u) {
      const int k = j - u;
      if (k < 0 || k > 2 * kLR) continue;
#pragma unroll
      for (int q = 0; q < 3; ++q) g[u][q] = fmaf(win.w[k], h[q], g[u][q]);
    }
  }
  float l1sum = 0.f;
  float* D = d_image + ic * HW;
#pragma unroll
  for (int u = 0; u < kV2; ++u) {
    const int y = oy + ry0 + u, x = ox + cx;
    if (x >= W || y >= H) continue;
    const float xv = xo[u], yv = yo[u];
    l1sum += fabsf(xv - yv);
    const float gs = g[u][0] + 2.f * (xv - shx) * g[u][1] + (yv - shy) * g[u][2];
    const float diff = xv - yv;
    const float sg = diff > 0.f ? 1.f : (diff < 0.f ? -1.f : 0.f);
    D[(int64_t)y * W + x] = mo[u] * (l1_coef * sg - ssim_coef * gs);
  }

  // block sums
  ssum = wave_sum(ssum);
  l1sum = wave_sum(l1sum);
  if ((t & 63) == 0) {
    s_red[0][t >> 6] = ssum;
    s_red[1][t >> 6] = l1sum;
  }
  __syncthreads();
  if (t == 0) {
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int w = 0; w < kLThreads / 64; ++w) {
      a0 += s_red[0][w];
      a1 += s_red[1][w];
    }
    part[2 * blockIdx.x] = a0;
    part[2 * blockIdx.x + 1] = a1;
  }
}

__global__ __launch_bounds__(256) void k_loss_final(const float* __restrict__ part,
                                                    int64_t blocks_per_img, double inv_n,
                                                    float lambda, float* __restrict__ loss_out,
                                                    int64_t* __restrict__ status) {
  __shared__ double sm[2][256];
  const int64_t img = blockIdx.x;
  double s = 0.0, l = 0.0;
  for (int64_t b = threadIdx.x; b < 3 * blocks_per_img; b += 256) {
    s += (double)part[2 * (img * 3 * blocks_per_img + b)];
    l += (double)part[2 * (img * 3 * blocks_per_img + b) + 1];
  }
  sm[0][threadIdx.x] = s;
  sm[1][threadIdx.x] = l;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) {
      sm[0][threadIdx.x] += sm[0][threadIdx.x + d];
      sm[1][threadIdx.x] += sm[1][threadIdx.x + d];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double ssim = sm[0][0] * inv_n, l1 = sm[1][0] * inv_n;
    const float L = (float)((1.0 - lambda) * l1 + lambda * (1.0 - ssim));
    loss_out[img] = L;
    if (status && !isfinite(L)) atomicOr((unsigned long long*)&status[0], (unsigned long long)GS_FLAG_NONFINITE);
  }
}

// ------------------------------------------------------------ masked PSNR

// Evaluation metric of the trainers (the paper judges reconstructions by
// PSNR, Sec. III; the background mask restricts it to the object):
// per image, se = sum over pixels of m sum_c (clamp(I, 0, 1) - G)^2 and
// cnt = 3 sum m, accumulated in FP64 per thread, per work-group in a fixed
// tree order, then over the work-groups of an image in a fixed order.
constexpr int kPsnrThreads = 256;
constexpr int64_t kPsnrMaxBlocks = 256;     // work-groups per image

static int64_t psnr_blocks(int64_t HW) {
  const int64_t b = ceil_div(HW, (int64_t)kPsnrThreads * 16);
  return b < 1 ? 1 : (b > kPsnrMaxBlocks ? kPsnrMaxBlocks : b);
}

__device__ __forceinline__ void block_sum2(double& a, double& b, double (*sm)[kPsnrThreads]) {
  const int t = threadIdx.x;
  sm[0][t] = a;
  sm[1][t] = b;
  __syncthreads();
  for (int d = kPsnrThreads / 2; d > 0; d >>= 1) {
    if (t < d) {
      sm[0][t] += sm[0][t + d];
      sm[1][t] += sm[1][t + d];
    }
    __syncthreads();
  }
  a = sm[0][0];
  b = sm[1][0];
}

__global__ __launch_bounds__(kPsnrThreads) void k_psnr_partial(
    const float* __restrict__ image, const float* __restrict__ target,
    const uint8_t* __restrict__ mask, int64_t HW, int64_t blocks_per_img,
    double* __restrict__ part) {
  __shared__ double sm[2][kPsnrThreads];
  const int64_t img = blockIdx.x / blocks_per_img, b = blockIdx.x - img * blocks_per_img;
  const float* I = image + img * 3 * HW;
  const float* G = target + img * 3 * HW;
  const uint8_t* M = mask ? mask + img * HW : nullptr;
  double se = 0.0, cnt = 0.0;
  for (int64_t p = b * kPsnrThreads + threadIdx.x; p < HW; p += blocks_per_img * kPsnrThreads) {
    if (M && M[p] == 0) continue;
    double e = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double d = (double)fminf(fmaxf(I[c * HW + p], 0.0f), 1.0f) - (double)G[c * HW + p];
      e = fma(d, d, e);
    }
    se += e;
    cnt += 3.0;
  }
  block_sum2(se, cnt, sm);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = se;
    part[2 * blockIdx.x + 1] = cnt;
  }
}

__global__ __launch_bounds__(kPsnrThreads) void k_psnr_final(const double* __restrict__ part,
                                                             int64_t blocks_per_img,
                                                             float* __restrict__ psnr) {
  __shared__ double sm[2][kPsnrThreads];
  const int64_t img = blockIdx.x;
  double se = 0.0, cnt = 0.0;
  for (int64_t b = threadIdx.x; b < blocks_per_img; b += kPsnrThreads) {
    se += part[2 * (img * blocks_per_img + b)];
    cnt += part[2 * (img * blocks_per_img + b) + 1];
  }
  block_sum2(se, cnt, sm);
  if (threadIdx.x == 0) {
    float r;
    if (cnt == 0.0) r = __builtin_nanf("");
    else if (se == 0.0) r = INFINITY;
    else r = (float)(10.0 * log10(cnt / se));
    psnr[img] = r;
  }
}

// x[r][i] *= scale[r] for r < rows, i < row_len (the chain rule of a loss
// through an upstream gradient per image).
__global__ __launch_bounds__(256) void k_scale_rows(float* __restrict__ x,
                                                    const float* __restrict__ scale, int64_t rows,
                                                    int64_t row_len) {
  const int64_t total = rows * row_len;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256)
    x[i] *= scale[i / row_len];
}

static gs_status launch_loss(const float* image, const float* target, const uint8_t* mask,
                             int32_t S, int32_t H, int32_t W, float lambda_dssim,
                             float grad_scale, float* part, float* loss_out, float* d_image,
                             int64_t* status, void* stream);

// Allocation-free form of the loss: its partial sums (8 bytes per image,
// channel and 32x32 tile, every one written by k_ssim before k_loss_final
// reads it, so nothing needs clearing) live in this file-scope array, one
// copy per device, held until the process ends.  Host code never passes the
// array's name to a kernel: it looks up the array's device address once per
// device with hipGetSymbolAddress and passes that.
constexpr size_t kLossScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kLossScratchBytes];

static gs_status loss_scratch_address(void** out) {
  static std::mutex mu;
  static std::vector<void*> addr;           // per device, from hipGetSymbolAddress
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_error("gs_loss_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    return GS_ERR_HIP;
  }
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (addr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error("gs_loss_noalloc: hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return GS_ERR_HIP;
    }
    addr[dev] = p;
  }
  *out = addr[dev];
  return GS_OK;
}

}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_loss_noalloc(const float* image, const float* target, const uint8_t* mask,
                          int32_t S, int32_t H, int32_t W, float lambda_dssim, float grad_scale,
                          float* loss_out, float* d_image, int64_t* status, void* stream) {
  clear_error();
  GS_REQUIRE(S >= 1 && H >= 1 && W >= 1, "gs_loss_noalloc: bad shape S=%d H=%d W=%d", S, H, W);
  GS_REQUIRE(image && target && loss_out && d_image, "gs_loss_noalloc: NULL argument");
  GS_REQUIRE(lambda_dssim >= 0.f && lambda_dssim <= 1.f,
             "gs_loss_noalloc: lambda %f outside [0,1]", (double)lambda_dssim);
  const LossLayout L = loss_layout(S, H, W);
  GS_REQUIRE(L.total <= kLossScratchBytes,
             "gs_loss_noalloc: S=%d images of %dx%d need %zu bytes of scratch, above the "
             "%zu-byte maximum (use gs_loss with a workspace)",
             S, W, H, L.total, kLossScratchBytes);
  void* ws = nullptr;
  const gs_status st = loss_scratch_address(&ws);
  if (st != GS_OK) return st;
  return launch_loss(image, target, mask, S, H, W, lambda_dssim, grad_scale,
                     (float*)((char*)ws + L.off_part), loss_out, d_image, status, stream);
}

size_t gs_loss_workspace_bytes(int32_t S, int32_t H, int32_t W) {
  if (S < 0 || H < 0 || W < 0) return 0;
  return loss_layout(S, H, W).total;
}

gs_status gs_loss(const float* image, const float* target, const uint8_t* mask, int32_t S,
                  int32_t H, int32_t W, float lambda_dssim, float grad_scale, void* ws,
                  size_t ws_bytes, float* loss_out, float* d_image, int64_t* status,
                  void* stream) {
  clear_error();
  GS_REQUIRE(S >= 1 && H >= 1 && W >= 1, "gs_loss: bad shape S=%d H=%d W=%d", S, H, W);
  GS_REQUIRE(image && target && ws && loss_out && d_image, "gs_loss: NULL argument");
  GS_REQUIRE(lambda_dssim >= 0.f && lambda_dssim <= 1.f, "gs_loss: lambda %f outside [0,1]",
             (double)lambda_dssim);
  LossLayout L = loss_layout(S, H, W);
  GS_REQUIRE(ws_bytes >= L.total, "gs_loss: workspace %zu < required %zu", ws_bytes, L.total);
  GS_REQUIRE(((uintptr_t)ws & 255) == 0, "gs_loss: workspace must be 256-byte aligned");
  return launch_loss(image, target, mask, S, H, W, lambda_dssim, grad_scale,
                     (float*)((char*)ws + L.off_part), loss_out, d_image, status, stream);
}

}  // extern "C"

namespace gsmi {

static gs_status launch_loss(const float* image, const float* target, const uint8_t* mask,
                             int32_t S, int32_t H, int32_t W, float lambda_dssim,
                             float grad_scale, float* part, float* loss_out, float* d_image,
                             int64_t* status, void* stream) {
  const LossLayout L = loss_layout(S, H, W);
  const Window win = ssim_window();
  const int64_t blocks = (int64_t)S * 3 * L.blocks_per_img;
  hipStream_t s = as_stream(stream);
  const double N = 3.0 * (double)H * (double)W;
  const float l1_coef = (float)((1.0 - lambda_dssim) * grad_scale / N);
  const float ssim_coef = (float)(lambda_dssim * grad_scale / N);
  if (mask)
    hipLaunchKernelGGL(k_ssim<true>, dim3((unsigned)blocks), dim3(kLThreads), 0, s, image, target,
                       mask, H, W, L.tiles_x, L.blocks_per_img, win, l1_coef, ssim_coef, d_image,
                       part);
  else
    hipLaunchKernelGGL(k_ssim<false>, dim3((unsigned)blocks), dim3(kLThreads), 0, s, image, target,
                       mask, H, W, L.tiles_x, L.blocks_per_img, win, l1_coef, ssim_coef, d_image,
                       part);
  GS_LAUNCH_CHECK("gs_loss/ssim");
  hipLaunchKernelGGL(k_loss_final, dim3((unsigned)S), dim3(256), 0, s, part, L.blocks_per_img,
                     1.0 / N, lambda_dssim, loss_out, status);
  GS_LAUNCH_CHECK("gs_loss/final");
  return GS_OK;
}

}  // namespace gsmi

extern "C" {

size_t gs_psnr_workspace_bytes(int32_t S, int32_t H, int32_t W) {
  if (S < 0 || H < 0 || W < 0) return 0;
  const size_t b = (size_t)psnr_blocks((int64_t)H * W);
  return ((sizeof(double) * 2 * b * (size_t)(S > 0 ? S : 1)) + 255) & ~size_t(255);
}

gs_status gs_masked_psnr(const float* image, const float* target, const uint8_t* mask, int32_t S,
                         int32_t H, int32_t W, void* ws, size_t ws_bytes, float* psnr_out,
                         void* stream) {
  clear_error();
  GS_REQUIRE(S >= 1 && H >= 1 && W >= 1, "gs_masked_psnr: bad shape S=%d H=%d W=%d", S, H, W);
  GS_REQUIRE(image && target && ws && psnr_out, "gs_masked_psnr: NULL argument");
  const size_t need = gs_psnr_workspace_bytes(S, H, W);
  GS_REQUIRE(ws_bytes >= need, "gs_masked_psnr: workspace %zu < required %zu", ws_bytes, need);
  GS_REQUIRE(((uintptr_t)ws & 7) == 0, "gs_masked_psnr: workspace must be 8-byte aligned");
  const int64_t HW = (int64_t)H * W;
  const int64_t B = psnr_blocks(HW);
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(k_psnr_partial, dim3((unsigned)(B * S)), dim3(kPsnrThreads), 0, s, image,
                     target, mask, HW, B, (double*)ws);
  GS_LAUNCH_CHECK("gs_masked_psnr/partial");
  hipLaunchKernelGGL(k_psnr_final, dim3((unsigned)S), dim3(kPsnrThreads), 0, s,
                     (const double*)ws, B, psnr_out);
  GS_LAUNCH_CHECK("gs_masked_psnr/final");
  return GS_OK;
}

gs_status gs_scale_rows(float* x, const float* scale, int64_t rows, int64_t row_len,
                        void* stream) {
  clear_error();
  GS_REQUIRE(rows >= 0 && row_len >= 0, "gs_scale_rows: negative size");
  if (rows == 0 || row_len == 0) return GS_OK;
  GS_REQUIRE(x && scale, "gs_scale_rows: NULL argument");
  int64_t blocks = ceil_div(rows * row_len, 256);
  const int64_t cap = (int64_t)device_cu_count() * 16;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), x,
                     scale, rows, row_len);
  GS_LAUNCH_CHECK("gs_scale_rows");
  return GS_OK;
}

}  // extern "C"
