// loss.hip — background-masked L1 + D-SSIM photometric loss and its image
// gradient (masks: the paper's Sec. II "Image Rendering and Masking" and
// Sec. III-A; L1 + D-SSIM: the 3D-GS training loss it trains with).
//
// One work-group per (image, channel, 32x32 output tile).
// k_ssim_fwd  per 32x32 output tile and channel: stage the masked image and
//             target (+5 px halo, zero outside the image) in LDS, blur the
//             five moment maps with the separable 11-tap window, form the
//             SSIM map and the three per-pixel partials dS/dmu_x, dS/dE[x^2],
//             dS/dE[xy]; write the partials, block sums of S and |x - y|.
// k_ssim_bwd  per tile: blur the partials with the same (symmetric) window,
//             which is the adjoint of the forward blur, and combine them
//             with the L1 subgradient into d loss / d image.
// k_loss_final one work-group per image: deterministic FP64 sum of the block
//             partials -> loss[s]; non-finite losses raise the status flag.
#include <math.h>

#include "gs_device.h"

namespace gsmi {

constexpr int kLT = 32;              // output tile edge
constexpr int kLR = 5;               // window radius
constexpr int kLIn = kLT + 2 * kLR;  // 42: staged edge
constexpr int kLThreads = 256;

struct Window {
  float w[2 * kLR + 1];
};

static Window ssim_window() {
  double w[2 * kLR + 1], s = 0;
  for (int k = 0; k <= 2 * kLR; ++k) {
    double d = k - kLR;
    w[k] = exp(-d * d / (2.0 * 1.5 * 1.5));
    s += w[k];
  }
  Window W;
  for (int k = 0; k <= 2 * kLR; ++k) W.w[k] = (float)(w[k] / s);
  return W;
}

struct LossLayout {
  int64_t tiles_x, tiles_y, blocks_per_img;
  size_t off_maps, off_part, total;
};

static LossLayout loss_layout(int S, int H, int W) {
  LossLayout L;
  L.tiles_x = ceil_div(W, kLT);
  L.tiles_y = ceil_div(H, kLT);
  L.blocks_per_img = L.tiles_x * L.tiles_y;
  L.off_maps = 0;
  size_t maps = sizeof(float) * 9 * (size_t)S * H * W;
  L.off_part = (maps + 255) & ~size_t(255);
  size_t part = sizeof(float) * 2 * 3 * (size_t)S * L.blocks_per_img;
  L.total = L.off_part + ((part + 255) & ~size_t(255));
  return L;
}

__global__ __launch_bounds__(kLThreads) void k_ssim_fwd(
    const float* __restrict__ image, const float* __restrict__ target,
    const uint8_t* __restrict__ mask, int H, int W, int64_t tiles_x, int64_t blocks_per_img,
    Window win, float* __restrict__ maps, float* __restrict__ part) {
  __shared__ float s_x[kLIn][kLIn + 1];
  __shared__ float s_y[kLIn][kLIn + 1];
  __shared__ float s_h[5][kLIn][kLT + 1];
  __shared__ float s_red[2][4];
  const int64_t ic = blockIdx.x / blocks_per_img;          // image * 3 + channel
  const int64_t img = ic / 3;
  const int ch = (int)(ic - img * 3);
  const int64_t b = blockIdx.x - ic * blocks_per_img;
  const int ty = (int)(b / tiles_x), tx = (int)(b - (int64_t)ty * tiles_x);
  const int x0 = tx * kLT - kLR, y0 = ty * kLT - kLR;
  const int t = threadIdx.x;
  const int64_t HW = (int64_t)H * W;
  float ssum = 0.f, l1sum = 0.f;
  {
    const float* I = image + (img * 3 + ch) * HW;
    const float* G = target + (img * 3 + ch) * HW;
    for (int i = t; i < kLIn * kLIn; i += kLThreads) {
      const int r = i / kLIn, c = i - r * kLIn;
      const int y = y0 + r, x = x0 + c;
      float xv = 0.f, yv = 0.f;
      if (x >= 0 && x < W && y >= 0 && y < H) {
        const int64_t o = (int64_t)y * W + x;
        const float mk = mask ? (float)(mask[img * HW + o] != 0) : 1.0f;
        xv = mk * I[o];
        yv = mk * G[o];
      }
      s_x[r][c] = xv;
      s_y[r][c] = yv;
    }
    __syncthreads();
    // horizontal pass: 42 rows x 32 columns, five moments
    for (int i = t; i < kLIn * kLT; i += kLThreads) {
      const int r = i / kLT, c = i - r * kLT;
      float mx = 0.f, my = 0.f, xx = 0.f, yy = 0.f, xy = 0.f;
#pragma unroll
      for (int k = 0; k <= 2 * kLR; ++k) {
        const float xv = s_x[r][c + k], yv = s_y[r][c + k], w = win.w[k];
        mx = fmaf(w, xv, mx);
        my = fmaf(w, yv, my);
        xx = fmaf(w, xv * xv, xx);
        yy = fmaf(w, yv * yv, yy);
        xy = fmaf(w, xv * yv, xy);
      }
      s_h[0][r][c] = mx;
      s_h[1][r][c] = my;
      s_h[2][r][c] = xx;
      s_h[3][r][c] = yy;
      s_h[4][r][c] = xy;
    }
    __syncthreads();
    for (int i = t; i < kLT * kLT; i += kLThreads) {
      const int r = i / kLT, c = i - r * kLT;
      const int y = ty * kLT + r, x = tx * kLT + c;
      float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k <= 2 * kLR; ++k) {
        const float w = win.w[k];
#pragma unroll
        for (int q = 0; q < 5; ++q) m[q] = fmaf(w, s_h[q][r + k][c], m[q]);
      }
      if (x < W && y < H) {
        const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
        const float mx = m[0], my = m[1];
        const float A1 = 2.f * mx * my + C1;
        const float A2 = 2.f * (m[4] - mx * my) + C2;
        const float B1 = mx * mx + my * my + C1;
        const float B2 = (m[2] - mx * mx) + (m[3] - my * my) + C2;
        const float iB = 1.0f / (B1 * B2);
        const float S = A1 * A2 * iB;
        ssum += S;
        const float xv = s_x[r + kLR][c + kLR], yv = s_y[r + kLR][c + kLR];
        l1sum += fabsf(xv - yv);
        const int64_t o = (int64_t)y * W + x;
        float* mp = maps + (img * 9 + ch * 3) * HW;
        mp[o] = 2.f * my * (A2 - A1) * iB - 2.f * mx * S * (1.0f / B1 - 1.0f / B2);
        mp[HW + o] = -S / B2;
        mp[2 * HW + o] = 2.f * A1 * iB;
      }
    }
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
    part[2 * blockIdx.x] = s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3];
    part[2 * blockIdx.x + 1] = s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3];
  }
}

__global__ __launch_bounds__(kLThreads) void k_ssim_bwd(
    const float* __restrict__ image, const float* __restrict__ target,
    const uint8_t* __restrict__ mask, int H, int W, int64_t tiles_x, int64_t blocks_per_img,
    Window win, const float* __restrict__ maps, float l1_coef, float ssim_coef,
    float* __restrict__ d_image) {
  __shared__ float s_m[3][kLIn][kLIn + 1];
  __shared__ float s_h[3][kLIn][kLT + 1];
  const int64_t ic = blockIdx.x / blocks_per_img;          // image * 3 + channel
  const int64_t img = ic / 3;
  const int ch = (int)(ic - img * 3);
  const int64_t b = blockIdx.x - ic * blocks_per_img;
  const int ty = (int)(b / tiles_x), tx = (int)(b - (int64_t)ty * tiles_x);
  const int x0 = tx * kLT - kLR, y0 = ty * kLT - kLR;
  const int t = threadIdx.x;
  const int64_t HW = (int64_t)H * W;
  {
    const float* mp = maps + (img * 9 + ch * 3) * HW;
    for (int i = t; i < kLIn * kLIn; i += kLThreads) {
      const int r = i / kLIn, c = i - r * kLIn;
      const int y = y0 + r, x = x0 + c;
      float a = 0.f, bb = 0.f, cc = 0.f;
      if (x >= 0 && x < W && y >= 0 && y < H) {
        const int64_t o = (int64_t)y * W + x;
        a = mp[o];
        bb = mp[HW + o];
        cc = mp[2 * HW + o];
      }
      s_m[0][r][c] = a;
      s_m[1][r][c] = bb;
      s_m[2][r][c] = cc;
    }
    __syncthreads();
    for (int i = t; i < kLIn * kLT; i += kLThreads) {
      const int r = i / kLT, c = i - r * kLT;
      float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k <= 2 * kLR; ++k) {
        const float w = win.w[k];
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[q] = fmaf(w, s_m[q][r][c + k], acc[q]);
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) s_h[q][r][c] = acc[q];
    }
    __syncthreads();
    const float* I = image + (img * 3 + ch) * HW;
    const float* G = target + (img * 3 + ch) * HW;
    float* D = d_image + (img * 3 + ch) * HW;
    for (int i = t; i < kLT * kLT; i += kLThreads) {
      const int r = i / kLT, c = i - r * kLT;
      const int y = ty * kLT + r, x = tx * kLT + c;
      if (x >= W || y >= H) continue;
      float g[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k <= 2 * kLR; ++k) {
        const float w = win.w[k];
#pragma unroll
        for (int q = 0; q < 3; ++q) g[q] = fmaf(w, s_h[q][r + k][c], g[q]);
      }
      const int64_t o = (int64_t)y * W + x;
      const float mk = mask ? (float)(mask[img * HW + o] != 0) : 1.0f;
      const float xv = mk * I[o], yv = mk * G[o];
      const float gs = g[0] + 2.f * xv * g[1] + yv * g[2];
      const float diff = xv - yv;
      const float sg = diff > 0.f ? 1.f : (diff < 0.f ? -1.f : 0.f);
      D[o] = mk * (l1_coef * sg - ssim_coef * gs);
    }
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

}  // namespace gsmi

using namespace gsmi;

extern "C" {

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
  char* w = (char*)ws;
  float* maps = (float*)(w + L.off_maps);
  float* part = (float*)(w + L.off_part);
  const Window win = ssim_window();
  const int64_t blocks = (int64_t)S * 3 * L.blocks_per_img;
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(k_ssim_fwd, dim3((unsigned)blocks), dim3(kLThreads), 0, s, image, target,
                     mask, H, W, L.tiles_x, L.blocks_per_img, win, maps, part);
  GS_LAUNCH_CHECK("gs_loss/ssim_fwd");
  const double N = 3.0 * (double)H * (double)W;
  const float l1_coef = (float)((1.0 - lambda_dssim) * grad_scale / N);
  const float ssim_coef = (float)(lambda_dssim * grad_scale / N);
  hipLaunchKernelGGL(k_ssim_bwd, dim3((unsigned)blocks), dim3(kLThreads), 0, s, image, target,
                     mask, H, W, L.tiles_x, L.blocks_per_img, win, maps, l1_coef, ssim_coef,
                     d_image);
  GS_LAUNCH_CHECK("gs_loss/ssim_bwd");
  hipLaunchKernelGGL(k_loss_final, dim3((unsigned)S), dim3(256), 0, s, part, L.blocks_per_img,
                     1.0 / N, lambda_dssim, loss_out, status);
  GS_LAUNCH_CHECK("gs_loss/final");
  return GS_OK;
}

}  // extern "C"
