// project.hip — EWA projection of 3D Gaussians and its backward (3D-GS
// method that the paper's Sec. II "Parallel Training" runs per partition).
//
// Forward: one thread per (Gaussian, slot) pair; planar SoA parameter loads
// are coalesced, the 48-byte record goes out as three 16-byte stores.
// Backward: one thread per Gaussian that loops over the slots drawing it, so
// gradients summed over views need no atomics and are deterministic.  The
// view-dependent colour (spherical harmonics up to degree 3) is a template
// parameter of every kernel.
#include <type_traits>

#include "gs_device.h"

namespace gsmi {

struct Params {
  const float* mean;
  const float* ls;
  const float* quat;
  const float* ol;
  const float* col;
  int64_t n;
};

struct GradPtrs {
  float* mean;
  float* ls;
  float* quat;
  float* ol;
  float* col;
};

// Everything the projection of one pair computes (FP32).
struct ProjState {
  float s[3], qn[4], qinv;
  float R[9];          // rotation of the Gaussian
  float Sig[6];        // 3D covariance xx, xy, xz, yy, yz, zz
  float t[3];
  float mean2d[2];
  float xc, yc;        // clamped tx, ty used by the Jacobian
  bool xcl, ycl;
  float T[6];          // J * Rv (2x3, row-major)
  float a, b, c, det;  // dilated 2D covariance
  float conic[3];
  float o, pre_rgb[3], rgb[3];
  float dir[3], ivlen; // unit vector camera centre -> mean, 1/|mean - centre|
  int bbox[4];         // inclusive tile range
  int n_tiles;
  bool valid;
};

__device__ __forceinline__ void load_gaussian(const Params& P, int64_t g, float mu[3], float ls[3],
                                              float q[4], float& ol) {
  const int64_t n = P.n;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    mu[k] = P.mean[k * n + g];
    ls[k] = P.ls[k * n + g];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = P.quat[k * n + g];
  ol = P.ol[g];
}

// ---------------------------------------------------------------------------
// View-dependent colour (3D-GS colour model): rgb_c = max(0, sum_k Y_k(d)
// f_kc + 1/2) over the real spherical harmonics of degree <= D, Condon-
// Shortley phase, index l*l + l + m, d the unit vector from the camera centre
// to the mean.  Y_k is written out as a polynomial of d's components.
// Colour coefficients are planar: coefficient k of channel c in row 3k + c.
// ---------------------------------------------------------------------------
constexpr float kSH1 = 0.4886025119029199f;  // sqrt(3 / (4 pi))
constexpr float kSH2a = 1.0925484305920792f; // sqrt(15 / (4 pi))
constexpr float kSH2b = 0.31539156525252005f;// sqrt(5 / (16 pi))
constexpr float kSH2c = 0.5462742152960396f; // sqrt(15 / (16 pi))
constexpr float kSH3a = 0.5900435899266435f; // sqrt(35 / (32 pi))
constexpr float kSH3b = 2.890611442640554f;  // sqrt(105 / (4 pi))
constexpr float kSH3c = 0.4570457994644658f; // sqrt(21 / (32 pi))
constexpr float kSH3d = 0.3731763325901154f; // sqrt(7 / (16 pi))
constexpr float kSH3e = 1.445305721320277f;  // sqrt(105 / (16 pi))

// f(k, Y_k, dY_k/dx, dY_k/dy, dY_k/dz) for k = 0 .. (D+1)^2 - 1 at the unit
// vector d; each term is made where it is consumed, so no table of basis
// values stays live.  No multiply-add contraction here: every kernel that
// evaluates the basis gets the same bits, wherever it is inlined.
template <int D, class F>
__device__ __forceinline__ void sh_for_each(const float d[3], F&& f) {
#pragma clang fp contract(off)
  f(0, kC0, 0.f, 0.f, 0.f);
  if constexpr (D >= 1) {
    const float x = d[0], y = d[1], z = d[2];
    f(1, -kSH1 * y, 0.f, -kSH1, 0.f);
    f(2, kSH1 * z, 0.f, 0.f, kSH1);
    f(3, -kSH1 * x, -kSH1, 0.f, 0.f);
    if constexpr (D >= 2) {
      const float xx = x * x, yy = y * y, zz = z * z;
      f(4, kSH2a * x * y, kSH2a * y, kSH2a * x, 0.f);
      f(5, -kSH2a * y * z, 0.f, -kSH2a * z, -kSH2a * y);
      f(6, kSH2b * (2.f * zz - xx - yy), -2.f * kSH2b * x, -2.f * kSH2b * y, 4.f * kSH2b * z);
      f(7, -kSH2a * x * z, -kSH2a * z, 0.f, -kSH2a * x);
      f(8, kSH2c * (xx - yy), 2.f * kSH2c * x, -2.f * kSH2c * y, 0.f);
      if constexpr (D >= 3) {
        f(9, -kSH3a * y * (3.f * xx - yy), -6.f * kSH3a * x * y, -kSH3a * (3.f * xx - 3.f * yy),
          0.f);
        f(10, kSH3b * x * y * z, kSH3b * y * z, kSH3b * x * z, kSH3b * x * y);
        f(11, -kSH3c * y * (4.f * zz - xx - yy), 2.f * kSH3c * x * y,
          -kSH3c * (4.f * zz - xx - 3.f * yy), -8.f * kSH3c * y * z);
        f(12, kSH3d * z * (2.f * zz - 3.f * xx - 3.f * yy), -6.f * kSH3d * x * z,
          -6.f * kSH3d * y * z, kSH3d * (6.f * zz - 3.f * xx - 3.f * yy));
        f(13, -kSH3c * x * (4.f * zz - xx - yy), -kSH3c * (4.f * zz - 3.f * xx - yy),
          2.f * kSH3c * x * y, -8.f * kSH3c * x * z);
        f(14, kSH3e * z * (xx - yy), 2.f * kSH3e * x * z, -2.f * kSH3e * y * z, kSH3e * (xx - yy));
        f(15, -kSH3a * x * (xx - 3.f * yy), -kSH3a * (3.f * xx - 3.f * yy), 6.f * kSH3a * x * y,
          0.f);
      }
    }
  }
}

// S.pre_rgb / S.rgb of Gaussian g from its colour coefficients.
template <int D>
__device__ __forceinline__ void colour_fwd(const float* __restrict__ col, int64_t n, int64_t g,
                                           ProjState& S) {
  float acc[3] = {0.f, 0.f, 0.f};
  sh_for_each<D>(S.dir, [&](int k, float Y, float, float, float) {
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += Y * col[(3 * k + c) * n + g];
  });
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    S.pre_rgb[c] = acc[c] + 0.5f;
    S.rgb[c] = fmaxf(S.pre_rgb[c], 0.0f);
  }
}

// Colour of one pair and its backward: rgb_c = max(0, sum_k Y_k(d) f_kc +
// 1/2) (sets S.pre_rgb / S.rgb); gc_c = dL/drgb_c where the clamp passes;
// the mean moves the direction: dL/dmean += (I - d d^T) dL/dd / |v| with
// dL/dd = sum_c gc_c sum_k f_kc grad Y_k.  One pass over the coefficients
// makes both the colour and the per-channel direction gradients.
template <int D>
__device__ __forceinline__ void colour_bwd(const float* __restrict__ col, int64_t n, int64_t g,
                                           ProjState& S, const float* __restrict__ drgb,
                                           float gc[3], float gmu[3]) {
  float acc[3] = {0.f, 0.f, 0.f};
  float gdc[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
  // walk the rows from a pointer the compiler cannot see through, so the
  // row addresses are made here and not kept live across the caller's loop
  const float* cp = col + g;
  if constexpr (D >= 1) asm volatile("" : "+v"(cp));
  sh_for_each<D>(S.dir, [&](int k, float Y, float gx, float gy, float gz) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float f = *cp;
      cp += n;
      acc[c] += Y * f;
      if (k > 0) {
        gdc[c][0] += f * gx;
        gdc[c][1] += f * gy;
        gdc[c][2] += f * gz;
      }
    }
  });
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    S.pre_rgb[c] = acc[c] + 0.5f;
    S.rgb[c] = fmaxf(S.pre_rgb[c], 0.0f);
    gc[c] = S.pre_rgb[c] >= 0.0f ? drgb[c] : 0.0f;
  }
  if constexpr (D >= 1) {
    float gd[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) gd[j] = gc[0] * gdc[0][j] + gc[1] * gdc[1][j] + gc[2] * gdc[2][j];
    const float x = S.dir[0], y = S.dir[1], z = S.dir[2];
    const float dd = gd[0] * x + gd[1] * y + gd[2] * z;
    gmu[0] += (gd[0] - x * dd) * S.ivlen;
    gmu[1] += (gd[1] - y * dd) * S.ivlen;
    gmu[2] += (gd[2] - z * dd) * S.ivlen;
  }
}

// add(r, Y_k(d) gc_c) for every coefficient row r = 3k + c: the pair's
// gradient of the colour coefficients.
template <int D, class Add>
__device__ __forceinline__ void colour_coef_grads(const float d[3], const float gc[3], Add&& add) {
  sh_for_each<D>(d, [&](int k, float Y, float, float, float) {
#pragma unroll
    for (int c = 0; c < 3; ++c) add(3 * k + c, Y * gc[c]);
  });
}

// Colour-gradient running sums of the fused kernel over several slots:
// registers at degree 0; above it an LDS array [rows][256] per block (48 KB
// at degree 3), which keeps up to 48 sums out of the registers the
// projection needs.
template <int D>
struct ColourAcc {
  static constexpr int NC = 3 * (D + 1) * (D + 1);
  static constexpr int STRIDE = D == 0 ? 1 : 256;
  float reg[D == 0 ? NC : 1];
  float* lds;
  __device__ __forceinline__ void init(float* block_lds) {
    lds = block_lds + threadIdx.x;
#pragma unroll
    for (int r = 0; r < NC; ++r) at(r) = 0.f;
  }
  __device__ __forceinline__ float& at(int r) {
    if constexpr (D == 0) return reg[r];
    else return lds[r * STRIDE];
  }
};

__device__ __forceinline__ void project_core(const float mu[3], const float ls[3], const float q[4],
                                             float ol, const gs_camera& cam,
                                             int W, int H, int tw, int th, ProjState& S) {
  S.valid = false;
  S.n_tiles = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) S.s[k] = expf(ls[k]);
  float qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  float qnorm = sqrtf(qq);
  S.qinv = 1.0f / qnorm;
#pragma unroll
  for (int k = 0; k < 4; ++k) S.qn[k] = q[k] * S.qinv;
  float w = S.qn[0], x = S.qn[1], y = S.qn[2], z = S.qn[3];
  float* R = S.R;
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
  float M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[r * 3 + k] = R[r * 3 + k] * S.s[k];
  // Sigma = M M^T
  S.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  S.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  S.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  S.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  S.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  S.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
  S.o = 1.0f / (1.0f + expf(-ol));
  const float* Rv = cam.R;
  {
    // v = mean - camera centre, centre = -Rv^T t
    float v[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
      v[i] = mu[i] + Rv[0 * 3 + i] * cam.t[0] + Rv[1 * 3 + i] * cam.t[1] + Rv[2 * 3 + i] * cam.t[2];
    const float vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    S.ivlen = vv > 0.0f ? rsqrtf(vv) : 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) S.dir[i] = v[i] * S.ivlen;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
    S.t[i] = Rv[i * 3 + 0] * mu[0] + Rv[i * 3 + 1] * mu[1] + Rv[i * 3 + 2] * mu[2] + cam.t[i];
  float tx = S.t[0], ty = S.t[1], tz = S.t[2];
  if (!(tz > cam.znear)) return;
  float itz = 1.0f / tz;
  S.mean2d[0] = cam.fx * tx * itz + cam.cx;
  S.mean2d[1] = cam.fy * ty * itz + cam.cy;
  float limx = kFrustum * 0.5f * (float)W / cam.fx;
  float limy = kFrustum * 0.5f * (float)H / cam.fy;
  float rx = tx * itz, ry = ty * itz;
  S.xcl = (rx < -limx) || (rx > limx);
  S.ycl = (ry < -limy) || (ry > limy);
  rx = fminf(fmaxf(rx, -limx), limx);
  ry = fminf(fmaxf(ry, -limy), limy);
  S.xc = rx * tz;
  S.yc = ry * tz;
  float j00 = cam.fx * itz, j02 = -cam.fx * S.xc * itz * itz;
  float j11 = cam.fy * itz, j12 = -cam.fy * S.yc * itz * itz;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    S.T[k] = j00 * Rv[0 * 3 + k] + j02 * Rv[2 * 3 + k];
    S.T[3 + k] = j11 * Rv[1 * 3 + k] + j12 * Rv[2 * 3 + k];
  }
  // V = T Sigma T^T
  const float* Sg = S.Sig;
  float u0[3], u1[3];  // Sigma T_row^T
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const float* Tr = S.T + 3 * r;
    float* u = r ? u1 : u0;
    u[0] = Sg[0] * Tr[0] + Sg[1] * Tr[1] + Sg[2] * Tr[2];
    u[1] = Sg[1] * Tr[0] + Sg[3] * Tr[1] + Sg[4] * Tr[2];
    u[2] = Sg[2] * Tr[0] + Sg[4] * Tr[1] + Sg[5] * Tr[2];
  }
  S.a = S.T[0] * u0[0] + S.T[1] * u0[1] + S.T[2] * u0[2] + kDilate;
  S.b = S.T[0] * u1[0] + S.T[1] * u1[1] + S.T[2] * u1[2];
  S.c = S.T[3] * u1[0] + S.T[4] * u1[1] + S.T[5] * u1[2] + kDilate;
  S.det = S.a * S.c - S.b * S.b;
  if (!(S.det > 0.0f)) return;
  float idet = 1.0f / S.det;
  S.conic[0] = S.c * idet;
  S.conic[1] = -S.b * idet;
  S.conic[2] = S.a * idet;
  if (!(255.0f * S.o > 1.0f)) return;
  float kappa = 2.0f * logf(255.0f * S.o);
  float hx = sqrtf(kappa * S.a), hy = sqrtf(kappa * S.c);
  float xl = S.mean2d[0] - hx, xh = S.mean2d[0] + hx;
  float yl = S.mean2d[1] - hy, yh = S.mean2d[1] + hy;
  float Wf = (float)W + 4.0f, Hf = (float)H + 4.0f;
  xl = (xl > -4.0f) ? fminf(xl, Wf) : -4.0f;
  xh = (xh > -4.0f) ? fminf(xh, Wf) : -4.0f;
  yl = (yl > -4.0f) ? fminf(yl, Hf) : -4.0f;
  yh = (yh > -4.0f) ? fminf(yh, Hf) : -4.0f;
  int x0 = max((int)floorf(xl) - 1, 0), x1 = min((int)floorf(xh) + 1, W - 1);
  int y0 = max((int)floorf(yl) - 1, 0), y1 = min((int)floorf(yh) + 1, H - 1);
  if (x0 > x1 || y0 > y1) return;
  S.bbox[0] = x0 / tw;
  S.bbox[1] = y0 / th;
  S.bbox[2] = x1 / tw;
  S.bbox[3] = y1 / th;
  S.n_tiles = (S.bbox[2] - S.bbox[0] + 1) * (S.bbox[3] - S.bbox[1] + 1);
  S.valid = true;
}

__device__ __forceinline__ int find_slot(const int64_t* __restrict__ pair_offset, int n_slots,
                                         int64_t p) {
  int lo = 0, hi = n_slots - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pair_offset[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int D>
__global__ __launch_bounds__(256) void k_project(Params P, const int64_t* __restrict__ pair_offset,
                                                 const int64_t* __restrict__ gauss_offset,
                                                 const gs_camera* __restrict__ cams, int n_slots,
                                                 int64_t m, int W, int H, int tw, int th,
                                                 float4* __restrict__ rec,
                                                 uint2* __restrict__ tile_bbox,
                                                 int32_t* __restrict__ n_tiles) {
  int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= m) return;
  int s = find_slot(pair_offset, n_slots, p);
  int64_t g = gauss_offset[s] + (p - pair_offset[s]);
  ProjState S;
  S.valid = false;
  S.n_tiles = 0;
  S.t[2] = 0.0f;
  if (g >= 0 && g < P.n) {
    float mu[3], ls[3], q[4], ol;
    load_gaussian(P, g, mu, ls, q, ol);
    project_core(mu, ls, q, ol, cams[s], W, H, tw, th, S);
    if (S.valid) colour_fwd<D>(P.col, P.n, g, S);
  }
  float4* r = rec + 3 * p;
  if (S.valid) {
    r[0] = make_float4(S.mean2d[0], S.mean2d[1], S.conic[0], S.conic[1]);
    r[1] = make_float4(S.conic[2], S.o, S.rgb[0], S.rgb[1]);
    r[2] = make_float4(S.rgb[2], S.t[2], __int_as_float(s), 0.0f);
    tile_bbox[p] = make_uint2((uint32_t)S.bbox[0] | ((uint32_t)S.bbox[1] << 16),
                              (uint32_t)S.bbox[2] | ((uint32_t)S.bbox[3] << 16));
    n_tiles[p] = S.n_tiles;
  } else {
    r[0] = make_float4(0.f, 0.f, 0.f, 0.f);
    r[1] = make_float4(0.f, 0.f, 0.f, 0.f);
    r[2] = make_float4(0.f, S.t[2], __int_as_float(s), 0.0f);
    tile_bbox[p] = make_uint2(0u, 0u);
    n_tiles[p] = 0;
  }
}

// Backward of project_core for one pair (everything but the colour):
// accumulates the parameter gradients of the pair into the per-thread sums.
__device__ __forceinline__ void project_bwd_core(const ProjState& S, const gs_camera& cam,
                                                 const float* __restrict__ dr, float gmu[3],
                                                 float gls[3], float gq[4], float& gol) {
  float dmx = dr[0], dmy = dr[1], dq11 = dr[2], dq12 = dr[3], dq22 = dr[4];
  float dop = dr[5];
  gol += S.o * (1.0f - S.o) * dop;
  // conic (c, -b, a)/det as a function of (a, b, c)
  float a = S.a, b = S.b, c = S.c;
  float idet = 1.0f / S.det, id2 = idet * idet;
  float da = (-c * c * dq11 + b * c * dq12 - b * b * dq22) * id2;
  float db = (2.f * b * c * dq11 - (S.det + 2.f * b * b) * dq12 + 2.f * a * b * dq22) * id2;
  float dc = (-b * b * dq11 + a * b * dq12 - a * a * dq22) * id2;
  float G00 = da, G01 = 0.5f * db, G11 = dc;
  const float* T = S.T;
  // dSigma = T^T G T  (symmetric 3x3: xx, xy, xz, yy, yz, zz)
  float gt0[3], gt1[3];  // rows of G T
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gt0[k] = G00 * T[k] + G01 * T[3 + k];
    gt1[k] = G01 * T[k] + G11 * T[3 + k];
  }
  float dS[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) dS[i * 3 + j] = T[i] * gt0[j] + T[3 + i] * gt1[j];
  // dT = 2 G T Sigma
  const float* Sg = S.Sig;
  float Sf[9] = {Sg[0], Sg[1], Sg[2], Sg[1], Sg[3], Sg[4], Sg[2], Sg[4], Sg[5]};
  float dT[6];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    dT[l] = 2.f * (gt0[0] * Sf[0 * 3 + l] + gt0[1] * Sf[1 * 3 + l] + gt0[2] * Sf[2 * 3 + l]);
    dT[3 + l] = 2.f * (gt1[0] * Sf[0 * 3 + l] + gt1[1] * Sf[1 * 3 + l] + gt1[2] * Sf[2 * 3 + l]);
  }
  // T = J Rv: dJ = dT Rv^T (only the non-constant entries of J)
  const float* Rv = cam.R;
  float dj00 = dT[0] * Rv[0] + dT[1] * Rv[1] + dT[2] * Rv[2];
  float dj02 = dT[0] * Rv[6] + dT[1] * Rv[7] + dT[2] * Rv[8];
  float dj11 = dT[3] * Rv[3] + dT[4] * Rv[4] + dT[5] * Rv[5];
  float dj12 = dT[3] * Rv[6] + dT[4] * Rv[7] + dT[5] * Rv[8];
  float tx = S.t[0], ty = S.t[1], tz = S.t[2];
  float itz = 1.0f / tz, itz2 = itz * itz, itz3 = itz2 * itz;
  float fx = cam.fx, fy = cam.fy;
  float dtx = 0.f, dty = 0.f, dtz = 0.f;
  dtz += -fx * itz2 * dj00 - fy * itz2 * dj11;
  if (!S.xcl) {
    dtx += -fx * itz2 * dj02;
    dtz += 2.f * fx * tx * itz3 * dj02;
  } else {
    dtz += fx * S.xc * itz3 * dj02;
  }
  if (!S.ycl) {
    dty += -fy * itz2 * dj12;
    dtz += 2.f * fy * ty * itz3 * dj12;
  } else {
    dtz += fy * S.yc * itz3 * dj12;
  }
  dtx += dmx * fx * itz;
  dty += dmy * fy * itz;
  dtz += -(dmx * fx * tx + dmy * fy * ty) * itz2;
#pragma unroll
  for (int k = 0; k < 3; ++k) gmu[k] += Rv[k] * dtx + Rv[3 + k] * dty + Rv[6 + k] * dtz;
  // Sigma = M M^T, M = R diag(s): dM = 2 dSigma M
  const float* R = S.R;
  float M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[r * 3 + k] = R[r * 3 + k] * S.s[k];
  float dM[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      dM[r * 3 + k] =
          2.f * (dS[r * 3 + 0] * M[0 * 3 + k] + dS[r * 3 + 1] * M[1 * 3 + k] + dS[r * 3 + 2] * M[2 * 3 + k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float ds = dM[0 * 3 + k] * R[0 * 3 + k] + dM[1 * 3 + k] * R[1 * 3 + k] + dM[2 * 3 + k] * R[2 * 3 + k];
    gls[k] += ds * S.s[k];
  }
  float dR[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) dR[r * 3 + k] = dM[r * 3 + k] * S.s[k];
  float w = S.qn[0], x = S.qn[1], y = S.qn[2], z = S.qn[3];
  float dw = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  float dx = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] +
                    w * dR[7] - 2.f * x * dR[8]);
  float dy = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                    z * dR[7] - 2.f * y * dR[8]);
  float dz = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] +
                    y * dR[5] + x * dR[6] + y * dR[7]);
  float dot = w * dw + x * dx + y * dy + z * dz;
  gq[0] += (dw - w * dot) * S.qinv;
  gq[1] += (dx - x * dot) * S.qinv;
  gq[2] += (dy - y * dot) * S.qinv;
  gq[3] += (dz - z * dot) * S.qinv;
}

// A thread owns a Gaussian and loops over the slots drawing it.  Degree 0
// sums the colour gradient in registers; above it every pair adds its
// coefficient gradients to the gradient array directly (in slot order, the
// same additions as a running sum into zeroed arrays).
template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(D == 3 ? 3 : 1))) void
k_project_bwd(
    Params P, GradPtrs Gr, const int64_t* __restrict__ pair_offset,
    const int64_t* __restrict__ gauss_offset, const gs_camera* __restrict__ cams, int n_slots,
    int W, int H, int tw, int th, const int32_t* __restrict__ n_tiles,
    const float* __restrict__ d_rec) {
  int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= P.n) return;
  const int64_t n = P.n;
  float acc0[3] = {0.f, 0.f, 0.f};
  float mu[3], ls[3], q[4], ol;
  load_gaussian(P, g, mu, ls, q, ol);
  float gmu[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
  float gol = 0.f;
  bool any = false;
  for (int s = 0; s < n_slots; ++s) {
    int64_t g0 = gauss_offset[s];
    int64_t cnt = pair_offset[s + 1] - pair_offset[s];
    if (g < g0 || g >= g0 + cnt) continue;
    int64_t p = pair_offset[s] + (g - g0);
    if (n_tiles[p] <= 0) continue;
    ProjState S;
    project_core(mu, ls, q, ol, cams[s], W, H, tw, th, S);
    if (!S.valid) continue;
    float dr[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) dr[k] = d_rec[p * GS_DREC_STRIDE + k];
    project_bwd_core(S, cams[s], dr, gmu, gls, gq, gol);
    // the colour last, so its coefficients are live only here
    float gc[3];
    colour_bwd<D>(P.col, n, g, S, dr + 6, gc, gmu);
    if constexpr (D == 0) {
      colour_coef_grads<0>(S.dir, gc, [&](int r, float x) { acc0[r] += x; });
    } else {
      float* gp = Gr.col + g;
      asm volatile("" : "+v"(gp));
      colour_coef_grads<D>(S.dir, gc, [&](int r, float x) { gp[(int64_t)r * n] += x; });
    }
    any = true;
  }
  if (!any) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Gr.mean[k * n + g] += gmu[k];
    Gr.ls[k * n + g] += gls[k];
  }
  if constexpr (D == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) Gr.col[k * n + g] += acc0[k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) Gr.quat[k * n + g] += gq[k];
  Gr.ol[g] += gol;
}

// gs_project_bwd and one Adam step in a single pass: a thread owns a
// Gaussian, sums its gradient over its pairs (the same arithmetic as
// k_project_bwd) and applies the update to its parameters (11 plus the
// colour rows), reading and writing m and v once.  Gaussians drawn by no
// pair get a zero gradient (dense Adam) or, with visible_only, are left as
// they are (sparse Adam).
struct AdamFused {
  float* p[5];            // mean, log_scale, quat, opacity_logit, colour (planar)
  float* m[5];
  float* v[5];
  int col_rows;           // rows of the colour arrays (>= 3 (D+1)^2)
  int visible_only;       // sparse Adam: Gaussians drawn by no pair are left as they are
  float lr[6], lr_final[6];   // [5]: colour rows from 3 on (= [4] with five groups)
  int decay_steps;
  float b1, b2, eps;
  const int32_t* step_dev;
};

// ONE (degree > 0, calls with a single slot): the Gaussian's colour
// gradient is Y(d) gc of its one pair, so only d and gc are kept and the
// sums are made in the update loop; otherwise above degree 0 the sums live
// in LDS, which allows 3 blocks per CU, and registers are capped to match.
template <int D, bool ONE>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(D == 0 || (ONE && D < 3) ? 1 : 3))) void k_project_bwd_adam(
    Params P, AdamFused A, const int64_t* __restrict__ pair_offset,
    const int64_t* __restrict__ gauss_offset, const gs_camera* __restrict__ cams, int n_slots,
    int W, int H, int tw, int th, const int32_t* __restrict__ n_tiles,
    const float* __restrict__ d_rec) {
  __shared__ float s_lr[6], s_ibc[2];
  if (threadIdx.x < 6) {
    float lr, ibc1, ibc2;
    adam_schedule(A.step_dev[0] + 1, A.b1, A.b2, A.lr[threadIdx.x], A.lr_final[threadIdx.x],
                  A.decay_steps, lr, ibc1, ibc2);
    s_lr[threadIdx.x] = lr;
    if (threadIdx.x == 0) {
      s_ibc[0] = ibc1;
      s_ibc[1] = ibc2;
    }
  }
  __syncthreads();
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= P.n) return;
  if (A.visible_only) {
    // sparse Adam: a Gaussian drawn by no pair keeps parameters and moments,
    // so nothing of it is read or written
    bool drawn = false;
    for (int s = 0; s < n_slots && !drawn; ++s) {
      const int64_t g0 = gauss_offset[s];
      if (g < g0 || g >= g0 + (pair_offset[s + 1] - pair_offset[s])) continue;
      drawn = n_tiles[pair_offset[s] + (g - g0)] > 0;
    }
    if (!drawn) return;
  }
  constexpr int NC = ColourAcc<D>::NC;
  constexpr bool kLds = D > 0 && !ONE;
  __shared__ float s_gcol[kLds ? NC * 256 : 1];
  ColourAcc<D> gcol;
  if constexpr (!ONE) gcol.init(s_gcol);
  float one_dir[3] = {0.f, 0.f, 1.f}, one_gc[3] = {0.f, 0.f, 0.f};
  float mu[3], ls[3], q[4], ol;
  load_gaussian(P, g, mu, ls, q, ol);
  float gmu[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
  float gol = 0.f;
  for (int s = 0; s < n_slots; ++s) {
    const int64_t g0 = gauss_offset[s];
    const int64_t cnt = pair_offset[s + 1] - pair_offset[s];
    if (g < g0 || g >= g0 + cnt) continue;
    const int64_t p = pair_offset[s] + (g - g0);
    if (n_tiles[p] <= 0) continue;
    ProjState S;
    project_core(mu, ls, q, ol, cams[s], W, H, tw, th, S);
    if (!S.valid) continue;
    float dr[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) dr[k] = d_rec[p * GS_DREC_STRIDE + k];
    project_bwd_core(S, cams[s], dr, gmu, gls, gq, gol);
    // the colour last, so its coefficients are live only here
    float gc[3];
    colour_bwd<D>(P.col, P.n, g, S, dr + 6, gc, gmu);
    if constexpr (ONE) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        one_dir[j] = S.dir[j];
        one_gc[j] = gc[j];
      }
    } else {
      colour_coef_grads<D>(S.dir, gc, [&](int r, float x) { gcol.at(r) += x; });
    }
  }
  // the gradient a separate pass would add to zeroed arrays
  const float G[11] = {0.f + gmu[0], 0.f + gmu[1], 0.f + gmu[2], 0.f + gls[0], 0.f + gls[1],
                       0.f + gls[2], 0.f + gq[0],  0.f + gq[1],  0.f + gq[2],  0.f + gq[3],
                       0.f + gol};
  float par[11] = {mu[0], mu[1], mu[2], ls[0], ls[1], ls[2], q[0], q[1], q[2], q[3], ol};
  constexpr int kGroup[11] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 2, 3};
  constexpr int kRow[11] = {0, 1, 2, 0, 1, 2, 0, 1, 2, 3, 0};
  const int64_t n = P.n;
  const float ibc1 = s_ibc[0], ibc2 = s_ibc[1];
#pragma unroll
  for (int e = 0; e < 11; ++e) {
    const int gr = kGroup[e];
    const int64_t o = (int64_t)kRow[e] * n + g;
    float m = A.m[gr][o], v = A.v[gr][o];
    adam_update(par[e], G[e], m, v, s_lr[gr], ibc1, ibc2, A.b1, A.b2, A.eps);
    A.p[gr][o] = par[e];
    A.m[gr][o] = m;
    A.v[gr][o] = v;
  }
  // colour rows: the active coefficients, then any stored beyond the
  // active degree (zero gradient)
  float* cp = A.p[4] + g;
  float* cm = A.m[4] + g;
  float* cv = A.v[4] + g;
  if constexpr (D >= 1) asm volatile("" : "+v"(cp), "+v"(cm), "+v"(cv));
  const float lr_dc = s_lr[4], lr_rest = s_lr[5];
  auto colour_row = [&](float grad, float lr) {
    float pv = *cp, m = *cm, v = *cv;
    adam_update(pv, 0.f + grad, m, v, lr, ibc1, ibc2, A.b1, A.b2, A.eps);
    *cp = pv;
    *cm = m;
    *cv = v;
    cp += n;
    cm += n;
    cv += n;
  };
  if constexpr (ONE) {
    colour_coef_grads<D>(one_dir, one_gc,
                         [&](int r, float x) { colour_row(x, r < 3 ? lr_dc : lr_rest); });
  } else {
#pragma unroll
    for (int r = 0; r < NC; ++r) colour_row(gcol.at(r), r < 3 ? lr_dc : lr_rest);
  }
  for (int r = NC; r < A.col_rows; ++r) {
    float pv = *cp, m = *cm, v = *cv;
    adam_update(pv, 0.f, m, v, r < 3 ? lr_dc : lr_rest, ibc1, ibc2, A.b1, A.b2, A.eps);
    *cp = pv;
    *cm = m;
    *cv = v;
    cp += n;
    cm += n;
    cv += n;
  }
}

__global__ void k_adam_step_inc(int32_t* step_dev) {
  if (threadIdx.x == 0) step_dev[0] += 1;
}

// Calls f(std::integral_constant<int, D>) for the run-time degree d (0..3).
template <class F>
static void sh_dispatch(int d, F&& f) {
  switch (d) {
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    default: f(std::integral_constant<int, 3>{}); break;
  }
}

}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_project(const gs_gaussians* g, const gs_views* views, const gs_tiling* tiling,
                     gs_projected* out, void* stream) {
  clear_error();
  GS_REQUIRE(g && out, "gs_project: NULL argument");
  gs_status st = check_views(views, tiling, "gs_project");
  if (st != GS_OK) return st;
  GS_REQUIRE(g->n >= 0, "gs_project: n=%lld < 0", (long long)g->n);
  GS_REQUIRE(g->sh_degree >= 0 && g->sh_degree <= GS_SH_MAX_DEGREE,
             "gs_project: sh_degree=%d outside 0..%d", g->sh_degree, GS_SH_MAX_DEGREE);
  GS_REQUIRE(out->m == views->total_pairs, "gs_project: out->m=%lld != total_pairs=%lld",
             (long long)out->m, (long long)views->total_pairs);
  if (out->m == 0) return GS_OK;
  GS_REQUIRE(g->n > 0 && g->mean && g->log_scale && g->quat && g->opacity_logit && g->color,
             "gs_project: Gaussian arrays must not be NULL");
  GS_REQUIRE(out->rec && out->tile_bbox && out->n_tiles, "gs_project: output arrays NULL");
  GS_REQUIRE(((uintptr_t)out->rec & 15) == 0 && ((uintptr_t)out->tile_bbox & 7) == 0,
             "gs_project: rec must be 16-byte and tile_bbox 8-byte aligned");
  Params P{g->mean, g->log_scale, g->quat, g->opacity_logit, g->color, g->n};
  int64_t blocks = ceil_div(out->m, 256);
  sh_dispatch(g->sh_degree, [&](auto D) {
    hipLaunchKernelGGL(k_project<decltype(D)::value>, dim3((unsigned)blocks), dim3(256), 0,
                       as_stream(stream), P, views->pair_offset, views->gauss_offset, views->cams,
                       views->n_slots, out->m, tiling->width, tiling->height, tiling->tile_w,
                       tiling->tile_h, (float4*)out->rec, (uint2*)out->tile_bbox, out->n_tiles);
  });
  GS_LAUNCH_CHECK("gs_project");
  return GS_OK;
}

gs_status gs_project_bwd(const gs_gaussians* g, const gs_views* views, const gs_tiling* tiling,
                         const gs_projected* proj, const float* d_rec, gs_grads* grads,
                         void* stream) {
  clear_error();
  GS_REQUIRE(g && proj && grads, "gs_project_bwd: NULL argument");
  gs_status st = check_views(views, tiling, "gs_project_bwd");
  if (st != GS_OK) return st;
  GS_REQUIRE(proj->m == views->total_pairs, "gs_project_bwd: proj->m != total_pairs");
  GS_REQUIRE(grads->n == g->n, "gs_project_bwd: grads->n=%lld != n=%lld", (long long)grads->n,
             (long long)g->n);
  GS_REQUIRE(g->sh_degree >= 0 && g->sh_degree <= GS_SH_MAX_DEGREE,
             "gs_project_bwd: sh_degree=%d outside 0..%d", g->sh_degree, GS_SH_MAX_DEGREE);
  if (g->n == 0 || proj->m == 0) return GS_OK;
  GS_REQUIRE(g->mean && g->log_scale && g->quat && g->opacity_logit && g->color,
             "gs_project_bwd: Gaussian arrays must not be NULL");
  GS_REQUIRE(grads->mean && grads->log_scale && grads->quat && grads->opacity_logit &&
                 grads->color && d_rec && proj->n_tiles,
             "gs_project_bwd: gradient arrays must not be NULL");
  Params P{g->mean, g->log_scale, g->quat, g->opacity_logit, g->color, g->n};
  GradPtrs G{grads->mean, grads->log_scale, grads->quat, grads->opacity_logit, grads->color};
  int64_t blocks = ceil_div(g->n, 256);
  sh_dispatch(g->sh_degree, [&](auto D) {
    hipLaunchKernelGGL(k_project_bwd<decltype(D)::value>, dim3((unsigned)blocks), dim3(256), 0,
                       as_stream(stream), P, G, views->pair_offset, views->gauss_offset,
                       views->cams, views->n_slots, tiling->width, tiling->height, tiling->tile_w,
                       tiling->tile_h, proj->n_tiles, d_rec);
  });
  GS_LAUNCH_CHECK("gs_project_bwd");
  return GS_OK;
}

gs_status gs_project_bwd_adam(const gs_gaussians* g, const gs_views* views,
                              const gs_tiling* tiling, const gs_projected* proj,
                              const float* d_rec, const gs_adam_group* groups,
                              int32_t n_groups, const float* lr_final, int32_t decay_steps,
                              float beta1, float beta2, float eps, int32_t visible_only,
                              int32_t* step_dev, void* stream) {
  clear_error();
  GS_REQUIRE(g && proj && groups && step_dev, "gs_project_bwd_adam: NULL argument");
  GS_REQUIRE(n_groups == 5 || n_groups == 6, "gs_project_bwd_adam: n_groups=%d (5 or 6)",
             n_groups);
  gs_status st = check_views(views, tiling, "gs_project_bwd_adam");
  if (st != GS_OK) return st;
  GS_REQUIRE(proj->m == views->total_pairs, "gs_project_bwd_adam: proj->m != total_pairs");
  GS_REQUIRE(decay_steps >= 0, "gs_project_bwd_adam: decay_steps < 0");
  GS_REQUIRE(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f,
             "gs_project_bwd_adam: bad betas");
  GS_REQUIRE(g->sh_degree >= 0 && g->sh_degree <= GS_SH_MAX_DEGREE,
             "gs_project_bwd_adam: sh_degree=%d outside 0..%d", g->sh_degree, GS_SH_MAX_DEGREE);
  const float* arrays[5] = {g->mean, g->log_scale, g->quat, g->opacity_logit, g->color};
  const int nc = 3 * (g->sh_degree + 1) * (g->sh_degree + 1);
  int col_rows = nc;
  if (g->n > 0) {
    // the colour rows: group 4's, plus group 5's when given
    int64_t col_count = groups[4].count;
    if (n_groups == 6) {
      const int64_t off = 3 * g->n;
      GS_REQUIRE(groups[4].count == off && groups[5].param == groups[4].param + off &&
                     (groups[4].m == nullptr ||
                      (groups[5].m == groups[4].m + off && groups[5].v == groups[4].v + off)),
                 "gs_project_bwd_adam: with 6 groups, group 4 must be colour rows 0-2 and "
                 "group 5 the rows after them in the same arrays");
      col_count += groups[5].count;
    }
    GS_REQUIRE(col_count % g->n == 0 && col_count / g->n >= nc && (col_count / g->n) % 3 == 0 &&
                   col_count / g->n <= 3 * (GS_SH_MAX_DEGREE + 1) * (GS_SH_MAX_DEGREE + 1),
               "gs_project_bwd_adam: colour count %lld must be 3k x n, k >= (D+1)^2 = %d, "
               "k <= %d",
               (long long)col_count, nc / 3, (GS_SH_MAX_DEGREE + 1) * (GS_SH_MAX_DEGREE + 1));
    col_rows = (int)(col_count / g->n);
  }
  const int rows[5] = {3, 3, 4, 1, n_groups == 6 ? 3 : col_rows};
  AdamFused A;
  A.col_rows = col_rows;
  A.visible_only = visible_only ? 1 : 0;
  for (int i = 0; i < 5; ++i) {
    GS_REQUIRE(groups[i].param == arrays[i] && groups[i].count == rows[i] * g->n,
               "gs_project_bwd_adam: group %d must be the Gaussians' array %d (%d x n elements)",
               i, i, rows[i]);
    GS_REQUIRE(g->n == 0 || (groups[i].m && groups[i].v), "gs_project_bwd_adam: group %d NULL m/v",
               i);
    const float lf = lr_final ? lr_final[i] : 0.0f;
    GS_REQUIRE(!(lf > 0.0f) || groups[i].lr > 0.0f,
               "gs_project_bwd_adam: decay needs lr > 0 (group %d)", i);
    A.p[i] = groups[i].param;
    A.m[i] = groups[i].m;
    A.v[i] = groups[i].v;
    A.lr[i] = groups[i].lr;
    A.lr_final[i] = lf;
  }
  A.lr[5] = A.lr[4];
  A.lr_final[5] = A.lr_final[4];
  if (n_groups == 6) {
    const float lf = lr_final ? lr_final[5] : 0.0f;
    GS_REQUIRE(!(lf > 0.0f) || groups[5].lr > 0.0f, "gs_project_bwd_adam: decay needs lr > 0 (group 5)");
    A.lr[5] = groups[5].lr;
    A.lr_final[5] = lf;
  }
  A.decay_steps = decay_steps;
  A.b1 = beta1;
  A.b2 = beta2;
  A.eps = eps;
  A.step_dev = step_dev;
  hipStream_t s = as_stream(stream);
  if (g->n > 0) {
    GS_REQUIRE(g->mean && g->log_scale && g->quat && g->opacity_logit && g->color &&
                   (proj->m == 0 || (d_rec && proj->n_tiles)),
               "gs_project_bwd_adam: arrays must not be NULL");
    Params P{g->mean, g->log_scale, g->quat, g->opacity_logit, g->color, g->n};
    const dim3 grid((unsigned)ceil_div(g->n, 256));
    sh_dispatch(g->sh_degree, [&](auto D) {
      constexpr int kD = decltype(D)::value;
      auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, grid, dim3(256), 0, s, P, A, views->pair_offset,
                           views->gauss_offset, views->cams, views->n_slots, tiling->width,
                           tiling->height, tiling->tile_w, tiling->tile_h, proj->n_tiles, d_rec);
      };
      if constexpr (kD > 0) {
        if (views->n_slots == 1) launch(k_project_bwd_adam<kD, true>);
        else launch(k_project_bwd_adam<kD, false>);
      } else {
        launch(k_project_bwd_adam<0, false>);
      }
    });
    GS_LAUNCH_CHECK("gs_project_bwd_adam");
  }
  hipLaunchKernelGGL(k_adam_step_inc, dim3(1), dim3(64), 0, s, step_dev);
  GS_LAUNCH_CHECK("gs_project_bwd_adam/step");
  return GS_OK;
}

}  // extern "C"
