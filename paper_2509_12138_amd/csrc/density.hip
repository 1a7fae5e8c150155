// density.hip — adaptive density control of the 3D-GS method the paper's
// Sec. II trains each partition with: between training steps, Gaussians
// whose screen-space position gradient stays large are cloned (small ones)
// or split (large ones), near-transparent or oversized ones are pruned, and
// opacities are periodically reset.
//
//   k_densify_stats   thread per Gaussian: adds, over its visible pairs of a
//                     step, the norm of the gradient of its projected mean in
//                     normalised device coordinates, and the pair count
//   k_densify_select  thread per Gaussian: its action and output count, and
//                     per-block count sums
//   k_densify_scan    one work-group: exclusive scan of the block sums; the
//                     output count
//   k_densify_apply   thread per Gaussian: writes its 0, 1 or 2 outputs
//                     (parameters and Adam moments) at its scanned offset
//   k_opacity_reset   element-wise clamp of the opacity logits, moments
//                     cleared
// Every decision compares an FP32 input with an FP32 threshold, so the
// output order and count are exact; a split child's mean is
// mu + R(q) (s * z) for a caller-supplied standard normal sample z.
#include <math.h>

#include "gs_device.h"

namespace gsmi {

constexpr int kDenThreads = 256;

// action codes
constexpr int32_t kActDrop = 0, kActKeep = 1, kActClone = 2, kActSplit = 3;

__device__ __forceinline__ int act_count(int32_t a) {
  return a == kActKeep ? 1 : (a == kActClone || a == kActSplit ? 2 : 0);
}

template <typename T>
__device__ __forceinline__ T den_block_exclusive_scan(T v, T* sm /*[kDenThreads / 64]*/, T& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T u = __shfl_up(inc, d, 64);
    if (lane >= d) inc += u;
  }
  if (lane == 63) sm[wave] = inc;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kDenThreads / 64; ++w) {
    const T x = sm[w];
    if (w < wave) base += x;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return base + inc - v;
}

// Correctly rounded FP32 square root: the hardware estimate (within 1 ulp)
// is moved to the neighbour on the right side of the rounding midpoints,
// which are exact in FP64 (25 significant bits, squares of 50 bits; a float
// never equals such a square, so there are no ties).
__device__ __forceinline__ float sqrt_rn(float x) {
#pragma clang fp contract(off)
  if (!(x > 0.0f) || !isfinite(x)) return sqrtf(x);
  float s = __builtin_amdgcn_sqrtf(x);
  const double xd = (double)x;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const uint32_t b = __float_as_uint(s);
    const float up = __uint_as_float(b + 1u), dn = __uint_as_float(b - 1u);
    const double mu = 0.5 * ((double)s + (double)up), md = 0.5 * ((double)s + (double)dn);
    if (xd > mu * mu) s = up;
    else if (xd < md * md) s = dn;
  }
  return s;
}

__global__ __launch_bounds__(kDenThreads) void k_densify_stats(
    const int64_t* __restrict__ pair_offset, const int64_t* __restrict__ gauss_offset,
    int n_slots, int64_t n, const int32_t* __restrict__ n_tiles, const float* __restrict__ d_rec,
    float half_w, float half_h, float* __restrict__ accum, float* __restrict__ denom) {
  // one rounding per operation: no multiply-add contraction here
#pragma clang fp contract(off)
  const int64_t g = (int64_t)blockIdx.x * kDenThreads + threadIdx.x;
  if (g >= n) return;
  float a = accum[g], d = denom[g];
  for (int s = 0; s < n_slots; ++s) {
    const int64_t g0 = gauss_offset[s];
    const int64_t cnt = pair_offset[s + 1] - pair_offset[s];
    if (g < g0 || g >= g0 + cnt) continue;
    const int64_t p = pair_offset[s] + (g - g0);
    if (n_tiles[p] <= 0) continue;
    // one rounding per operation (contraction is off in this function): the
    // statistic decides integers (the actions)
    const float gx = d_rec[p * GS_DREC_STRIDE + 0] * half_w;
    const float gy = d_rec[p * GS_DREC_STRIDE + 1] * half_h;
    const float gx2 = gx * gx, gy2 = gy * gy;
    a = a + sqrt_rn(gx2 + gy2);
    d = d + 1.0f;
  }
  accum[g] = a;
  denom[g] = d;
}

struct DenThresholds {
  float grad;        // mean gradient norm at or above which a Gaussian densifies
  float log_dense;   // largest log-scale of a Gaussian that is cloned (else split)
  float logit_min;   // opacity logits below this are pruned
  float log_big;     // log-scales above this are pruned
  float log_split;   // log of the split children's scale divisor
};

__global__ __launch_bounds__(kDenThreads) void k_densify_select(
    const float* __restrict__ log_scale, const float* __restrict__ opacity_logit,
    const float* __restrict__ accum, const float* __restrict__ denom, int64_t n,
    DenThresholds th, int32_t* __restrict__ action, int64_t* __restrict__ block_sums) {
  __shared__ int64_t sm[kDenThreads / 64];
  const int64_t g = (int64_t)blockIdx.x * kDenThreads + threadIdx.x;
  int32_t act = kActDrop;
  if (g < n) {
    const float ls = fmaxf(fmaxf(log_scale[g], log_scale[n + g]), log_scale[2 * n + g]);
    const float dn = denom[g];
    // mean >= threshold decided exactly: FP64 products of FP32 values are
    // exact
    const bool grow = dn > 0.0f && (double)accum[g] >= (double)th.grad * (double)dn;
    const bool faint = opacity_logit[g] < th.logit_min;
    if (faint) {
      act = kActDrop;                       // copies would inherit the opacity
    } else if (grow && ls <= th.log_dense) {
      act = ls > th.log_big ? kActDrop : kActClone;
    } else if (grow) {
      act = __fsub_rn(ls, th.log_split) > th.log_big ? kActDrop : kActSplit;
    } else {
      act = ls > th.log_big ? kActDrop : kActKeep;
    }
    action[g] = act;
  }
  int64_t total;
  den_block_exclusive_scan<int64_t>((int64_t)act_count(act), sm, total);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Exclusive scan of the per-block counts in place; n_out[0] = the total.
__global__ __launch_bounds__(kDenThreads) void k_densify_scan(int64_t* __restrict__ block_sums,
                                                             int64_t nb,
                                                             int64_t* __restrict__ n_out) {
  __shared__ int64_t sm[kDenThreads / 64];
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += kDenThreads) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < nb ? block_sums[i] : 0;
    int64_t total;
    const int64_t ex = den_block_exclusive_scan<int64_t>(v, sm, total);
    if (i < nb) block_sums[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) n_out[0] = carry;
}

struct DenState {
  float* p[5];   // mean, log_scale, quat, opacity_logit, colour (planar [rows][n])
  float* m[5];
  float* v[5];
  int64_t n;
  int rows[5];   // 3, 3, 4, 1 and the colour rows 3 (D+1)^2
};

// R(q / |q|) column-major application: out = R (s * z).
__device__ __forceinline__ void rotate_scaled(const float q[4], const float s[3], const float z[3],
                                              float out[3]) {
  const float inv = 1.0f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, zq = q[3] * inv;
  const float R[9] = {1.f - 2.f * (y * y + zq * zq), 2.f * (x * y - w * zq), 2.f * (x * zq + w * y),
                      2.f * (x * y + w * zq), 1.f - 2.f * (x * x + zq * zq), 2.f * (y * zq - w * x),
                      2.f * (x * zq - w * y), 2.f * (y * zq + w * x), 1.f - 2.f * (x * x + y * y)};
  const float a[3] = {s[0] * z[0], s[1] * z[1], s[2] * z[2]};
#pragma unroll
  for (int r = 0; r < 3; ++r) out[r] = R[3 * r] * a[0] + R[3 * r + 1] * a[1] + R[3 * r + 2] * a[2];
}

__global__ __launch_bounds__(kDenThreads) void k_densify_apply(
    DenState in, const int32_t* __restrict__ action, const int64_t* __restrict__ block_offsets,
    const float* __restrict__ z, float log_split, DenState out) {
  __shared__ int64_t sm[kDenThreads / 64];
  const int64_t g = (int64_t)blockIdx.x * kDenThreads + threadIdx.x;
  const int32_t act = g < in.n ? action[g] : kActDrop;
  int64_t total;
  const int64_t o =
      block_offsets[blockIdx.x] + den_block_exclusive_scan<int64_t>((int64_t)act_count(act), sm, total);
  // outputs beyond the caller's arrays (out.n smaller than the count) are
  // not written
  if (act == kActDrop || o >= out.n) return;
  const int64_t n = in.n, no = out.n;
  if (act == kActKeep || act == kActClone) {
    const int copies = (act == kActClone && o + 1 < no) ? 2 : 1;
#pragma unroll
    for (int grp = 0; grp < 5; ++grp)
      for (int r = 0; r < in.rows[grp]; ++r) {
        const float pv = in.p[grp][r * n + g];
        const float mv = in.m[grp] ? in.m[grp][r * n + g] : 0.0f;
        const float vv = in.v[grp] ? in.v[grp][r * n + g] : 0.0f;
        for (int c = 0; c < copies; ++c) {
          out.p[grp][r * no + o + c] = pv;
          // the clone starts with fresh moments
          if (out.m[grp]) out.m[grp][r * no + o + c] = c == 0 ? mv : 0.0f;
          if (out.v[grp]) out.v[grp][r * no + o + c] = c == 0 ? vv : 0.0f;
        }
      }
    return;
  }
  // split: two children at mu + R (s * z_c), scales divided by exp(log_split)
  float mu[3], ls[3], q[4], s[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    mu[r] = in.p[0][r * n + g];
    ls[r] = in.p[1][r * n + g];
    s[r] = expf(ls[r]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) q[r] = in.p[2][r * n + g];
  for (int c = 0; c < 2 && o + c < no; ++c) {
    const float zc[3] = {z[(g * 2 + c) * 3 + 0], z[(g * 2 + c) * 3 + 1], z[(g * 2 + c) * 3 + 2]};
    float off[3];
    rotate_scaled(q, s, zc, off);
    const int64_t oc = o + c;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      out.p[0][r * no + oc] = mu[r] + off[r];
      out.p[1][r * no + oc] = __fsub_rn(ls[r], log_split);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) out.p[2][r * no + oc] = q[r];
    out.p[3][oc] = in.p[3][g];
    for (int r = 0; r < in.rows[4]; ++r) out.p[4][r * no + oc] = in.p[4][r * n + g];
#pragma unroll
    for (int grp = 0; grp < 5; ++grp)
      for (int r = 0; r < in.rows[grp]; ++r) {
        if (out.m[grp]) out.m[grp][r * no + oc] = 0.0f;
        if (out.v[grp]) out.v[grp][r * no + oc] = 0.0f;
      }
  }
}

__global__ __launch_bounds__(kDenThreads) void k_opacity_reset(float* __restrict__ logit,
                                                              float* __restrict__ m,
                                                              float* __restrict__ v, int64_t n,
                                                              float max_logit) {
  const int64_t g = (int64_t)blockIdx.x * kDenThreads + threadIdx.x;
  if (g >= n) return;
  logit[g] = fminf(logit[g], max_logit);
  if (m) m[g] = 0.0f;
  if (v) v[g] = 0.0f;
}

static DenState den_state(const gs_gaussian_state* s) {
  DenState d;
  for (int i = 0; i < 5; ++i) {
    d.p[i] = s->param[i];
    d.m[i] = s->m[i];
    d.v[i] = s->v[i];
  }
  d.n = s->n;
  const int rows[5] = {3, 3, 4, 1, s->color_rows > 0 ? s->color_rows : 3};
  for (int i = 0; i < 5; ++i) d.rows[i] = rows[i];
  return d;
}

static bool state_ok(const gs_gaussian_state* s) {
  if (!s || s->n < 0) return false;
  if (s->color_rows < 0 || s->color_rows % 3 != 0 ||
      s->color_rows > 3 * (GS_SH_MAX_DEGREE + 1) * (GS_SH_MAX_DEGREE + 1))
    return false;
  if (s->n == 0) return true;
  for (int i = 0; i < 5; ++i)
    if (!s->param[i] || ((s->m[i] == nullptr) != (s->v[i] == nullptr))) return false;
  return true;
}

}  // namespace gsmi

using namespace gsmi;

extern "C" {

size_t gs_densify_workspace_bytes(int64_t n) {
  if (n < 0) return 0;
  return sizeof(int64_t) * (size_t)(ceil_div(n > 0 ? n : 1, kDenThreads) + 1);
}

gs_status gs_densify_stats(const gs_views* views, const gs_tiling* tiling,
                           const gs_projected* proj, const float* d_rec, int64_t n, float* accum,
                           float* denom, void* stream) {
  clear_error();
  GS_REQUIRE(proj != nullptr, "gs_densify_stats: NULL proj");
  gs_status st = check_views(views, tiling, "gs_densify_stats");
  if (st != GS_OK) return st;
  GS_REQUIRE(proj->m == views->total_pairs, "gs_densify_stats: proj->m != total_pairs");
  GS_REQUIRE(n >= 0, "gs_densify_stats: n < 0");
  if (n == 0) return GS_OK;
  GS_REQUIRE(accum && denom, "gs_densify_stats: NULL accum/denom");
  GS_REQUIRE(proj->m == 0 || (d_rec && proj->n_tiles), "gs_densify_stats: NULL d_rec/n_tiles");
  hipLaunchKernelGGL(k_densify_stats, dim3((unsigned)ceil_div(n, kDenThreads)), dim3(kDenThreads),
                     0, as_stream(stream), views->pair_offset, views->gauss_offset,
                     views->n_slots, n, proj->n_tiles, d_rec, 0.5f * (float)tiling->width,
                     0.5f * (float)tiling->height, accum, denom);
  GS_LAUNCH_CHECK("gs_densify_stats");
  return GS_OK;
}

gs_status gs_densify_select(const gs_gaussian_state* state, const float* accum,
                            const float* denom, float grad_threshold, float max_log_scale_clone,
                            float min_opacity_logit, float max_log_scale, float log_split,
                            void* ws, size_t ws_bytes, int32_t* action, int64_t* n_out,
                            void* stream) {
  clear_error();
  GS_REQUIRE(state_ok(state), "gs_densify_select: bad state (NULL arrays or n < 0)");
  GS_REQUIRE(n_out && ws, "gs_densify_select: NULL n_out/workspace");
  const int64_t n = state->n;
  GS_REQUIRE(ws_bytes >= gs_densify_workspace_bytes(n), "gs_densify_select: workspace too small");
  GS_REQUIRE(n == 0 || (accum && denom && action), "gs_densify_select: NULL statistics/action");
  GS_REQUIRE(log_split >= 0.0f, "gs_densify_select: log_split < 0");
  const int64_t nb = ceil_div(n > 0 ? n : 1, kDenThreads);
  hipStream_t s = as_stream(stream);
  int64_t* block_sums = (int64_t*)ws;
  DenThresholds th{grad_threshold, max_log_scale_clone, min_opacity_logit, max_log_scale,
                   log_split};
  if (n > 0) {
    hipLaunchKernelGGL(k_densify_select, dim3((unsigned)nb), dim3(kDenThreads), 0, s,
                       state->param[1], state->param[3], accum, denom, n, th, action, block_sums);
    GS_LAUNCH_CHECK("gs_densify_select");
  } else {
    gs_status z = gs_zero(block_sums, sizeof(int64_t), stream);
    if (z != GS_OK) return z;
  }
  hipLaunchKernelGGL(k_densify_scan, dim3(1), dim3(kDenThreads), 0, s, block_sums, nb, n_out);
  GS_LAUNCH_CHECK("gs_densify_select/scan");
  return GS_OK;
}

gs_status gs_densify_apply(const gs_gaussian_state* in, const int32_t* action, const void* ws,
                           const float* z, float log_split, gs_gaussian_state* out,
                           void* stream) {
  clear_error();
  GS_REQUIRE(state_ok(in) && state_ok(out), "gs_densify_apply: bad state (NULL arrays or n < 0)");
  GS_REQUIRE(in->n == 0 || (action && ws && z), "gs_densify_apply: NULL action/workspace/z");
  GS_REQUIRE((in->color_rows > 0 ? in->color_rows : 3) == (out->color_rows > 0 ? out->color_rows : 3),
             "gs_densify_apply: colour rows differ (%d in, %d out)", in->color_rows,
             out->color_rows);
  for (int i = 0; i < 5; ++i)
    GS_REQUIRE(out->n == 0 || in->n == 0 || ((in->m[i] == nullptr) == (out->m[i] == nullptr)),
               "gs_densify_apply: moments given on one side only (group %d)", i);
  if (in->n == 0 || out->n == 0) return GS_OK;
  hipLaunchKernelGGL(k_densify_apply, dim3((unsigned)ceil_div(in->n, kDenThreads)),
                     dim3(kDenThreads), 0, as_stream(stream), den_state(in), action,
                     (const int64_t*)ws, z, log_split, den_state(out));
  GS_LAUNCH_CHECK("gs_densify_apply");
  return GS_OK;
}

gs_status gs_opacity_reset(gs_gaussian_state* state, float max_opacity_logit, void* stream) {
  clear_error();
  GS_REQUIRE(state_ok(state), "gs_opacity_reset: bad state");
  if (state->n == 0) return GS_OK;
  hipLaunchKernelGGL(k_opacity_reset, dim3((unsigned)ceil_div(state->n, kDenThreads)),
                     dim3(kDenThreads), 0, as_stream(stream), state->param[3], state->m[3],
                     state->v[3], state->n, max_opacity_logit);
  GS_LAUNCH_CHECK("gs_opacity_reset");
  return GS_OK;
}

}  // extern "C"
