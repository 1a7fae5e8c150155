// adam.hip — dense bias-corrected Adam over up to GS_MAX_ADAM_GROUPS
// parameter groups in one launch (the optimiser of the 3D-GS training step
// the paper's Sec. II runs per partition).  Element-wise and HBM-bound:
// 16 bytes read + 12 bytes written per element (+4 when clearing the
// gradient); float4 accesses where a group is 16-byte aligned.
#include <math.h>

#include "gs_device.h"

namespace gsmi {

struct AdamGroupDev {
  float* p;
  float* g;
  float* m;
  float* v;
  int64_t n;
  float lr;
  int vec4;
};

struct AdamArgs {
  AdamGroupDev grp[GS_MAX_ADAM_GROUPS];
  int n_groups;
  float b1, b2, eps, ibc1, ibc2, zero_grad;
  // device schedule (gs_adam_dev): step count on the device, log-linear lr decay
  const int32_t* step_dev;
  float lr_final[GS_MAX_ADAM_GROUPS];
  int32_t decay_steps;
};

// Learning rate and bias corrections of the step the device counter names.
__device__ __forceinline__ void device_schedule(const AdamArgs& A, const AdamGroupDev& G,
                                                float& lr, float& ibc1, float& ibc2) {
  adam_schedule(A.step_dev[0] + 1, A.b1, A.b2, G.lr, A.lr_final[blockIdx.y], A.decay_steps, lr,
                ibc1, ibc2);
}

__device__ __forceinline__ void adam_one(float& p, float& g, float& m, float& v, float lr,
                                         float ibc1, float ibc2, const AdamArgs& A) {
  adam_update(p, g, m, v, lr, ibc1, ibc2, A.b1, A.b2, A.eps);
}

__global__ __launch_bounds__(256) void k_adam(AdamArgs A) {
  const AdamGroupDev& G = A.grp[blockIdx.y];
  float lr = G.lr, ibc1 = A.ibc1, ibc2 = A.ibc2;
  if (A.step_dev) device_schedule(A, G, lr, ibc1, ibc2);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const bool zero = A.zero_grad != 0.0f;
  if (G.vec4) {
    const int64_t n4 = G.n >> 2;
    float4* p4 = reinterpret_cast<float4*>(G.p);
    float4* g4 = reinterpret_cast<float4*>(G.g);
    float4* m4 = reinterpret_cast<float4*>(G.m);
    float4* v4 = reinterpret_cast<float4*>(G.v);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
      float4 p = p4[i], g = g4[i], m = m4[i], v = v4[i];
      adam_one(p.x, g.x, m.x, v.x, lr, ibc1, ibc2, A);
      adam_one(p.y, g.y, m.y, v.y, lr, ibc1, ibc2, A);
      adam_one(p.z, g.z, m.z, v.z, lr, ibc1, ibc2, A);
      adam_one(p.w, g.w, m.w, v.w, lr, ibc1, ibc2, A);
      p4[i] = p;
      m4[i] = m;
      v4[i] = v;
      if (zero) g4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    for (int64_t i = (n4 << 2) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G.n; i += stride) {
      float p = G.p[i], g = G.g[i], m = G.m[i], v = G.v[i];
      adam_one(p, g, m, v, lr, ibc1, ibc2, A);
      G.p[i] = p;
      G.m[i] = m;
      G.v[i] = v;
      if (zero) G.g[i] = 0.0f;
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G.n; i += stride) {
      float p = G.p[i], g = G.g[i], m = G.m[i], v = G.v[i];
      adam_one(p, g, m, v, lr, ibc1, ibc2, A);
      G.p[i] = p;
      G.m[i] = m;
      G.v[i] = v;
      if (zero) G.g[i] = 0.0f;
    }
  }
}

__global__ void k_step_inc(int32_t* step_dev) {
  if (threadIdx.x == 0) step_dev[0] += 1;
}

static gs_status adam_fill(const gs_adam_group* groups, int32_t n_groups, float beta1,
                           float beta2, float eps, int32_t zero_grad, AdamArgs& A,
                           int64_t& maxn, const char* who) {
  GS_REQUIRE(groups != nullptr || n_groups == 0, "%s: NULL groups", who);
  GS_REQUIRE(n_groups >= 0 && n_groups <= GS_MAX_ADAM_GROUPS, "%s: n_groups=%d outside [0, %d]",
             who, n_groups, GS_MAX_ADAM_GROUPS);
  GS_REQUIRE(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f, "%s: bad betas", who);
  maxn = 0;
  for (int i = 0; i < n_groups; ++i) {
    const gs_adam_group& g = groups[i];
    GS_REQUIRE(g.count >= 0, "%s: group %d count < 0", who, i);
    GS_REQUIRE(g.count == 0 || (g.param && g.grad && g.m && g.v), "%s: group %d NULL", who, i);
    A.grp[i].p = g.param;
    A.grp[i].g = g.grad;
    A.grp[i].m = g.m;
    A.grp[i].v = g.v;
    A.grp[i].n = g.count;
    A.grp[i].lr = g.lr;
    uintptr_t al = (uintptr_t)g.param | (uintptr_t)g.grad | (uintptr_t)g.m | (uintptr_t)g.v;
    A.grp[i].vec4 = (al & 15) == 0;
    if (g.count > maxn) maxn = g.count;
  }
  A.n_groups = n_groups;
  A.b1 = beta1;
  A.b2 = beta2;
  A.eps = eps;
  A.zero_grad = zero_grad ? 1.0f : 0.0f;
  A.step_dev = nullptr;
  A.decay_steps = 0;
  for (int i = 0; i < GS_MAX_ADAM_GROUPS; ++i) A.lr_final[i] = 0.0f;
  return GS_OK;
}

static unsigned adam_blocks(int64_t maxn) {
  int64_t bx = ceil_div(ceil_div(maxn, 4), 256);
  int64_t cap = (int64_t)device_cu_count() * 8;
  return (unsigned)(bx > cap ? cap : bx);
}

}  // namespace gsmi

using namespace gsmi;

extern "C" {

gs_status gs_adam(const gs_adam_group* groups, int32_t n_groups, float beta1, float beta2,
                  float eps, int32_t step, int32_t zero_grad, void* stream) {
  clear_error();
  GS_REQUIRE(step >= 1, "gs_adam: step=%d < 1", step);
  AdamArgs A;
  int64_t maxn = 0;
  gs_status st = adam_fill(groups, n_groups, beta1, beta2, eps, zero_grad, A, maxn, "gs_adam");
  if (st != GS_OK || maxn == 0) return st;
  A.ibc1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)step)));
  A.ibc2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)step)));
  hipLaunchKernelGGL(k_adam, dim3(adam_blocks(maxn), (unsigned)n_groups), dim3(256), 0,
                     as_stream(stream), A);
  GS_LAUNCH_CHECK("gs_adam");
  return GS_OK;
}

gs_status gs_adam_dev(const gs_adam_group* groups, int32_t n_groups, const float* lr_final,
                      int32_t decay_steps, float beta1, float beta2, float eps, int32_t* step_dev,
                      int32_t zero_grad, void* stream) {
  clear_error();
  GS_REQUIRE(step_dev != nullptr, "gs_adam_dev: NULL step_dev");
  GS_REQUIRE(decay_steps >= 0, "gs_adam_dev: decay_steps < 0");
  AdamArgs A;
  int64_t maxn = 0;
  gs_status st = adam_fill(groups, n_groups, beta1, beta2, eps, zero_grad, A, maxn, "gs_adam_dev");
  if (st != GS_OK) return st;
  A.step_dev = step_dev;
  A.decay_steps = decay_steps;
  for (int i = 0; i < n_groups; ++i) {
    const float lf = lr_final ? lr_final[i] : 0.0f;
    GS_REQUIRE(!(lf > 0.0f) || groups[i].lr > 0.0f, "gs_adam_dev: decay needs lr > 0 (group %d)", i);
    A.lr_final[i] = lf;
  }
  A.ibc1 = A.ibc2 = 1.0f;
  hipStream_t s = as_stream(stream);
  if (maxn > 0) {
    hipLaunchKernelGGL(k_adam, dim3(adam_blocks(maxn), (unsigned)n_groups), dim3(256), 0, s, A);
    GS_LAUNCH_CHECK("gs_adam_dev");
  }
  hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, s, step_dev);
  GS_LAUNCH_CHECK("gs_adam_dev/step");
  return GS_OK;
}

}  // extern "C"
