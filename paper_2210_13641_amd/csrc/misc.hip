// Adam, buffer clearing and small helpers on gfx950.
#include "kernels.h"

namespace nsl {

namespace {

// Bias-corrected Adam (dense), gradient = grads * gscale; clears grads.
// Streams 4 floats per thread per array: params, grads, m, v.
// With a loss-scale state, the step's gradient is unscaled by state[0], a
// step whose gradient overflowed (state[3]) only clears the gradient, and
// the bias correction counts the updates actually made: t = step - state[2]
// (the steps skipped before this one), at least 1.
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   int64_t n, float lr, float b1, float b2,
                                                   float eps, float bc1, float bc2, float gscale,
                                                   int step, const float* __restrict__ state) {
  const int64_t i4 = (int64_t)(blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * 4;
  if (state) {
    if (state[3] != 0.0f) {  // overflow: skip the update, clear the gradient
      for (int64_t i = i4; i < min(n, i4 + 4); ++i) g[i] = 0.0f;
      return;
    }
    gscale = 1.0f / state[0];
    const float t = fmaxf(1.0f, (float)step - state[2]);
    bc1 = 1.0f - powf(b1, t);
    bc2 = 1.0f - powf(b2, t);
  }
  if (i4 + 4 <= n) {
    float4 pp = *reinterpret_cast<float4*>(p + i4);
    float4 gg = *reinterpret_cast<float4*>(g + i4);
    float4 mm = *reinterpret_cast<float4*>(m + i4);
    float4 vv = *reinterpret_cast<float4*>(v + i4);
    float* P = &pp.x;
    float* G = &gg.x;
    float* M = &mm.x;
    float* V = &vv.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float gk = G[k] * gscale;
      M[k] = b1 * M[k] + (1.0f - b1) * gk;
      V[k] = b2 * V[k] + (1.0f - b2) * gk * gk;
      P[k] -= lr * (M[k] / bc1) / (sqrtf(V[k] / bc2) + eps);
    }
    *reinterpret_cast<float4*>(p + i4) = pp;
    *reinterpret_cast<float4*>(m + i4) = mm;
    *reinterpret_cast<float4*>(v + i4) = vv;
    *reinterpret_cast<float4*>(g + i4) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  } else {
    for (int64_t i = i4; i < n; ++i) {
      const float gk = g[i] * gscale;
      m[i] = b1 * m[i] + (1.0f - b1) * gk;
      v[i] = b2 * v[i] + (1.0f - b2) * gk * gk;
      p[i] -= lr * (m[i] / bc1) / (sqrtf(v[i] / bc2) + eps);
      g[i] = 0.0f;
    }
  }
}

// Clears p[0, n).
__global__ __launch_bounds__(256) void fill_zero_kernel(float* p, int64_t n) {
  const int64_t i4 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i4 + 4 <= n) {
    *reinterpret_cast<float4*>(p + i4) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  } else {
    for (int64_t i = i4; i < n; ++i) p[i] = 0.0f;
  }
}

__global__ void scale_begin_kernel(float* state) { state[3] = 0.0f; }

__global__ void scale_end_kernel(float* state) {
  if (state[3] != 0.0f) {
    state[0] *= 0.5f;
    state[1] = 0.0f;
    state[2] += 1.0f;
  } else {
    state[1] += 1.0f;
    if (state[1] >= 2000.0f) {
      state[0] *= 2.0f;
      state[1] = 0.0f;
    }
  }
}

__global__ void store_request_kernel(nsl_render_request r, const float* __restrict__ pose,
                                     const float* __restrict__ intr, nsl_render_request* dst) {
  for (int i = 0; i < 12; ++i) r.pose[i] = pose[i];
  for (int i = 0; i < 4; ++i) r.intr[i] = intr[i];
  *dst = r;
}

}  // namespace

hipError_t adam_update(float* p, float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, int step, float grad_scale, const float* scale_state,
                       hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const float bc1 = 1.0f - powf(b1, (float)step);
  const float bc2 = 1.0f - powf(b2, (float)step);
  const int64_t threads = (n + 3) / 4;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, p, g, m, v,
                     n, lr, b1, b2, eps, bc1, bc2, grad_scale, step, scale_state);
  return hipGetLastError();
}

hipError_t fill_zero(float* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)(((n + 3) / 4 + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t scale_begin(float* state, hipStream_t st) {
  hipLaunchKernelGGL(scale_begin_kernel, dim3(1), dim3(1), 0, st, state);
  return hipGetLastError();
}

hipError_t scale_end(float* state, hipStream_t st) {
  hipLaunchKernelGGL(scale_end_kernel, dim3(1), dim3(1), 0, st, state);
  return hipGetLastError();
}

hipError_t store_request(const nsl_render_request* r, const float* pose, const float* intr,
                         nsl_render_request* dst, hipStream_t st) {
  hipLaunchKernelGGL(store_request_kernel, dim3(1), dim3(1), 0, st, *r, pose, intr, dst);
  return hipGetLastError();
}

}  // namespace nsl
