// Adam, buffer clearing and render ray setup on gfx950.
#include "kernels.h"

namespace nsl {

namespace {

// Bias-corrected Adam (dense), gradient = grads * gscale; clears grads.
// Streams 4 floats per thread per array: params, grads, m, v.
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   int64_t n, float lr, float b1, float b2,
                                                   float eps, float bc1, float bc2, float gscale) {
  const int64_t i4 = (int64_t)(blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * 4;
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

__global__ __launch_bounds__(256) void fill_zero_kernel(float* __restrict__ p, int64_t n) {
  const int64_t i4 = (int64_t)(blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * 4;
  if (i4 + 4 <= n) {
    *reinterpret_cast<float4*>(p + i4) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  } else {
    for (int64_t i = i4; i < n; ++i) p[i] = 0.0f;
  }
}

// One thread per pixel: ray record, uniform samples, offsets.
__global__ __launch_bounds__(256) void render_setup_kernel(const float* __restrict__ pose,
                                                           const float* __restrict__ intr, int H, int W,
                                                           float t_near, float dt, int n_samples,
                                                           float4* __restrict__ rays, float* __restrict__ t,
                                                           uint32_t* __restrict__ ray, uint32_t* __restrict__ off) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = H * W;
  if (r > n) return;
  off[r] = (uint32_t)r * (uint32_t)n_samples;
  if (r == n) return;
  const int v = r / W, u = r - v * W;
  float o[3], d[3], s;
  camera_ray(pose, intr, u, v, o, d, s);
  rays[2 * r] = make_float4(o[0], o[1], o[2], s);
  rays[2 * r + 1] = make_float4(d[0], d[1], d[2], 0.0f);
  for (int i = 0; i < n_samples; ++i) {
#pragma clang fp contract(off)
    t[(size_t)r * n_samples + i] = t_near + ((float)i + 0.5f) * dt;
    ray[(size_t)r * n_samples + i] = (uint32_t)r;
  }
}

__global__ __launch_bounds__(256) void render_finish_kernel(const float* __restrict__ out6,
                                                            const float4* __restrict__ rays, int n,
                                                            float* __restrict__ rgb, float* __restrict__ depth,
                                                            float* __restrict__ var, float* __restrict__ opacity) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const float* o = out6 + 6 * (size_t)r;
  const float s = rays[2 * r].w;
  rgb[3 * r] = o[0];
  rgb[3 * r + 1] = o[1];
  rgb[3 * r + 2] = o[2];
  depth[r] = o[3] / s;
  var[r] = o[4] / (s * s);
  if (opacity) opacity[r] = o[5];
}

}  // namespace

hipError_t adam_update(float* p, float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, int step, float grad_scale, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const float bc1 = 1.0f - powf(b1, (float)step);
  const float bc2 = 1.0f - powf(b2, (float)step);
  const int64_t threads = (n + 3) / 4;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, p, g, m, v,
                     n, lr, b1, b2, eps, bc1, bc2, grad_scale);
  return hipGetLastError();
}

hipError_t fill_zero(float* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t threads = (n + 3) / 4;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t render_setup(const float* pose, const float* intr, int H, int W, float t_near, float dt,
                        int n_samples, Aabb box, float4* rays, float* t, uint32_t* ray, uint32_t* off,
                        hipStream_t st) {
  (void)box;
  const int n = H * W + 1;
  hipLaunchKernelGGL(render_setup_kernel, dim3((n + 255) / 256), dim3(256), 0, st, pose, intr, H, W,
                     t_near, dt, n_samples, rays, t, ray, off);
  return hipGetLastError();
}

hipError_t render_finish(const float* out6, const float4* rays, int n, float* rgb, float* depth,
                         float* var, float* opacity, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(render_finish_kernel, dim3((n + 255) / 256), dim3(256), 0, st, out6, rays, n, rgb,
                       depth, var, opacity);
  return hipGetLastError();
}

}  // namespace nsl
