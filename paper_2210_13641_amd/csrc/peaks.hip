// Machine-peak probes on gfx950: the denominators of the measured roofline
// fractions.  A stream copy (HBM bandwidth), random 4-byte gathers from a
// table small enough to stay in L2 or the Infinity Cache (the access pattern
// of the hash-grid encoding), and MFMA loops in FP32 and BF16 (the MLP's
// instructions).  None of them is part of the mapping step.
#include "kernels.h"

namespace nsl {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// dst = src, 16 bytes per access, four in flight per thread.
__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                   size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// Random 4-byte reads: every thread reads `loads` entries of the table at
// indices drawn by a 32-bit xorshift generator seeded from its thread id,
// sixteen reads in flight, and stores the xor of what it read (so that no
// read can be dropped).
__global__ __launch_bounds__(256) void gather_kernel(const uint32_t* __restrict__ table, uint32_t mask,
                                                     uint32_t* __restrict__ out, int loads) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t x = tid * 2654435761u + 0x9E3779B9u;
  x ^= x >> 16;
  uint32_t acc = 0u;
  for (int k = 0; k < loads; k += 16) {
    uint32_t idx[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      x ^= x << 13;
      x ^= x >> 17;
      x ^= x << 5;
      idx[j] = x & mask;
    }
    uint32_t v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = table[idx[j]];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc ^= v[j];
  }
  out[tid] = acc;
}

// Eight independent MFMA accumulation chains per wave, `iters` rounds.
__global__ __launch_bounds__(256) void mfma_bf16_kernel(float* __restrict__ out, int iters) {
  const float s = (float)(threadIdx.x & 63) * 1e-3f;
  bf8 a, b;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = (__bf16)(s + (float)j);
    b[j] = (__bf16)(s - (float)j);
  }
  f4 c[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[k], 0, 0, 0);
  }
  float r = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) r += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

__global__ __launch_bounds__(256) void mfma_f32_kernel(float* __restrict__ out, int iters) {
  const float a = (float)(threadIdx.x & 63) * 1e-3f, b = 1.0f - a;
  f4 c[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[k], 0, 0, 0);
  }
  float r = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) r += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

}  // namespace

hipError_t peak_copy(const void* src, void* dst, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 16;
  if (n == 0) return hipSuccess;
  const size_t want = (n + 1023) / 1024;
  const unsigned grid = (unsigned)(want < 65536 ? want : 65536);
  hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, st, static_cast<const float4*>(src),
                     static_cast<float4*>(dst), n);
  return hipGetLastError();
}

hipError_t peak_gather(const uint32_t* table, int log2_entries, uint32_t* out, int n_threads, int loads,
                       hipStream_t st) {
  if (n_threads <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)(n_threads / 256)), dim3(256), 0, st, table,
                     (uint32_t)((1u << log2_entries) - 1u), out, loads);
  return hipGetLastError();
}

hipError_t peak_mfma(int bf16, float* out, int n_workgroups, int iters, hipStream_t st) {
  if (n_workgroups <= 0) return hipSuccess;
  if (bf16)
    hipLaunchKernelGGL(mfma_bf16_kernel, dim3((unsigned)n_workgroups), dim3(256), 0, st, out, iters);
  else
    hipLaunchKernelGGL(mfma_f32_kernel, dim3((unsigned)n_workgroups), dim3(256), 0, st, out, iters);
  return hipGetLastError();
}

}  // namespace nsl
