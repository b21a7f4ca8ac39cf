// Device helpers shared by the gfx950 kernels of the mapping step.
//
// Sample positions decide integer quantities (occupancy cell, trilinear
// cell, AABB membership), so they are formed in IEEE single precision with
// every operation rounded separately, in a fixed order:
//   a = ((u + 0.5) - cx) / fx,  b = ((v + 0.5) - cy) / fy,
//   s = sqrt((a*a + b*b) + 1),  d_i = ((R_i0*a + R_i1*b) + R_i2) / s,
//   x_i = o_i + t*d_i,  xn_i = clamp((x_i - lo_i) * inv_i, 0, 1).
// Contraction into FMA is switched off in these functions, and division and
// square root are the correctly rounded ones (the library is built with
// -fhip-fp32-correctly-rounded-divide-sqrt), so any IEEE implementation of the
// same sequence lands on the same bits.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nsl {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
constexpr int kMaxLevels = 16;
constexpr uint32_t kPrime1 = 2654435761u;
constexpr uint32_t kPrime2 = 805459861u;

struct LevelInfo {
  int levels;
  uint32_t table_mask;          // table entries per hashed level - 1 (power of two)
  uint32_t dense_bits;          // bit l set: level l is dense
  int res[kMaxLevels];          // N_l
  uint32_t offset[kMaxLevels];  // first entry of level l
};

struct Aabb {
  float lo[3], hi[3], inv[3];
};

__device__ __forceinline__ void camera_ray(const float* __restrict__ pose,
                                           const float* __restrict__ intr, int u, int v,
                                           float o[3], float d[3], float& s) {
#pragma clang fp contract(off)
  const float a = (((float)u + 0.5f) - intr[2]) / intr[0];
  const float b = (((float)v + 0.5f) - intr[3]) / intr[1];
  s = __builtin_sqrtf((a * a + b * b) + 1.0f);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    d[i] = ((pose[4 * i] * a + pose[4 * i + 1] * b) + pose[4 * i + 2]) / s;
    o[i] = pose[4 * i + 3];
  }
}

__device__ __forceinline__ float pos_axis(float o, float d, float t) {
#pragma clang fp contract(off)
  return o + t * d;
}

__device__ __forceinline__ float normalise_axis(float x, float lo, float inv) {
#pragma clang fp contract(off)
  float xn = (x - lo) * inv;
  return fminf(fmaxf(xn, 0.0f), 1.0f);
}

// floor(xn*N) taken on the exact product (TwoProduct: xn*N = ph + pl exactly),
// clamped to N-1; f = xn*N - i0 rounded once.
__device__ __forceinline__ int cell_floor(float xn, int n, float& f) {
  const float nf = (float)n;
  const float ph = xn * nf;
  const float pl = __builtin_fmaf(xn, nf, -ph);
  float fl = __builtin_floorf(ph);
  if (ph == fl && pl < 0.0f) fl -= 1.0f;
  int i = (int)fl;
  if (i > n - 1) i = n - 1;
  f = (ph - (float)i) + pl;
  return i;
}

__device__ __forceinline__ uint32_t grid_index(uint32_t x, uint32_t y, uint32_t z, int n,
                                               bool dense, uint32_t mask) {
  if (dense) {
    const uint32_t m = (uint32_t)n + 1u;
    return x + m * (y + m * z);
  }
  return (x ^ (y * kPrime1) ^ (z * kPrime2)) & mask;
}

__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + __expf(-z)); }

// Wave-wide helpers (wave64).
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Inclusive scan across the wave.
__device__ __forceinline__ float wave_incl_scan(float v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    float n = __shfl_up(v, o, kWave);
    if (l >= o) v += n;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t n = __shfl_up(v, o, kWave);
    if (l >= o) v += n;
  }
  return v;
}

// DPP row shift towards lower lanes: lane i of each 16-lane row receives the
// value of lane i+N of the same row (0 when i+N leaves the row).
template <int N>
__device__ __forceinline__ int row_from_above(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x100 + N, 0xF, 0xF, true);
}
template <int N>
__device__ __forceinline__ float row_from_above(float v) {
  return __int_as_float(row_from_above<N>(__float_as_int(v)));
}
// Lane i receives lane i-N of its row (0 when i-N leaves the row).
template <int N>
__device__ __forceinline__ int row_from_below(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x110 + N, 0xF, 0xF, true);
}

// Runs of equal keys among consecutive lanes of each 16-lane row: the first
// lane of every run gets the sums of a and b over the run (segmented suffix
// scan); returns whether this lane starts a run.
__device__ __forceinline__ bool row_run_sums(uint32_t key, float& a, float& b) {
  const int r = threadIdx.x & 15;
  const uint32_t above = (uint32_t)row_from_above<1>((int)key);
  const uint32_t below = (uint32_t)row_from_below<1>((int)key);
  const bool head = r == 0 || below != key;
  int tail = (r == 15 || above != key) ? 1 : 0;  // a run ends within [r, r + span)
#define NSL_RUN_STEP(N)                               \
  {                                                   \
    const float na = row_from_above<N>(a);            \
    const float nb = row_from_above<N>(b);            \
    const int nt = row_from_above<N>(tail);           \
    if (!tail) {                                      \
      a += na;                                        \
      b += nb;                                        \
      tail = nt;                                      \
    }                                                 \
  }
  NSL_RUN_STEP(1)
  NSL_RUN_STEP(2)
  NSL_RUN_STEP(4)
  NSL_RUN_STEP(8)
#undef NSL_RUN_STEP
  return head;
}

// p_k[0] += a_k, p_k[1] += b_k for K table entries, each as one 64-bit
// compare-and-swap (one memory-side atomic per entry instead of two: the two
// features of an entry share 8 aligned bytes).  All K reads, then all K
// swaps are issued before any result is awaited; only swaps that lost a race
// (or started from a stale read) go round again.
__device__ __forceinline__ unsigned long long add_pair_bits(unsigned long long v, float a, float b) {
  const float x = __uint_as_float((unsigned)(v & 0xFFFFFFFFull)) + a;
  const float y = __uint_as_float((unsigned)(v >> 32)) + b;
  return (unsigned long long)__float_as_uint(x) | ((unsigned long long)__float_as_uint(y) << 32);
}

template <int K>
__device__ __forceinline__ void atomic_add_pairs(float* const p[K], const bool on[K], const float a[K],
                                                 const float b[K]) {
  unsigned long long seen[K], got[K];
#pragma unroll
  for (int k = 0; k < K; ++k)
    seen[k] = on[k] ? __hip_atomic_load(reinterpret_cast<unsigned long long*>(p[k]), __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT)
                    : 0ull;
#pragma unroll
  for (int k = 0; k < K; ++k)
    got[k] = on[k] ? atomicCAS(reinterpret_cast<unsigned long long*>(p[k]), seen[k], add_pair_bits(seen[k], a[k], b[k]))
                   : seen[k];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    while (got[k] != seen[k]) {
      seen[k] = got[k];
      got[k] = atomicCAS(reinterpret_cast<unsigned long long*>(p[k]), seen[k], add_pair_bits(seen[k], a[k], b[k]));
    }
  }
}

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

}  // namespace nsl
