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
// clamped to N-1; f = xn*N - i0 and g = (i0 + 1) - xn*N, each rounded once
// from the exact product (ph - i0 and (i0 + 1) - ph are exact), so both
// trilinear factors keep full relative precision: 1 - f formed from a
// rounded f loses it when f is near 1.
__device__ __forceinline__ int cell_floor(float xn, int n, float& f, float& g) {
  // no contraction: fused, xn*N - i would be rounded once with the product's
  // error inside it, and adding pl would count that error twice
#pragma clang fp contract(off)
  const float nf = (float)n;
  const float ph = xn * nf;
  const float pl = __builtin_fmaf(xn, nf, -ph);
  float fl = __builtin_floorf(ph);
  if (ph == fl && pl < 0.0f) fl -= 1.0f;
  int i = (int)fl;
  if (i > n - 1) i = n - 1;
  f = (ph - (float)i) + pl;
  g = ((float)(i + 1) - ph) - pl;
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

// A pixel's depth target along its ray and the precision of its measurement
// (Eq. 4 read with Sigma_D a variance): (D_z s, 1 / (Sigma_z s^2)) when D_z
// and Sigma_z are finite and Sigma_z > 0, else (0, 0): an unusable
// measurement carries no depth loss.
__device__ __forceinline__ float2 depth_target(float Dz, float Vz, float s) {
  const bool ok = isfinite(Dz) && isfinite(Vz) && Vz > 0.0f;
  return ok ? make_float2(Dz * s, 1.0f / (Vz * s * s)) : make_float2(0.0f, 0.0f);
}

// One ray's terms of the mapping loss (Eq. 3, 4, 7) and the seeds of its
// adjoint: l_rgb = |I* - I|^2, l_d = pi (d* - D)^2, dL/dI* = k_rgb (I* - I),
// dL/dd* = k_d pi (d* - D), with the caller's factors k (2/R times the loss
// scale, times lambda_D for the depth term, in the step).
struct RayLoss {
  float l_rgb, l_d, gC[3], gD;
};
__device__ __forceinline__ RayLoss ray_loss(const float C[3], float D, float4 target, float pi, float k_rgb,
                                            float k_d) {
  RayLoss o;
  const float e0 = C[0] - target.x, e1 = C[1] - target.y, e2 = C[2] - target.z, ed = D - target.w;
  o.l_rgb = e0 * e0 + e1 * e1 + e2 * e2;
  o.l_d = pi * ed * ed;
  o.gC[0] = k_rgb * e0;
  o.gC[1] = k_rgb * e1;
  o.gC[2] = k_rgb * e2;
  o.gD = k_d * pi * ed;
  return o;
}

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

// Whether this lane starts a run of row_cell_runs below (a valid lane whose
// lower row neighbour is invalid, outside the row or in another cell).
__device__ __forceinline__ bool row_run_head(const uint32_t cell[3], bool valid) {
  const int r = threadIdx.x & 15;
  const int vb = row_from_below<1>((int)valid);  // every DPP read with all lanes active
  uint32_t cb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) cb[i] = (uint32_t)row_from_below<1>((int)cell[i]);
  bool same_below = valid & (r != 0) & (vb != 0);
#pragma unroll
  for (int i = 0; i < 3; ++i) same_below &= cb[i] == cell[i];
  return valid & !same_below;
}

// Runs of consecutive valid lanes of each 16-lane row whose samples lie in
// the same grid cell (equal cell coordinates).  Such lanes share all eight
// corner entries, so one run structure serves every value: a segmented
// suffix sum gives the first lane of each run the sums of v[0..K) over the
// run.  Returns whether this lane starts a run.  When no lane of the wave
// shares its cell with the lane below, the scan is skipped (every lane is
// its own run and keeps its values).
template <int K>
__device__ __forceinline__ bool row_cell_runs(const uint32_t cell[3], bool valid, float (&v)[K]) {
  const int r = threadIdx.x & 15;
  // every neighbour read first, with all lanes active: a DPP read under a
  // partial exec mask (a short-circuit && would make it one) sees inactive
  // lanes as zero
  const int vb = row_from_below<1>((int)valid), va = row_from_above<1>((int)valid);
  uint32_t cb[3], ca[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    cb[i] = (uint32_t)row_from_below<1>((int)cell[i]);
    ca[i] = (uint32_t)row_from_above<1>((int)cell[i]);
  }
  bool same_below = valid & (r != 0) & (vb != 0);
  bool same_above = valid & (r != 15) & (va != 0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    same_below &= cb[i] == cell[i];
    same_above &= ca[i] == cell[i];
  }
  if (__ballot(same_below) == 0ull) return true;
  int tail = same_above ? 0 : 1;  // the run continues above this lane
#define NSL_RUN_STEP(N)                                               \
  {                                                                   \
    const int nt = row_from_above<N>(tail);                           \
    float nv[K];                                                      \
    _Pragma("unroll") for (int k = 0; k < K; ++k) nv[k] = row_from_above<N>(v[k]); \
    if (!tail) {                                                      \
      _Pragma("unroll") for (int k = 0; k < K; ++k) v[k] += nv[k];    \
      tail = nt;                                                      \
    }                                                                 \
  }
  // once every lane's sum reaches the end of its run (no lane still has a
  // continuation), the remaining steps would add nothing: runs of one or two
  // samples, the usual case at the middle levels, stop after the first step
  NSL_RUN_STEP(1)
  if (__ballot(!tail) == 0ull) return !same_below;
  NSL_RUN_STEP(2)
  if (__ballot(!tail) == 0ull) return !same_below;
  NSL_RUN_STEP(4)
  if (__ballot(!tail) == 0ull) return !same_below;
  NSL_RUN_STEP(8)
#undef NSL_RUN_STEP
  return !same_below;
}

// The 64-bit word of a (g0, g1) float pair after adding (a, b): the step of
// a compare-and-swap accumulation of both features at once.
__device__ __forceinline__ unsigned long long add_pair_bits(unsigned long long v, float a, float b) {
  const float x = __uint_as_float((unsigned)(v & 0xFFFFFFFFull)) + a;
  const float y = __uint_as_float((unsigned)(v >> 32)) + b;
  return (unsigned long long)__float_as_uint(x) | ((unsigned long long)__float_as_uint(y) << 32);
}

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

}  // namespace nsl
