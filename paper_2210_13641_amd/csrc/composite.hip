// Volume rendering (Eq. 5, 6), the mapping loss (Eq. 3, 4, 7) and their
// adjoint on gfx950.  One wave owns one ray and walks its samples 64 at a
// time; the transmittance exponent sum_{j<i} tau_j is a wave-level prefix
// scan carried across chunks, so T_i = exp(-prefix) never multiplies
// rounding errors along the ray.  Everything is FP32.
//
// Adjoint, for Q = sum_i w_i q_i:  dQ/dtau_k = T_{k+1} q_k - (Q - Q_{<=k})
// (q = c for colour, t for d*, 1 for the opacity A),
// dV*/dtau_k = [T_{k+1} u_k - (V* - V_{<=k})] - 2 d* (1 - A) dd*/dtau_k with
// u_i = (t_i - d*)^2; dL/dsigma_k = delta dL/dtau_k and dL/dc_k = g_C w_k.
#include "bins.h"

namespace nsl {

namespace {

constexpr int kWavesPerBlock = 4;

struct RaySums {
  float C[3], D, A, V;
};

// Bounds of ray r, or false if it is not composited.
__device__ __forceinline__ bool ray_span(const CompositeIO& io, int r, uint32_t& b, uint32_t& n) {
  b = io.off[r];
  if (io.counts) {
    n = io.counts[r];
    return n > 0 && b + n <= (uint32_t)io.max_samples;
  }
  n = io.off[r + 1] - b;
  return n > 0;
}

struct Chunk {
  float tau, T, Tn, w, t, c[3];
  bool on;
};

// Load chunk [i0, i0+64) of the ray and its transmittance given the carried
// exponent; returns the chunk's total tau.
__device__ __forceinline__ float load_chunk(const CompositeIO& io, uint32_t b, uint32_t n, uint32_t i0,
                                            float carry, Chunk& c) {
  const int lane = lane_id();
  const uint32_t i = i0 + lane;
  c.on = i < n;
  float sg = 0.0f;
  c.t = 0.0f;
  c.c[0] = c.c[1] = c.c[2] = 0.0f;
  if (c.on) {
    const uint32_t s = b + i;
    sg = io.sigma[s];
    c.t = io.t[s];
    c.c[0] = io.rgb[3 * s];
    c.c[1] = io.rgb[3 * s + 1];
    c.c[2] = io.rgb[3 * s + 2];
  }
  c.tau = sg * io.delta;
  const float incl = wave_incl_scan(c.tau);
  const float excl = incl - c.tau;
  c.T = expf(-(carry + excl));
  c.Tn = expf(-(carry + incl));
  const float alpha = -expm1f(-c.tau);
  c.w = c.on ? c.T * alpha : 0.0f;
  if (io.stop_T > 0.0f && c.T < io.stop_T) {
    c.w = 0.0f;
    c.on = false;
  }
  return __shfl(incl, kWave - 1, kWave);
}

// Forward sums of one ray (two passes: V* about the final d*).
__device__ __forceinline__ RaySums ray_forward(const CompositeIO& io, uint32_t b, uint32_t n) {
  RaySums r{};
  float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, D = 0.0f, A = 0.0f;
  float carry = 0.0f;
  for (uint32_t i0 = 0; i0 < n; i0 += kWave) {
    Chunk c;
    carry += load_chunk(io, b, n, i0, carry, c);
    C0 += c.w * c.c[0];
    C1 += c.w * c.c[1];
    C2 += c.w * c.c[2];
    D += c.w * c.t;
    A += c.w;
    if (io.stop_T > 0.0f && __ballot(c.on && lane_id() < (int)(n - i0)) == 0ull) break;
  }
  r.C[0] = wave_sum(C0);
  r.C[1] = wave_sum(C1);
  r.C[2] = wave_sum(C2);
  r.D = wave_sum(D);
  r.A = wave_sum(A);
  float V = 0.0f;
  carry = 0.0f;
  for (uint32_t i0 = 0; i0 < n; i0 += kWave) {
    Chunk c;
    carry += load_chunk(io, b, n, i0, carry, c);
    const float e = c.t - r.D;
    V += c.w * e * e;
    if (io.stop_T > 0.0f && __ballot(c.on && lane_id() < (int)(n - i0)) == 0ull) break;
  }
  r.V = wave_sum(V);
  return r;
}

// Adjoint of one ray for seeds (gC, gD, gV); writes dL/dsigma and dL/dc.
__device__ __forceinline__ void ray_backward(const CompositeIO& io, uint32_t b, uint32_t n,
                                             const RaySums& r, const float gC[3], float gD, float gV, float gA,
                                             float* __restrict__ g_sigma, float* __restrict__ g_rgb) {
  float carry = 0.0f, p0 = 0.0f, p1 = 0.0f, p2 = 0.0f, pD = 0.0f, pV = 0.0f, pA = 0.0f;
  const float kV = 2.0f * r.D * (1.0f - r.A);
  for (uint32_t i0 = 0; i0 < n; i0 += kWave) {
    Chunk c;
    carry += load_chunk(io, b, n, i0, carry, c);
    const float u = (c.t - r.D) * (c.t - r.D);
    const float q0 = wave_incl_scan(c.w * c.c[0]) + p0;
    const float q1 = wave_incl_scan(c.w * c.c[1]) + p1;
    const float q2 = wave_incl_scan(c.w * c.c[2]) + p2;
    const float qD = wave_incl_scan(c.w * c.t) + pD;
    const float qV = wave_incl_scan(c.w * u) + pV;
    const float qA = gA != 0.0f ? wave_incl_scan(c.w) + pA : 0.0f;
    const float dC0 = c.Tn * c.c[0] - (r.C[0] - q0);
    const float dC1 = c.Tn * c.c[1] - (r.C[1] - q1);
    const float dC2 = c.Tn * c.c[2] - (r.C[2] - q2);
    const float dD = c.Tn * c.t - (r.D - qD);
    const float dV = (c.Tn * u - (r.V - qV)) - kV * dD;
    const float dA = c.Tn - (r.A - qA);
    const float dtau = gC[0] * dC0 + gC[1] * dC1 + gC[2] * dC2 + gD * dD + gV * dV + gA * dA;
    const uint32_t i = i0 + lane_id();
    if (i < n) {
      const uint32_t s = b + i;
      g_sigma[s] = io.delta * dtau;
      g_rgb[3 * s] = gC[0] * c.w;
      g_rgb[3 * s + 1] = gC[1] * c.w;
      g_rgb[3 * s + 2] = gC[2] * c.w;
    }
    p0 = __shfl(q0, kWave - 1, kWave);
    p1 = __shfl(q1, kWave - 1, kWave);
    p2 = __shfl(q2, kWave - 1, kWave);
    pD = __shfl(qD, kWave - 1, kWave);
    pV = __shfl(qV, kWave - 1, kWave);
    pA = __shfl(qA, kWave - 1, kWave);
  }
}

__global__ __launch_bounds__(256) void composite_fwd_kernel(CompositeIO io) {
  const int r = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (r >= io.R) return;
  uint32_t b, n;
  RaySums s{};
  if (ray_span(io, r, b, n)) s = ray_forward(io, b, n);
  if (lane_id() == 0 && io.out6) {
    float* o = io.out6 + 6 * (size_t)r;
    o[0] = s.C[0]; o[1] = s.C[1]; o[2] = s.C[2]; o[3] = s.D; o[4] = s.V; o[5] = s.A;
  }
}

__global__ __launch_bounds__(256) void composite_bwd_kernel(CompositeIO io, const float* __restrict__ g_rgb,
                                                            const float* __restrict__ g_depth,
                                                            const float* __restrict__ g_var,
                                                            const float* __restrict__ g_opacity,
                                                            float* __restrict__ g_sigma,
                                                            float* __restrict__ g_rgb_s) {
  const int r = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (r >= io.R) return;
  uint32_t b, n;
  if (!ray_span(io, r, b, n)) return;
  const RaySums s = ray_forward(io, b, n);
  const float gC[3] = {g_rgb ? g_rgb[3 * r] : 0.0f, g_rgb ? g_rgb[3 * r + 1] : 0.0f,
                       g_rgb ? g_rgb[3 * r + 2] : 0.0f};
  ray_backward(io, b, n, s, gC, g_depth ? g_depth[r] : 0.0f, g_var ? g_var[r] : 0.0f,
               g_opacity ? g_opacity[r] : 0.0f, g_sigma, g_rgb_s);
}

// Rays of at most kCacheChunks * 64 samples (every training ray: the march
// caps them at 256) keep their chunks in registers, so the V* pass and the
// adjoint reuse the loads and the transmittance of the forward pass.
constexpr int kCacheChunks = 4;

__device__ __forceinline__ RaySums ray_forward_cached(const CompositeIO& io, uint32_t b, uint32_t n,
                                                      Chunk (&cc)[kCacheChunks]) {
  RaySums r{};
  float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, D = 0.0f, A = 0.0f;
  float carry = 0.0f;
#pragma unroll
  for (int k = 0; k < kCacheChunks; ++k) {
    const uint32_t i0 = (uint32_t)k * kWave;
    if (i0 < n) {
      carry += load_chunk(io, b, n, i0, carry, cc[k]);
      C0 += cc[k].w * cc[k].c[0];
      C1 += cc[k].w * cc[k].c[1];
      C2 += cc[k].w * cc[k].c[2];
      D += cc[k].w * cc[k].t;
      A += cc[k].w;
    }
  }
  r.C[0] = wave_sum(C0);
  r.C[1] = wave_sum(C1);
  r.C[2] = wave_sum(C2);
  r.D = wave_sum(D);
  r.A = wave_sum(A);
  float V = 0.0f;
#pragma unroll
  for (int k = 0; k < kCacheChunks; ++k) {
    if ((uint32_t)k * kWave < n) {
      const float e = cc[k].t - r.D;
      V += cc[k].w * e * e;
    }
  }
  r.V = wave_sum(V);
  return r;
}

__device__ __forceinline__ void ray_backward_cached(uint32_t b, uint32_t n, const RaySums& r,
                                                    const Chunk (&cc)[kCacheChunks], const float gC[3], float gD,
                                                    float delta, float* __restrict__ g_sigma,
                                                    float* __restrict__ g_rgb) {
  float p0 = 0.0f, p1 = 0.0f, p2 = 0.0f, pD = 0.0f;
#pragma unroll
  for (int k = 0; k < kCacheChunks; ++k) {
    const uint32_t i0 = (uint32_t)k * kWave;
    if (i0 < n) {
      const Chunk& c = cc[k];
      const float q0 = wave_incl_scan(c.w * c.c[0]) + p0;
      const float q1 = wave_incl_scan(c.w * c.c[1]) + p1;
      const float q2 = wave_incl_scan(c.w * c.c[2]) + p2;
      const float qD = wave_incl_scan(c.w * c.t) + pD;
      const float dC0 = c.Tn * c.c[0] - (r.C[0] - q0);
      const float dC1 = c.Tn * c.c[1] - (r.C[1] - q1);
      const float dC2 = c.Tn * c.c[2] - (r.C[2] - q2);
      const float dD = c.Tn * c.t - (r.D - qD);
      const float dtau = gC[0] * dC0 + gC[1] * dC1 + gC[2] * dC2 + gD * dD;
      const uint32_t i = i0 + lane_id();
      if (i < n) {
        const uint32_t s = b + i;
        g_sigma[s] = delta * dtau;
        g_rgb[3 * s] = gC[0] * c.w;
        g_rgb[3 * s + 1] = gC[1] * c.w;
        g_rgb[3 * s + 2] = gC[2] * c.w;
      }
      p0 = __shfl(q0, kWave - 1, kWave);
      p1 = __shfl(q1, kWave - 1, kWave);
      p2 = __shfl(q2, kWave - 1, kWave);
      pD = __shfl(qD, kWave - 1, kWave);
    }
  }
}

// Train step: forward sums, loss terms and seeds, adjoint.
__global__ __launch_bounds__(256) void composite_loss_kernel(CompositeIO io, LossIO lo,
                                                             float* __restrict__ g_sigma,
                                                             float* __restrict__ g_rgb_s, BinPrep bp) {
  // with bp.nbins, the last workgroup sets the table-gradient bin starts
  // (bins.h): they need only the column scan of the forward launch
  if (bp.nbins > 0 && blockIdx.x == gridDim.x - 1) {
    bin_start_block<256>(bp.rb, bp.nbins, bp.chunk, bp.split);
    return;
  }
  const int r = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (r >= io.R) return;
  uint32_t b, n;
  const bool on = ray_span(io, r, b, n);
  if (!on) {
    if (lane_id() == 0) {
      lo.parts[2 * r] = lo.parts[2 * r + 1] = 0.0f;
      if (lo.ray_out) {
        float* o = lo.ray_out + 6 * (size_t)r;
        o[0] = o[1] = o[2] = o[3] = o[4] = o[5] = 0.0f;
      }
    }
    return;
  }
  // no early termination in training (stop_T = 0): the cached path holds
  const bool cached = n <= (uint32_t)(kCacheChunks * kWave) && !(io.stop_T > 0.0f);
  Chunk cc[kCacheChunks];
  const RaySums s = cached ? ray_forward_cached(io, b, n, cc) : ray_forward(io, b, n);
  const float Rf = (float)lo.stats[0];
  const float scale = lo.scale_dev ? lo.scale_dev[0] : lo.loss_scale;
  const float k = 2.0f * scale / Rf;
  const RayLoss L = ray_loss(s.C, s.D, lo.target[r], lo.prec[r], k, k * lo.lambda_d);
  const float gC[3] = {L.gC[0], L.gC[1], L.gC[2]};
  const float gD = L.gD;
  if (lane_id() == 0) {
    lo.parts[2 * r] = L.l_rgb / Rf;
    lo.parts[2 * r + 1] = L.l_d / Rf;
    if (lo.ray_out) {
      const float sc = lo.rays[2 * r].w;
      float* o = lo.ray_out + 6 * (size_t)r;
      o[0] = s.C[0]; o[1] = s.C[1]; o[2] = s.C[2];
      o[3] = s.D / sc; o[4] = s.V / (sc * sc); o[5] = s.A;
    }
  }
  if (cached)
    ray_backward_cached(b, n, s, cc, gC, gD, io.delta, g_sigma, g_rgb_s);
  else
    ray_backward(io, b, n, s, gC, gD, 0.0f, 0.0f, g_sigma, g_rgb_s);
}

// The loss of rays rendered outside the step (out6 from compositing, ray
// units), one thread per ray: per-ray shares of L_rgb and L_D (divided by R)
// into parts, and with g_out the seeds of the adjoint for the upstream
// gradients g_loss of (L, L_rgb, L_D) (NULL: (1, 0, 0)); masked
// measurements are counted into n_masked.
__global__ __launch_bounds__(256) void loss_terms_kernel(const float* __restrict__ out6, int R,
                                                         const float* __restrict__ rgb_target,
                                                         const float* __restrict__ depth_z,
                                                         const float* __restrict__ var_z,
                                                         const float* __restrict__ ray_scale, float lambda_d,
                                                         const float* __restrict__ g_loss, float* __restrict__ parts,
                                                         float* __restrict__ g_out, uint32_t* __restrict__ n_masked) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = r < R;
  float2 dp = make_float2(0.0f, 0.0f);
  if (on) {
    const float* o = out6 + 6 * (size_t)r;
    const float C[3] = {o[0], o[1], o[2]};
    dp = depth_target(depth_z[r], var_z[r], ray_scale[r]);
    const float4 tg = make_float4(rgb_target[3 * r], rgb_target[3 * r + 1], rgb_target[3 * r + 2], dp.x);
    const float gL = g_loss ? g_loss[0] : 1.0f, gLr = g_loss ? g_loss[1] : 0.0f, gLd = g_loss ? g_loss[2] : 0.0f;
    const float Rf = (float)R;
    const RayLoss L = ray_loss(C, o[3], tg, dp.y, 2.0f * (gL + gLr) / Rf, 2.0f * (gL * lambda_d + gLd) / Rf);
    if (parts) {
      parts[2 * r] = L.l_rgb / Rf;
      parts[2 * r + 1] = L.l_d / Rf;
    }
    if (g_out) {
      float* g = g_out + 6 * (size_t)r;
      g[0] = L.gC[0]; g[1] = L.gC[1]; g[2] = L.gC[2]; g[3] = L.gD; g[4] = 0.0f; g[5] = 0.0f;
    }
  }
  if (n_masked) {
    const uint64_t bad = __ballot(on && dp.y == 0.0f);
    if (lane_id() == 0 && bad) atomicAdd(n_masked, (uint32_t)__popcll(bad));
  }
}

dim3 grid_for(int R) { return dim3((R + kWavesPerBlock - 1) / kWavesPerBlock); }

}  // namespace

hipError_t composite_forward(const CompositeIO& io, hipStream_t st) {
  if (io.R > 0) hipLaunchKernelGGL(composite_fwd_kernel, grid_for(io.R), dim3(256), 0, st, io);
  return hipGetLastError();
}

hipError_t composite_backward(const CompositeIO& io, const float* g_rgb, const float* g_depth,
                              const float* g_var, const float* g_opacity, float* g_sigma, float* g_rgb_s,
                              hipStream_t st) {
  if (io.R > 0)
    hipLaunchKernelGGL(composite_bwd_kernel, grid_for(io.R), dim3(256), 0, st, io, g_rgb, g_depth,
                       g_var, g_opacity, g_sigma, g_rgb_s);
  return hipGetLastError();
}

hipError_t loss_terms(const float* out6, int R, const float* rgb_target, const float* depth_z, const float* var_z,
                      const float* ray_scale, float lambda_d, const float* g_loss, float* parts, float* g_out,
                      uint32_t* n_masked, hipStream_t st) {
  if (R > 0)
    hipLaunchKernelGGL(loss_terms_kernel, dim3((R + 255) / 256), dim3(256), 0, st, out6, R, rgb_target, depth_z,
                       var_z, ray_scale, lambda_d, g_loss, parts, g_out, n_masked);
  return hipGetLastError();
}

hipError_t composite_loss_backward(const CompositeIO& io, const LossIO& lo, float* g_sigma,
                                   float* g_rgb_s, hipStream_t st, const BinPrep* bp) {
  const BinPrep none{};
  const BinPrep& b = bp ? *bp : none;
  const int grid = (int)grid_for(io.R).x + (b.nbins > 0 ? 1 : 0);
  if (grid > 0)
    hipLaunchKernelGGL(composite_loss_kernel, dim3(grid), dim3(256), 0, st, io, lo, g_sigma, g_rgb_s, b);
  return hipGetLastError();
}

}  // namespace nsl
