// Ray setup and occupancy marching of one candidate pixel ray, shared by the
// march kernels and the mixed-precision step's preparation launch (which
// counts the samples of every candidate beside its table conversion).
//
// One wave owns one candidate pixel ray.  For the occupancy sampler the 64
// lanes test 64 consecutive lattice points t_k = (k+1/2) dt at a time
// (AABB membership and the cell's occupancy bit), and a ballot compacts the
// kept ones; the lattice range is first narrowed to the ray's AABB chord
// (with one point of margin each side, the exact per-point test decides).
#pragma once
#include "kernels.h"

namespace nsl {
namespace march_detail {

struct Ray {
  float o[3], d[3], s;
};

__device__ __forceinline__ Ray make_ray(const KeyframeStore& kf, uint32_t id, int& k, int& pix) {
  const int hw = kf.H * kf.W;
  k = (int)(id / (uint32_t)hw);
  pix = (int)(id - (uint32_t)k * (uint32_t)hw);
  const int v = pix / kf.W, u = pix - v * kf.W;
  Ray r;
  camera_ray(kf.pose + 12 * k, kf.intr + 4 * k, u, v, r.o, r.d, r.s);
  return r;
}

// Lattice index range [k0, k1] that can hold kept samples.
__device__ __forceinline__ bool lattice_range(const Ray& r, const MarchParams& mp, int& k0, int& k1) {
  float tmin = mp.t_near, tmax = mp.t_far;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (r.d[i] == 0.0f) {
      if (r.o[i] < mp.box.lo[i] || r.o[i] > mp.box.hi[i]) return false;
    } else {
      const float a = (mp.box.lo[i] - r.o[i]) / r.d[i];
      const float b = (mp.box.hi[i] - r.o[i]) / r.d[i];
      tmin = fmaxf(tmin, fminf(a, b));
      tmax = fminf(tmax, fmaxf(a, b));
    }
  }
  if (!(tmin <= tmax + 2.0f * mp.dt)) return false;
  k0 = max(0, (int)floorf(tmin / mp.dt - 0.5f) - 1);
  k1 = (int)ceilf(tmax / mp.dt) + 1;
  return true;
}

__device__ __forceinline__ bool keep_point(const Ray& r, int k, const MarchParams& mp,
                                           const uint32_t* __restrict__ occ, int G, float& t) {
#pragma clang fp contract(off)
  t = ((float)k + 0.5f) * mp.dt;
  if (!(t >= mp.t_near && t <= mp.t_far)) return false;
  int cell[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float x = pos_axis(r.o[i], r.d[i], t);
    if (!(x >= mp.box.lo[i] && x <= mp.box.hi[i])) return false;
    const float xn = normalise_axis(x, mp.box.lo[i], mp.box.inv[i]);
    cell[i] = min((int)__builtin_floorf(xn * (float)G), G - 1);
  }
  const uint32_t bit = (uint32_t)cell[0] + (uint32_t)G * ((uint32_t)cell[1] + (uint32_t)G * (uint32_t)cell[2]);
  return (occ[bit >> 5] >> (bit & 31u)) & 1u;
}

__device__ __forceinline__ float uniform_t(const MarchParams& mp, int i) {
#pragma clang fp contract(off)
  return mp.t_near + ((float)i + 0.5f) * mp.dt;
}

constexpr int kWavesPerBlock = 4;

// The ray record, target and sample count of candidate r (one wave; 256
// threads a workgroup, block b takes candidates 4b .. 4b + 3).
__device__ __forceinline__ void rays_count_block(const KeyframeStore& kf, const MarchParams& mp,
                                                 const uint32_t* __restrict__ ids, int n, const RayBuffers& rb,
                                                 int block) {
  const int r = block * kWavesPerBlock + (int)threadIdx.x / kWave;
  if (r >= n) return;
  const int lane = lane_id();
  if (ids[r] >= (uint32_t)kf.K * (uint32_t)(kf.H * kf.W)) {  // not a stored pixel: empty ray
    if (lane == 0) {
      rb.rays[2 * r] = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
      rb.rays[2 * r + 1] = make_float4(0.0f, 0.0f, 1.0f, 0.0f);
      rb.target[r] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      rb.prec[r] = 0.0f;
      rb.counts[r] = 0;
    }
    return;
  }
  int k, pix;
  const Ray ray = make_ray(kf, ids[r], k, pix);
  if (lane == 0) {
    rb.rays[2 * r] = make_float4(ray.o[0], ray.o[1], ray.o[2], ray.s);
    rb.rays[2 * r + 1] = make_float4(ray.d[0], ray.d[1], ray.d[2], 0.0f);
    const size_t p = (size_t)k * kf.H * kf.W + pix;
    const float2 dp = depth_target(kf.depth[p], kf.var[p], ray.s);
    rb.target[r] = make_float4(kf.rgb[3 * p], kf.rgb[3 * p + 1], kf.rgb[3 * p + 2], dp.x);
    rb.prec[r] = dp.y;
  }
  uint32_t count = 0;
  if (mp.sampler == 0) {
    count = (uint32_t)mp.n_uniform;
  } else {
    int k0, k1;
    if (lattice_range(ray, mp, k0, k1)) {
      for (int kb = k0; kb <= k1 && count < (uint32_t)mp.max_per_ray; kb += kWave) {
        float t;
        const int kk = kb + lane;
        const bool keep = kk <= k1 && keep_point(ray, kk, mp, kf.occ, kf.grid_res, t);
        count += (uint32_t)__popcll(__ballot(keep));
      }
    }
    count = min(count, (uint32_t)mp.max_per_ray);
  }
  if (lane == 0) rb.counts[r] = count;
}

}  // namespace march_detail
}  // namespace nsl
