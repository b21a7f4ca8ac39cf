// Rays, samples and the batch cut of the mapping step on gfx950.
//
// The first pass sets up every candidate ray and counts its samples (one
// wave a ray, march_common.h), a scan turns counts into offsets and applies
// the batch cut, the second pass writes the samples.  Up to kEmitScanMax
// candidates the second pass does the scan itself (each workgroup the prefix
// before its candidates, one more workgroup the statistics), else a
// single-block scan runs between the two.
#include "march_common.h"

namespace nsl {

namespace {

using namespace march_detail;

__global__ __launch_bounds__(256) void rays_count_kernel(KeyframeStore kf, MarchParams mp,
                                                         const uint32_t* __restrict__ ids, int n,
                                                         RayBuffers rb) {
  rays_count_block(kf, mp, ids, n, rb, (int)blockIdx.x);
}

constexpr int kScanThreads = 1024;

// Single-block exclusive scan of the counts, batch cut and statistics, over
// segments of 4 * kScanThreads rays: each thread loads four consecutive rays
// (counts and precisions, one 16-byte load each), a wave scan (DPP) and the
// totals of the waves before give its exclusive offset, and the segment's
// total carries over to the next.
__global__ __launch_bounds__(kScanThreads) void scan_cut_kernel(RayBuffers rb, int n, int max_samples) {
  __shared__ uint32_t wtot[kScanThreads / kWave];
  __shared__ uint32_t red[3][kScanThreads / kWave];
  const int tid = threadIdx.x, wave = tid / kWave;
  uint32_t carry = 0, nr = 0, nk = 0, nm = 0;
  for (int seg = 0; seg < n; seg += 4 * kScanThreads) {
    const int i0 = seg + 4 * tid;
    uint32_t cr[4] = {0u, 0u, 0u, 0u};
    bool pz[4] = {false, false, false, false};
    if (i0 + 4 <= n) {
      const uint4 c4 = *reinterpret_cast<const uint4*>(rb.counts + i0);
      const float4 p4 = *reinterpret_cast<const float4*>(rb.prec + i0);
      cr[0] = c4.x; cr[1] = c4.y; cr[2] = c4.z; cr[3] = c4.w;
      pz[0] = p4.x == 0.0f; pz[1] = p4.y == 0.0f; pz[2] = p4.z == 0.0f; pz[3] = p4.w == 0.0f;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (i0 + k < n) {
          cr[k] = rb.counts[i0 + k];
          pz[k] = rb.prec[i0 + k] == 0.0f;
        }
      }
    }
    const uint32_t sum = cr[0] + cr[1] + cr[2] + cr[3];
    const uint32_t incl = wave_incl_scan_u32(sum);
    if (lane_id() == kWave - 1) wtot[wave] = incl;
    __syncthreads();
    uint32_t run = carry + incl - sum, total = 0;  // exclusive
    for (int w = 0; w < kScanThreads / kWave; ++w) {
      run += w < wave ? wtot[w] : 0u;
      total += wtot[w];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (i0 + k < n) {
        rb.offsets[i0 + k] = run;
        run += cr[k];
        if (run <= (uint32_t)max_samples) {
          ++nk;
          if (cr[k] > 0) {
            ++nr;
            if (pz[k]) ++nm;
          }
        }
      }
    }
    carry += total;
    __syncthreads();
  }
  if (tid == 0) rb.offsets[n] = carry;
  // reductions
  for (int o = 32; o > 0; o >>= 1) {
    nr += __shfl_xor(nr, o, kWave);
    nk += __shfl_xor(nk, o, kWave);
    nm += __shfl_xor(nm, o, kWave);
  }
  if (lane_id() == 0) {
    red[0][tid / kWave] = nr;
    red[1][tid / kWave] = nk;
    red[2][tid / kWave] = nm;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t R = 0, K = 0, M = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) {
      R += red[0][w];
      K += red[1][w];
      M += red[2][w];
    }
    rb.stats[0] = R;
    rb.stats[1] = K > 0 ? rb.offsets[K] : 0u;
    rb.stats[2] = K;
    rb.stats[3] = M;
    if (rb.loss) rb.loss[0] = rb.loss[1] = rb.loss[2] = 0.0f;
  }
}

// The statistics of the batch cut alone (R, S, kept, masked, as
// scan_cut_kernel leaves them), by one workgroup of 256 threads: each thread
// takes a contiguous run of candidates, a scan of the run totals gives its
// offset, and a second pass over its run counts what the cut keeps.
constexpr int kStatsThreads = 256;
__device__ __forceinline__ void cut_stats_block(const RayBuffers& rb, int n, int max_samples) {
  __shared__ uint32_t wtot[kStatsThreads / kWave];
  __shared__ uint32_t red[4][kStatsThreads / kWave];
  const int tid = threadIdx.x, wave = tid / kWave, lane = lane_id();
  const int per = (n + kStatsThreads - 1) / kStatsThreads;
  const int i0 = min(n, tid * per), i1 = min(n, i0 + per);
  // (sixteen loads in flight a thread, in both passes)
  uint32_t sum = 0;
  for (int c = i0; c < i1; c += 16) {
    uint32_t v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = c + k < i1 ? rb.counts[c + k] : 0u;
#pragma unroll
    for (int k = 0; k < 16; ++k) sum += v[k];
  }
  const uint32_t incl = wave_incl_scan_u32(sum);
  if (lane == kWave - 1) wtot[wave] = incl;
  __syncthreads();
  uint32_t run = incl - sum;
  for (int w = 0; w < wave; ++w) run += wtot[w];
  uint32_t nr = 0, nk = 0, nm = 0, smax = 0;
  for (int c = i0; c < i1; c += 16) {
    uint32_t v[16];
    bool pz[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      v[k] = c + k < i1 ? rb.counts[c + k] : 0u;
      pz[k] = c + k < i1 && rb.prec[c + k] == 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (c + k >= i1) continue;
      run += v[k];
      if (run <= (uint32_t)max_samples) {  // kept candidates are a prefix
        ++nk;
        smax = run;
        if (v[k] > 0) {
          ++nr;
          if (pz[k]) ++nm;
        }
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    nr += __shfl_xor(nr, o, kWave);
    nk += __shfl_xor(nk, o, kWave);
    nm += __shfl_xor(nm, o, kWave);
    smax = max(smax, (uint32_t)__shfl_xor((int)smax, o, kWave));
  }
  if (lane == 0) {
    red[0][wave] = nr;
    red[1][wave] = nk;
    red[2][wave] = nm;
    red[3][wave] = smax;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t R = 0, K = 0, M = 0, S = 0;
    for (int w = 0; w < kStatsThreads / kWave; ++w) {
      R += red[0][w];
      K += red[1][w];
      M += red[2][w];
      S = max(S, red[3][w]);
    }
    rb.stats[0] = R;
    rb.stats[1] = S;
    rb.stats[2] = K;
    rb.stats[3] = M;
    if (rb.loss) rb.loss[0] = rb.loss[1] = rb.loss[2] = 0.0f;
  }
}

// The samples of each kept candidate (one wave a candidate).  kScan: the
// launch also does what scan_cut_kernel would (for at most kEmitScanMax
// candidates): each workgroup sums the counts before its first candidate
// (sixteen loads in flight per thread) and writes its candidates' offsets,
// and one more workgroup, the first (so that it starts first), sets the
// statistics.
constexpr int kEmitScanMax = 16384;
template <bool kScan>
__global__ __launch_bounds__(256) void emit_kernel(KeyframeStore kf, MarchParams mp, int n,
                                                   RayBuffers rb, float* __restrict__ t_out,
                                                   uint32_t* __restrict__ ray_out) {
  const int w = (int)threadIdx.x / kWave, lane = lane_id();
  const int blk = kScan ? (int)blockIdx.x - 1 : (int)blockIdx.x;
  const int r = blk * kWavesPerBlock + w;
  uint32_t cnt, base;
  if (kScan) {
    if (blk < 0) {
      cut_stats_block(rb, n, mp.max_samples);
      return;
    }
    __shared__ uint32_t part[kWavesPerBlock], own[kWavesPerBlock];
    const int r0 = blk * kWavesPerBlock;
    uint32_t sum = 0;
    for (int i0 = 0; i0 < r0; i0 += 256 * 16) {
      uint32_t v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int i = i0 + 256 * k + (int)threadIdx.x;
        v[k] = i < r0 ? rb.counts[i] : 0u;
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) sum += v[k];
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, kWave);
    if (lane == 0) {
      part[w] = sum;
      own[w] = r < n ? rb.counts[r] : 0u;
    }
    __syncthreads();
    base = 0;
#pragma unroll
    for (int k = 0; k < kWavesPerBlock; ++k) base += part[k] + (k < w ? own[k] : 0u);
    cnt = own[w];
    if (r < n && lane == 0) {
      rb.offsets[r] = base;
      if (r == n - 1) rb.offsets[n] = base + cnt;
    }
    if (r >= n) return;
  } else {
    if (r >= n) return;
    cnt = rb.counts[r];
    base = rb.offsets[r];
  }
  if (cnt == 0 || base + cnt > (uint32_t)mp.max_samples) return;
  if (mp.sampler == 0) {
    for (int i = lane; i < (int)cnt; i += kWave) {
      t_out[base + i] = uniform_t(mp, i);
      ray_out[base + i] = (uint32_t)r;
    }
    return;
  }
  // the ray as the counting pass stored it (the same values make_ray gives)
  const float4 ro = rb.rays[2 * r], rd = rb.rays[2 * r + 1];
  Ray ray;
  ray.o[0] = ro.x; ray.o[1] = ro.y; ray.o[2] = ro.z; ray.s = ro.w;
  ray.d[0] = rd.x; ray.d[1] = rd.y; ray.d[2] = rd.z;
  int k0, k1;
  if (!lattice_range(ray, mp, k0, k1)) return;
  uint32_t done = 0;
  for (int kb = k0; kb <= k1 && done < cnt; kb += kWave) {
    float t = 0.0f;
    const int kk = kb + lane;
    const bool keep = kk <= k1 && keep_point(ray, kk, mp, kf.occ, kf.grid_res, t);
    const uint64_t mask = __ballot(keep);
    const uint32_t before = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    if (keep && done + before < cnt) {
      t_out[base + done + before] = t;
      ray_out[base + done + before] = (uint32_t)r;
    }
    done += (uint32_t)__popcll(mask);
  }
}

}  // namespace

size_t march_block_count(int n) {
  return (size_t)(n + march_detail::kWavesPerBlock - 1) / march_detail::kWavesPerBlock;
}

// The emit does the scan itself for 1 <= n <= kEmitScanMax candidates.
static bool emit_scans(int n) { return n >= 1 && n <= kEmitScanMax; }

hipError_t march_rays(const KeyframeStore& kf, const MarchParams& mp, const uint32_t* ids, int n,
                      const RayBuffers& rb, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(rays_count_kernel, dim3(march_block_count(n)), dim3(256), 0, st, kf, mp, ids, n, rb);
  return march_scan(mp, n, rb, st);
}

hipError_t march_scan(const MarchParams& mp, int n, const RayBuffers& rb, hipStream_t st) {
  if (!emit_scans(n)) hipLaunchKernelGGL(scan_cut_kernel, dim3(1), dim3(kScanThreads), 0, st, rb, n, mp.max_samples);
  return hipGetLastError();
}

hipError_t march_emit(const KeyframeStore& kf, const MarchParams& mp, const uint32_t* /*ids*/, int n,
                      const RayBuffers& rb, float* t_out, uint32_t* ray_out, hipStream_t st) {
  // the rays come from rb, stored by the counting pass from ids
  if (emit_scans(n))
    hipLaunchKernelGGL(emit_kernel<true>, dim3(march_block_count(n) + 1), dim3(256), 0, st, kf, mp, n, rb, t_out,
                       ray_out);
  else if (n > 0)
    hipLaunchKernelGGL(emit_kernel<false>, dim3(march_block_count(n)), dim3(256), 0, st, kf, mp, n, rb, t_out,
                       ray_out);
  return hipGetLastError();
}

}  // namespace nsl
