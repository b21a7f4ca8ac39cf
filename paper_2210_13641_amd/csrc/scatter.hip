// Table-gradient accumulation without global atomics on the hot path.
//
// The backward kernels do not add w_c * dL/de into the gradient table
// directly (the chain rule through the trilinear blend of Sec. 3.3's
// encoding: every sample adds to the 8 corner entries of every level).
// Device-coherent atomics on gfx950 retire at roughly one lane per clock per
// XCD whatever the address pattern, and under contention a compare-and-swap
// loop degrades much further, so each backward wave instead appends records
// (entry index, two feature gradients) to a region of its own.  The records
// are then partitioned by bin (2^13 consecutive entries) with a counting
// sort, and each bin is reduced in LDS by a workgroup that owns it:
//
//   count   per region, records per bin (LDS histogram)       [region][bin]
//   scan    per bin, exclusive prefix over regions; bin totals
//   start   exclusive prefix over bins; chunks of kChunk records per bin
//   place   records to their bin's slice (ordered by bin in LDS first)
//   reduce  one workgroup per chunk: LDS accumulation of the bin, then
//           grad += acc (a bin of one chunk owns its entries; chunks of a
//           bin with several use atomics, one per touched entry)
#include "kernels.h"

namespace nsl {

namespace {

constexpr int kCountThreads = 512;
constexpr int kReduceThreads = 512;
constexpr int kReducePer = 8;                        // records in flight per thread
constexpr int kPlaceThreads = 512;
constexpr int kPlacePer = 8;                         // records per thread and chunk
constexpr int kPlaceChunk = kPlaceThreads * kPlacePer;

__global__ __launch_bounds__(kCountThreads) void bin_count_kernel(RecordBuffers rb, int nbins) {
  extern __shared__ uint32_t h[];
  for (int i = threadIdx.x; i < nbins; i += kCountThreads) h[i] = 0u;
  __syncthreads();
  const int r = blockIdx.x;
  for (int q = 0; q < rb.nsub; ++q) {
    const size_t sub = (size_t)r * rb.nsub + q;
    const uint32_t n = rb.count[sub];
    const uint32_t* key = rb.key + sub * rb.cap;
    for (uint32_t base = 0; base < n; base += kCountThreads * 8) {
      uint32_t k[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint32_t i = base + j * kCountThreads + threadIdx.x;
        k[j] = i < n ? key[i] : 0xFFFFFFFFu;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (k[j] != 0xFFFFFFFFu) atomicAdd(&h[k[j] >> kBinShift], 1u);
    }
  }
  __syncthreads();
  uint32_t* out = rb.hist + (size_t)r * nbins;
  for (int i = threadIdx.x; i < nbins; i += kCountThreads) out[i] = h[i];
}

// off[r][b] = sum over regions r' < r of hist[r'][b]; total[b] = sum over
// all.  A block takes 16 bins; each bin's regions are split over 16 threads
// (partial sums, a 16-way exclusive scan, then the running prefix).
__global__ __launch_bounds__(256) void bin_colscan_kernel(RecordBuffers rb, int nbins, int nregions) {
  __shared__ uint32_t part[16][17];
  const int bl = threadIdx.x & 15, q = threadIdx.x >> 4;
  const int b = blockIdx.x * 16 + bl;
  const int per = (nregions + 15) / 16;
  const int r0 = min(nregions, q * per), r1 = min(nregions, r0 + per);
  uint32_t sum = 0;
  if (b < nbins) {
#pragma unroll 8
    for (int r = r0; r < r1; ++r) sum += rb.hist[(size_t)r * nbins + b];
  }
  part[q][bl] = sum;
  __syncthreads();
  if (b >= nbins) return;
  uint32_t run = 0, total = 0;
  for (int k = 0; k < 16; ++k) {
    const uint32_t x = part[k][bl];
    run += k < q ? x : 0u;
    total += x;
  }
  if (q == 0) rb.bin_total[b] = total;
#pragma unroll 8
  for (int r = r0; r < r1; ++r) {
    const uint32_t h = rb.hist[(size_t)r * nbins + b];
    rb.off[(size_t)r * nbins + b] = run;
    run += h;
  }
}

// bin_start = exclusive prefix of the totals, chunk_start = exclusive prefix
// of ceil(total / kChunk); both with the grand total at [nbins].
__global__ __launch_bounds__(1024) void bin_start_kernel(RecordBuffers rb, int nbins) {
  __shared__ uint32_t s_rec[1024], s_chk[1024];
  const int t = threadIdx.x;
  const int per = (nbins + 1023) / 1024;
  const int b0 = min(nbins, t * per), b1 = min(nbins, b0 + per);
  uint32_t rec = 0, chk = 0;
  for (int b = b0; b < b1; ++b) {
    const uint32_t n = rb.bin_total[b];
    rec += n;
    chk += (n + kChunk - 1) / kChunk;
  }
  s_rec[t] = rec;
  s_chk[t] = chk;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t a = t >= o ? s_rec[t - o] : 0u, c = t >= o ? s_chk[t - o] : 0u;
    __syncthreads();
    s_rec[t] += a;
    s_chk[t] += c;
    __syncthreads();
  }
  uint32_t run_r = s_rec[t] - rec, run_c = s_chk[t] - chk;
  for (int b = b0; b < b1; ++b) {
    const uint32_t n = rb.bin_total[b];
    rb.bin_start[b] = run_r;
    rb.chunk_start[b] = run_c;
    run_r += n;
    run_c += (n + kChunk - 1) / kChunk;
  }
  if (t == 1023) {
    rb.bin_start[nbins] = s_rec[1023];
    rb.chunk_start[nbins] = s_chk[1023];
  }
}

// Records of one region to their bins' slices.  Chunks of kPlaceChunk
// records are first ordered by bin in LDS (counting sort with LDS integer
// atomics), so that the global stores of a wave cover runs of consecutive
// slots of a few bins instead of one cache line per lane.
__global__ __launch_bounds__(kPlaceThreads) void bin_place_kernel(RecordBuffers rb, int nbins) {
  extern __shared__ uint32_t bins_lds[];  // gcur, cnt, lst: [nbins] each
  uint32_t* gcur = bins_lds;
  uint32_t* cnt = bins_lds + nbins;
  uint32_t* lst = bins_lds + 2 * nbins;
  __shared__ uint32_t wsum[kPlaceThreads / kWave];
  __shared__ uint3 stage[kPlaceChunk];
  const int r = blockIdx.x, t = threadIdx.x;
  const uint32_t* off = rb.off + (size_t)r * nbins;
  for (int b = t; b < nbins; b += kPlaceThreads) gcur[b] = rb.bin_start[b] + off[b];
  const int per = (nbins + kPlaceThreads - 1) / kPlaceThreads;
  const int b0 = min(nbins, t * per), b1 = min(nbins, b0 + per);
  for (int q = 0; q < rb.nsub; ++q) {
  const size_t sub = (size_t)r * rb.nsub + q;
  const uint32_t n = rb.count[sub];
  const uint32_t* key = rb.key + sub * rb.cap;
  const float2* val = rb.val + sub * rb.cap;
  for (uint32_t base = 0; base < n; base += kPlaceChunk) {
    const uint32_t m = min((uint32_t)kPlaceChunk, n - base);
    for (int b = t; b < nbins; b += kPlaceThreads) cnt[b] = 0u;
    __syncthreads();
    uint32_t k[kPlacePer], rank[kPlacePer];
    float2 v[kPlacePer];
#pragma unroll
    for (int j = 0; j < kPlacePer; ++j) {
      const uint32_t i = j * kPlaceThreads + t;
      if (i < m) {
        k[j] = key[base + i];
        v[j] = val[base + i];
        rank[j] = atomicAdd(&cnt[k[j] >> kBinShift], 1u);
      }
    }
    __syncthreads();
    // lst = exclusive prefix of cnt: per-thread runs of bins, then a scan of
    // the thread totals
    uint32_t mine = 0;
    for (int b = b0; b < b1; ++b) mine += cnt[b];
    const uint32_t incl = wave_incl_scan_u32(mine);
    if (lane_id() == kWave - 1) wsum[t / kWave] = incl;
    __syncthreads();
    uint32_t run = incl - mine;
    for (int w = 0; w < t / kWave; ++w) run += wsum[w];
    for (int b = b0; b < b1; ++b) {
      lst[b] = run;
      run += cnt[b];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPlacePer; ++j) {
      const uint32_t i = j * kPlaceThreads + t;
      if (i < m) stage[lst[k[j] >> kBinShift] + rank[j]] = make_uint3(k[j], __float_as_uint(v[j].x),
                                                                        __float_as_uint(v[j].y));
    }
    __syncthreads();
    for (uint32_t i = t; i < m; i += kPlaceThreads) {
      const uint3 rec = stage[i];
      const uint32_t b = rec.x >> kBinShift;
      rb.sorted[gcur[b] + (i - lst[b])] = rec;
    }
    __syncthreads();
    for (int b = t; b < nbins; b += kPlaceThreads) gcur[b] += cnt[b];
  }
  }
}

__global__ __launch_bounds__(kReduceThreads) void bin_reduce_kernel(RecordBuffers rb, int nbins, uint32_t entries,
                                                                    float* __restrict__ grad_table) {
  // (g0, g1) of each entry as one 64-bit word: float pairs are added with
  // LDS 64-bit compare-and-swap, which retires far faster than LDS float
  // atomics on this architecture
  __shared__ unsigned long long acc[kBinEntries];
  const uint32_t c = blockIdx.x;
  if (c >= rb.chunk_start[nbins]) return;
  // bin b: chunk_start[b] <= c < chunk_start[b + 1]
  int lo = 0, hi = nbins;  // invariant: chunk_start[lo] <= c < chunk_start[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (rb.chunk_start[mid] <= c) lo = mid; else hi = mid;
  }
  const int b = lo;
  const uint32_t nch = rb.chunk_start[b + 1] - rb.chunk_start[b];
  const uint32_t first = rb.bin_start[b] + (c - rb.chunk_start[b]) * kChunk;
  const uint32_t last = min(rb.bin_start[b + 1], first + kChunk);
  for (int i = threadIdx.x; i < kBinEntries; i += kReduceThreads) acc[i] = 0ull;
  __syncthreads();
  const uint32_t e0 = (uint32_t)b << kBinShift;
  for (uint32_t base = first; base < last; base += kReduceThreads * kReducePer) {
    uint3 rec[kReducePer];
#pragma unroll
    for (int j = 0; j < kReducePer; ++j) {
      const uint32_t i = base + j * kReduceThreads + threadIdx.x;
      rec[j] = i < last ? rb.sorted[i] : make_uint3(0xFFFFFFFFu, 0u, 0u);
    }
#pragma unroll
    for (int j = 0; j < kReducePer; ++j) {
      if (rec[j].x == 0xFFFFFFFFu) continue;
      const uint32_t e = rec[j].x - e0;
      const float a = __uint_as_float(rec[j].y), c = __uint_as_float(rec[j].z);
      unsigned long long seen = acc[e];
      for (;;) {
        const unsigned long long got = atomicCAS(&acc[e], seen, add_pair_bits(seen, a, c));
        if (got == seen) break;
        seen = got;
      }
    }
  }
  __syncthreads();
  const uint32_t ne = min((uint32_t)kBinEntries, entries - e0);
  float2* g = reinterpret_cast<float2*>(grad_table) + e0;
  for (uint32_t e = threadIdx.x; e < ne; e += kReduceThreads) {
    const unsigned long long w = acc[e];
    const float a0 = __uint_as_float((uint32_t)w), a1 = __uint_as_float((uint32_t)(w >> 32));
    if (a0 == 0.0f && a1 == 0.0f) continue;
    if (nch == 1) {
      float2 v = g[e];
      v.x += a0;
      v.y += a1;
      g[e] = v;
    } else {
      atomicAdd(&g[e].x, a0);
      atomicAdd(&g[e].y, a1);
    }
  }
}

}  // namespace

BinPlan bin_plan(uint32_t entries, int levels, int nregions, int64_t max_samples) {
  BinPlan p;
  p.entries = entries;
  p.nbins = (int)((entries + kBinEntries - 1) / kBinEntries);
  p.nregions = nregions;
  p.nsub = levels / 4;
  const int64_t tiles = (max_samples + 15) / 16;
  const int64_t per_region = (tiles + nregions - 1) / nregions;
  p.cap = (uint32_t)(per_region * 64 * 8);  // 64 lanes x 8 corners per tile and level group
  const int64_t records = (int64_t)p.cap * p.nsub * nregions;
  p.max_chunks = (int)(p.nbins + (records + kChunk - 1) / kChunk);
  return p;
}

hipError_t bin_scatter(const BinPlan& p, const RecordBuffers& rb, float* grad_table, hipStream_t st) {
  if (p.nbins == 0) return hipSuccess;
  const size_t hist_lds = (size_t)p.nbins * sizeof(uint32_t);
  hipLaunchKernelGGL(bin_count_kernel, dim3(p.nregions), dim3(kCountThreads), hist_lds, st, rb, p.nbins);
  hipLaunchKernelGGL(bin_colscan_kernel, dim3((p.nbins + 15) / 16), dim3(256), 0, st, rb, p.nbins, p.nregions);
  hipLaunchKernelGGL(bin_start_kernel, dim3(1), dim3(1024), 0, st, rb, p.nbins);
  hipLaunchKernelGGL(bin_place_kernel, dim3(p.nregions), dim3(kPlaceThreads), 3 * hist_lds, st, rb, p.nbins);
  hipLaunchKernelGGL(bin_reduce_kernel, dim3(p.max_chunks), dim3(kReduceThreads), 0, st, rb, p.nbins, p.entries,
                     grad_table);
  return hipGetLastError();
}

}  // namespace nsl
