// Table-gradient accumulation without global atomics on the hot path.
//
// The gradient of a table entry is the sum, over every sample and every
// corner of its cell that lands on the entry, of the corner's trilinear
// weight times dL/de of that level (the chain rule through the encoding of
// Sec. 3.3).  Device-coherent atomics on gfx950 retire at roughly one lane
// per clock per XCD whatever the address pattern, and LDS float atomics at a
// third of a lane per clock per CU, so the sum is formed by a counting sort
// into bins of 2^13 consecutive entries and an LDS reduction per bin:
//
//   (backward)  dL/de of every sample, level-major [level][sample]
//   count       per block of samples: records per bin (LDS integer atomics)
//   scan        per bin, exclusive prefix over blocks; bin totals
//   start       exclusive prefix over bins; chunks of kChunk records per bin
//   place       the block's records again, ordered by bin in LDS, stored to
//               their bins' slices
//   reduce      one workgroup per chunk: LDS accumulation of the bin with
//               64-bit compare-and-swap on (g0, g1) pairs, then grad += acc,
//               or grad = acc when the step clears its gradients (a bin of
//               one chunk owns its entries; chunks of a bin with several add
//               with atomics, one per touched entry)
//
// A record is (entry, w * dL/de_l0, w * dL/de_l1), the values in FP32, or in
// BF16 for the mixed-precision step (accumulated in FP32 all the same).
// Count and place generate
// the same records from the sample positions and dL/de: the 16 lanes of a
// row hold 16 consecutive samples (mostly along one ray) at one level;
// neighbouring lanes in the same cell form a run, and each run gives eight
// records (one per corner) carrying the run's sums.
#include "field_common.h"

namespace nsl {

namespace {

constexpr int kRecThreads = 512;                     // count and place
constexpr int kRecWaves = kRecThreads / kWave;
constexpr int kRecTilesPerWave = 1;
constexpr int kRecSamples = kRecWaves * kRecTilesPerWave * 16;      // samples per block
constexpr int kPlaceChunk = kRecWaves * kRecTilesPerWave * 64 * 8;  // records of one level group
constexpr int kMaxPer = (kMaxBins + kRecThreads - 1) / kRecThreads;  // bins per thread in the placement scan
constexpr int kReduceThreads = 1024;

// Record formats: FP32 values (entry, g0, g1), or, for mixed precision,
// BF16 values (entry, g0 | g1 << 16).  In the sorted array a record keeps
// only the entry's 16-bit offset in its bin (10 or 6 bytes a record).  Either
// way the reduction accumulates in FP32.
struct RecF32 {
  typedef uint3 T;
  static __device__ __forceinline__ T pack(uint32_t e, float a, float b) {
    return make_uint3(e, __float_as_uint(a), __float_as_uint(b));
  }
  // In the sorted array a record takes 10 bytes: the entry's 16-bit offset
  // in its bin (the bin is implied by the slot) and the two FP32 values.
  static __device__ __forceinline__ void store(const RecordBuffers& rb, uint32_t pos, const T& r) {
    static_assert(kBinShift <= 16, "in-bin offsets are 16-bit");
    static_cast<uint16_t*>(rb.sorted)[pos] = (uint16_t)(r.x & (uint32_t)(kBinEntries - 1));
    reinterpret_cast<uint2*>(rb.sorted_vals)[pos] = make_uint2(r.y, r.z);
  }
  // the values of the four slots 4 gi .. 4 gi + 3
  static __device__ __forceinline__ void vals4(const RecordBuffers& rb, uint32_t gi, float2 (&v)[4]) {
    const uint4* p = reinterpret_cast<const uint4*>(rb.sorted_vals) + 2 * (size_t)gi;
    const uint4 a = p[0], b = p[1];
    v[0] = make_float2(__uint_as_float(a.x), __uint_as_float(a.y));
    v[1] = make_float2(__uint_as_float(a.z), __uint_as_float(a.w));
    v[2] = make_float2(__uint_as_float(b.x), __uint_as_float(b.y));
    v[3] = make_float2(__uint_as_float(b.z), __uint_as_float(b.w));
  }
  static __device__ __forceinline__ uint32_t key(const T& r) { return r.x; }
  static __device__ __forceinline__ float2 val(const T& r) {
    return make_float2(__uint_as_float(r.y), __uint_as_float(r.z));
  }
  static __device__ __forceinline__ T none() { return make_uint3(0xFFFFFFFFu, 0u, 0u); }
};
struct RecBF16 {
  typedef uint2 T;
  static __device__ __forceinline__ T pack(uint32_t e, float a, float b) {
    const __bf16 x = (__bf16)a, y = (__bf16)b;
    return make_uint2(e, (uint32_t)__builtin_bit_cast(uint16_t, x) | ((uint32_t)__builtin_bit_cast(uint16_t, y) << 16));
  }
  // In the sorted array a record takes 6 bytes: the entry's offset in its
  // bin (the bin is implied by the slot) and the two BF16 values.
  static __device__ __forceinline__ void store(const RecordBuffers& rb, uint32_t pos, const T& r) {
    static_assert(kBinShift <= 16, "in-bin offsets are 16-bit");
    static_cast<uint16_t*>(rb.sorted)[pos] = (uint16_t)(r.x & (uint32_t)(kBinEntries - 1));
    rb.sorted_vals[pos] = r.y;
  }
  static __device__ __forceinline__ uint32_t key(const T& r) { return r.x; }
  static __device__ __forceinline__ float2 val(const T& r) {
    return make_float2((float)__builtin_bit_cast(__bf16, (uint16_t)(r.y & 0xFFFFu)),
                       (float)__builtin_bit_cast(__bf16, (uint16_t)(r.y >> 16)));
  }
  static __device__ __forceinline__ T none() { return make_uint2(0xFFFFFFFFu, 0u); }
  // the values of the four slots 4 gi .. 4 gi + 3
  static __device__ __forceinline__ void vals4(const RecordBuffers& rb, uint32_t gi, float2 (&v)[4]) {
    const uint4 w = reinterpret_cast<const uint4*>(rb.sorted_vals)[gi];
    v[0] = val(make_uint2(0u, w.x));
    v[1] = val(make_uint2(0u, w.y));
    v[2] = val(make_uint2(0u, w.z));
    v[3] = val(make_uint2(0u, w.w));
  }
};

// The records of one level (l = g + 4q for lane group g) of one tile: the
// eight corners of this lane's cell with their run sums; on = this lane
// starts a run of samples in one cell (and is valid).
struct LevelRecords {
  uint32_t idx[8];
  float v0[8], v1[8];
  bool on;
};

// dL/de of this lane's levels g + 4q (zero for samples beyond the batch).
__device__ __forceinline__ void load_de(const float2* __restrict__ de, int stride, int levels, int g, int s,
                                       bool valid, float2 d[kMaxLevels / 4]) {
#pragma unroll
  for (int q = 0; q < kMaxLevels / 4; ++q)
    d[q] = valid && 4 * q < levels ? de[(size_t)(g + 4 * q) * stride + s] : make_float2(0.0f, 0.0f);
}

__device__ __forceinline__ void level_records(const LevelInfo& lv, float2 d, int l, bool valid, const float xn[3],
                                              LevelRecords& r) {
  Corner8 c;
  corners(xn[0], xn[1], xn[2], lv.res[l], (lv.dense_bits >> l) & 1u, lv.table_mask, lv.offset[l], c);
  float v[16];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[2 * k] = c.w[k] * d.x;
    v[2 * k + 1] = c.w[k] * d.y;
  }
  r.on = row_cell_runs<16>(c.cell, valid, v) && valid;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    r.idx[k] = c.idx[k];
    r.v0[k] = v[2 * k];
    r.v1[k] = v[2 * k + 1];
  }
}

__device__ __forceinline__ int sample_count(const SampleSrc& src) { return src.n_dev ? (int)*src.n_dev : src.n; }

// Workgroups are dispatched round-robin over the 8 XCDs.  Block i runs the
// sample range of logical block (i % 8) * (nblk / 8) + i / 8, so that each
// XCD walks a contiguous stretch of logical blocks in order; the slices the
// placement writes into a bin are ordered by logical block, hence the runs
// that consecutive workgroups of one XCD store are adjacent in memory and
// meet in that XCD's L2.  nblk is a multiple of 8.
__device__ __forceinline__ int logical_block(int nblk) {
  return (int)(blockIdx.x % 8u) * (nblk / 8) + (int)(blockIdx.x / 8u);
}

__global__ __launch_bounds__(kRecThreads) void bin_count_kernel(SampleSrc src, LevelInfo lv, RecordBuffers rb,
                                                               int nbins) {
  extern __shared__ uint32_t h[];
  for (int i = threadIdx.x; i < nbins; i += kRecThreads) h[i] = 0u;
  __syncthreads();
  const int S = sample_count(src);
  const int blk = logical_block(gridDim.x);
  const int wave = threadIdx.x / kWave, lane = lane_id(), g = lane >> 4, jc = lane & 15;
  for (int j = 0; j < kRecTilesPerWave; ++j) {
    const int tile = (blk * kRecWaves + wave) * kRecTilesPerWave + j;
    if (tile * 16 >= S) break;
    const int s = tile * 16 + jc;
    const bool valid = s < S;
    float xn[3] = {0.5f, 0.5f, 0.5f};
    if (valid) load_position(src, s, xn);
    float2 dl[kMaxLevels / 4];
    load_de(rb.de, rb.stride, lv.levels, g, s, valid, dl);
    for (int q = 0; q < lv.levels / 4; ++q) {
      LevelRecords r;
      level_records(lv, dl[q], g + 4 * q, valid, xn, r);
      if (r.on) {
        // the two x-neighbour corners (k, k + 1) nearly always share a bin:
        // one atomic counts both
#pragma unroll
        for (int k = 0; k < 8; k += 2) {
          const uint32_t ba = r.idx[k] >> kBinShift, bb = r.idx[k + 1] >> kBinShift;
          if (ba == bb) {
            atomicAdd(&h[ba], 2u);
          } else {
            atomicAdd(&h[ba], 1u);
            atomicAdd(&h[bb], 1u);
          }
        }
      }
    }
  }
  __syncthreads();
  uint32_t* out = rb.hist + (size_t)blk * nbins;
  for (int i = threadIdx.x; i < nbins; i += kRecThreads) out[i] = h[i];
}

// off[b'][b] = sum over blocks b'' < b' of hist[b''][b]; total[b] = sum over
// all.  A workgroup takes 4 bins and splits the blocks into segments of
// 256 x kColRows: thread group q (4 threads, one per bin) owns kColRows
// consecutive blocks of a segment, loads their counts at once and keeps them
// in registers; the 256 group sums of a bin are scanned by one wave (4 per
// lane, then a DPP scan), and each thread writes the running prefix over its
// blocks.  A 128-byte row segment holds 32 bins, read by 8 workgroups: those
// are placed on one XCD (workgroups go round-robin over the 8 XCDs), so the
// segment is fetched into one L2 only.
constexpr int kColBins = 4;
constexpr int kColGroups = 256;
constexpr int kColRows = 8;
__device__ __forceinline__ int colscan_first_bin() {
  const int x = (int)(blockIdx.x % 8u), j = (int)(blockIdx.x / 8u);
  return ((j / 8) * 8 + x) * 32 + (j % 8) * kColBins;
}
int colscan_grid(int nbins) { return 64 * ((nbins + 255) / 256); }

__global__ __launch_bounds__(kColBins * kColGroups) void bin_colscan_kernel(RecordBuffers rb, int nbins, int nblk) {
  __shared__ uint32_t part[kColGroups][kColBins];
  __shared__ uint32_t tot[kColBins];
  const int bl = threadIdx.x & (kColBins - 1), q = threadIdx.x / kColBins;
  const int b = colscan_first_bin() + bl;
  const bool on = b < nbins;
  const int wave = threadIdx.x / kWave, lane = lane_id();
  uint32_t carry = 0;
  for (int seg = 0; seg < nblk; seg += kColGroups * kColRows) {
    const int r0 = seg + q * kColRows;
    uint32_t v[kColRows], sum = 0;
#pragma unroll
    for (int k = 0; k < kColRows; ++k) v[k] = on && r0 + k < nblk ? rb.hist[(size_t)(r0 + k) * nbins + b] : 0u;
#pragma unroll
    for (int k = 0; k < kColRows; ++k) sum += v[k];
    part[q][bl] = sum;
    __syncthreads();
    if (wave < kColBins) {
      // wave w scans bin w: lane l holds groups 4l .. 4l + 3
      uint32_t g[4], x = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        g[k] = part[4 * lane + k][wave];
        x += g[k];
      }
      const uint32_t incl = wave_incl_scan_u32(x);
      uint32_t run = incl - x;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        part[4 * lane + k][wave] = run;
        run += g[k];
      }
      if (lane == kWave - 1) tot[wave] = incl;
    }
    __syncthreads();
    uint32_t run = carry + part[q][bl];
    if (on) {
#pragma unroll
      for (int k = 0; k < kColRows; ++k) {
        if (r0 + k < nblk) rb.off[(size_t)(r0 + k) * nbins + b] = run;
        run += v[k];
      }
    }
    carry += tot[bl];
    __syncthreads();
  }
  if (on && q == 0) rb.bin_total[b] = carry;
}

// bin_start = exclusive prefix of the totals, chunk_start = exclusive prefix
// of ceil(total / kChunk); both with the grand total at [nbins].
__global__ __launch_bounds__(1024) void bin_start_kernel(RecordBuffers rb, int nbins) {
  __shared__ uint32_t w_rec[1024 / kWave], w_chk[1024 / kWave];
  const int t = threadIdx.x;
  const int per = (nbins + 1023) / 1024;
  const int b0 = min(nbins, t * per), b1 = min(nbins, b0 + per);
  uint32_t rec = 0, chk = 0;
  for (int b = b0; b < b1; ++b) {
    const uint32_t n = rb.bin_total[b];
    rec += n;
    chk += (n + kChunk - 1) / kChunk;
  }
  // wave scans, then the totals of the waves before
  const int wave = t / kWave;
  const uint32_t ir = wave_incl_scan_u32(rec), ic = wave_incl_scan_u32(chk);
  if (lane_id() == kWave - 1) {
    w_rec[wave] = ir;
    w_chk[wave] = ic;
  }
  __syncthreads();
  uint32_t run_r = ir - rec, run_c = ic - chk, all_r = 0, all_c = 0;
  for (int w = 0; w < 1024 / kWave; ++w) {
    run_r += w < wave ? w_rec[w] : 0u;
    run_c += w < wave ? w_chk[w] : 0u;
    all_r += w_rec[w];
    all_c += w_chk[w];
  }
  for (int b = b0; b < b1; ++b) {
    const uint32_t n = rb.bin_total[b];
    rb.bin_start[b] = run_r;
    rb.chunk_start[b] = run_c;
    const uint32_t nc = (n + kChunk - 1) / kChunk;
    for (uint32_t k = 0; k < nc; ++k) rb.chunk_bin[run_c + k] = (uint32_t)b;
    run_r += n;
    run_c += nc;
  }
  if (t == 1023) {
    rb.bin_start[nbins] = all_r;
    rb.chunk_start[nbins] = all_c;
  }
}

// The block's records, one level group at a time: generated as in the
// count, ordered by bin in LDS (counting sort with LDS integer atomics), and
// stored so that the global stores of a wave cover runs of consecutive slots
// of a few bins instead of one cache line per lane.
//
// zero_table (overwriting reductions only, else null): the gradient entries of
// the bins that the reduction will not overwrite (bins with no records, or
// with several chunks, which add with atomics) are cleared here first.
template <class R, int G, int PER>
__global__ __launch_bounds__(kRecThreads) void bin_place_kernel(SampleSrc src, LevelInfo lv, RecordBuffers rb,
                                                               int nbins, float* __restrict__ zero_table,
                                                               uint32_t entries) {
  static_assert(kRecTilesPerWave == 1, "one tile per wave");
  typedef typename R::T Rec;
  // base: slot of the round's record i of bin b is base[b] + i; cnt: the
  // round's count per bin; lst: its exclusive prefix.  Thread t owns bins
  // [b0, b1) (at most PER) and keeps their global cursors in registers.
  extern __shared__ uint32_t bins_lds[];
  uint32_t* base = bins_lds;
  uint32_t* cnt = bins_lds + nbins;
  uint32_t* lst = bins_lds + 2 * nbins;
  __shared__ uint32_t wsum[kRecWaves];
  __shared__ Rec stage[kPlaceChunk * G];
  const int t = threadIdx.x;
  const int blk = logical_block(gridDim.x);
  const uint32_t* off = rb.off + (size_t)blk * nbins;
  for (int b = t; b < nbins; b += kRecThreads) cnt[b] = 0u;
  const int per = (nbins + kRecThreads - 1) / kRecThreads;  // at most PER
  const int b0 = min(nbins, t * per), b1 = min(nbins, b0 + per);
  uint32_t cur[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) cur[k] = b0 + k < b1 ? rb.bin_start[b0 + k] + off[b0 + k] : 0u;
  if (zero_table) {
    // two entries (one float4) per thread and step; the table is 16-byte
    // aligned, an odd last entry is cleared on its own
    const uint32_t units = (entries + 1) / 2;
    for (uint32_t u = blockIdx.x * kRecThreads + t; u < units; u += gridDim.x * kRecThreads) {
      const uint32_t e = 2 * u, bin = e >> kBinShift;
      if (rb.chunk_start[bin + 1] - rb.chunk_start[bin] == 1u) continue;
      if (e + 1 < entries)
        reinterpret_cast<float4*>(zero_table)[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      else
        reinterpret_cast<float2*>(zero_table)[e] = make_float2(0.0f, 0.0f);
    }
  }
  const int S = sample_count(src);
  const int wave = t / kWave, lane = lane_id(), g = lane >> 4, jc = lane & 15;
  const int s = (blk * kRecWaves + wave) * 16 + jc;
  const bool valid = s < S;
  float xn[3] = {0.5f, 0.5f, 0.5f};
  if (valid) load_position(src, s, xn);
  float2 dl[kMaxLevels / 4];
  load_de(rb.de, rb.stride, lv.levels, g, s, valid, dl);
  __syncthreads();
  const int groups = lv.levels / 4;
  for (int q0 = 0; q0 < groups; q0 += G) {
    // G level groups per round: the records in their stored format, off
    // lanes (and groups beyond the last) holding R::none()
    Rec rec[G][8];
    uint32_t rank[G][8];
#pragma unroll
    for (int h = 0; h < G; ++h) {
      const int q = q0 + h;
      if (q < groups) {
        LevelRecords r;
        level_records(lv, dl[q], g + 4 * q, valid, xn, r);
#pragma unroll
        for (int k = 0; k < 8; ++k) rec[h][k] = r.on ? R::pack(r.idx[k], r.v0[k], r.v1[k]) : R::none();
      } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) rec[h][k] = R::none();
      }
      // ranks in the bins; the two x-neighbour corners (k, k + 1) nearly
      // always share a bin and then take two consecutive ranks from one
      // atomic (a lane's records are all present or all absent)
#pragma unroll
      for (int k = 0; k < 8; k += 2) {
        if (R::key(rec[h][k]) != 0xFFFFFFFFu) {
          const uint32_t ba = R::key(rec[h][k]) >> kBinShift, bb = R::key(rec[h][k + 1]) >> kBinShift;
          if (ba == bb) {
            rank[h][k] = atomicAdd(&cnt[ba], 2u);
            rank[h][k + 1] = rank[h][k] + 1u;
          } else {
            rank[h][k] = atomicAdd(&cnt[ba], 1u);
            rank[h][k + 1] = atomicAdd(&cnt[bb], 1u);
          }
        }
      }
    }
    __syncthreads();
    // lst = exclusive prefix of cnt (per-thread runs of bins, a wave scan of
    // the thread totals, then the totals of the waves before); the owners
    // of the bins also set base, advance their cursors and clear the counts
    // for the next round
    uint32_t c[PER], mine = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      c[k] = b0 + k < b1 ? cnt[b0 + k] : 0u;
      mine += c[k];
    }
    const uint32_t incl = wave_incl_scan_u32(mine);
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    uint32_t run = incl - mine, m = 0;
    for (int w = 0; w < kRecWaves; ++w) {
      run += w < wave ? wsum[w] : 0u;
      m += wsum[w];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      if (b0 + k < b1) {
        lst[b0 + k] = run;
        base[b0 + k] = cur[k] - run;
        cnt[b0 + k] = 0u;
        cur[k] += c[k];
      }
      run += c[k];
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < G; ++h)
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (R::key(rec[h][k]) != 0xFFFFFFFFu) stage[lst[R::key(rec[h][k]) >> kBinShift] + rank[h][k]] = rec[h][k];
    __syncthreads();
    for (uint32_t i = t; i < m; i += kRecThreads) {
      const Rec r = stage[i];
      R::store(rb, base[R::key(r) >> kBinShift] + i, r);
    }
    __syncthreads();
  }
}

// overwrite: a bin of one chunk stores its sums over every entry (zeros
// included) instead of adding them to the gradient.
template <class R>
__global__ __launch_bounds__(kReduceThreads) void bin_reduce_kernel(RecordBuffers rb, int nbins, uint32_t entries,
                                                                    float* __restrict__ grad_table,
                                                                    float* __restrict__ overflow, bool overwrite) {
  // (g0, g1) of each entry as one 64-bit word: float pairs are added with
  // LDS 64-bit compare-and-swap, which retires far faster than LDS float
  // atomics on this architecture
  __shared__ unsigned long long acc[kBinEntries];
  const uint32_t c = blockIdx.x;
  if (c >= rb.chunk_start[nbins]) return;
  const int b = (int)rb.chunk_bin[c];
  const uint32_t nch = rb.chunk_start[b + 1] - rb.chunk_start[b];
  const uint32_t first = rb.bin_start[b] + (c - rb.chunk_start[b]) * kChunk;
  const uint32_t last = min(rb.bin_start[b + 1], first + kChunk);
  for (int i = threadIdx.x; i < kBinEntries; i += kReduceThreads) acc[i] = 0ull;
  __syncthreads();
  const uint32_t e0 = (uint32_t)b << kBinShift;
  // adds (a, cc) to entry e of the bin
  auto add = [&](uint32_t e, float a, float cc) {
    unsigned long long seen = acc[e];
    for (;;) {
      const unsigned long long got = atomicCAS(&acc[e], seen, add_pair_bits(seen, a, cc));
      if (got == seen) break;
      seen = got;
    }
  };
  // A lane reads four consecutive records at a time: their in-bin offsets
  // with one 8-byte load and their values with one (BF16) or two (FP32)
  // 16-byte loads.  Groups of four slots are aligned; slots outside
  // [first, last) are skipped.
  const uint32_t g0 = first / 4, g1 = (last + 3) / 4;
  const uint2* __restrict__ keys = static_cast<const uint2*>(rb.sorted);
  for (uint32_t gb = g0; gb < g1; gb += kReduceThreads * 2) {
    uint2 kk[2];
    float2 vv[2][4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint32_t gi = gb + j * kReduceThreads + threadIdx.x;
      const uint32_t gc = gi < g1 ? gi : g0;  // a group of this chunk either way
      kk[j] = keys[gc];
      R::vals4(rb, gc, vv[j]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint32_t p0 = 4 * (gb + j * kReduceThreads + threadIdx.x);
      const uint32_t k4[4] = {kk[j].x & 0xFFFFu, kk[j].x >> 16, kk[j].y & 0xFFFFu, kk[j].y >> 16};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (p0 + u < first || p0 + u >= last) continue;
        add(k4[u], vv[j][u].x, vv[j][u].y);
      }
    }
  }
  __syncthreads();
  // every gradient value written is checked for the loss-scale overflow flag
  // (for the atomic adds, the value each add leaves)
  const uint32_t ne = min((uint32_t)kBinEntries, entries - e0);
  float2* gt = reinterpret_cast<float2*>(grad_table) + e0;
  bool bad = false;
  for (uint32_t e = threadIdx.x; e < ne; e += kReduceThreads) {
    const unsigned long long w = acc[e];
    const float a0 = __uint_as_float((uint32_t)w), a1 = __uint_as_float((uint32_t)(w >> 32));
    if (nch == 1 && overwrite) {
      gt[e] = make_float2(a0, a1);
      bad |= !isfinite(a0) || !isfinite(a1);
      continue;
    }
    if (a0 == 0.0f && a1 == 0.0f) continue;
    if (nch == 1) {
      float2 v = gt[e];
      v.x += a0;
      v.y += a1;
      gt[e] = v;
      bad |= !isfinite(v.x) || !isfinite(v.y);
    } else {
      const float o0 = atomicAdd(&gt[e].x, a0);
      const float o1 = atomicAdd(&gt[e].y, a1);
      bad |= !isfinite(o0 + a0) || !isfinite(o1 + a1);
    }
  }
  if (overflow && bad) *overflow = 1.0f;
}

}  // namespace

BinPlan bin_plan(uint32_t entries, int levels, int64_t max_samples) {
  BinPlan p;
  p.entries = entries;
  p.nbins = (int)((entries + kBinEntries - 1) / kBinEntries);
  p.levels = levels;
  p.stride = (int)max_samples;
  p.nblk = (int)((max_samples + kRecSamples - 1) / kRecSamples + 7) / 8 * 8;  // whole rounds over the XCDs
  p.max_records = max_samples * 8 * levels;
  p.max_chunks = (int)(p.nbins + (p.max_records + kChunk - 1) / kChunk);
  return p;
}

hipError_t bin_scatter(const BinPlan& p, const RecordBuffers& rb, const SampleSrc& src, const LevelInfo& lv,
                       bool bf16_values, bool overwrite, float* grad_table, float* overflow, hipStream_t st,
                       bool counted) {
  if (p.nbins == 0 || p.nblk == 0) return hipSuccess;
  float* zero_table = overwrite ? grad_table : nullptr;
  const size_t bins_lds = (size_t)p.nbins * sizeof(uint32_t);
  if (!counted)
    hipLaunchKernelGGL(bin_count_kernel, dim3(p.nblk), dim3(kRecThreads), bins_lds, st, src, lv, rb, p.nbins);
  hipLaunchKernelGGL(bin_colscan_kernel, dim3(colscan_grid(p.nbins)), dim3(kColBins * kColGroups), 0, st, rb,
                     p.nbins, p.nblk);
  hipLaunchKernelGGL(bin_start_kernel, dim3(1), dim3(1024), 0, st, rb, p.nbins);
  if (bf16_values) {
    if (p.nbins <= 2 * kRecThreads)
      hipLaunchKernelGGL((bin_place_kernel<RecBF16, 1, 2>), dim3(p.nblk), dim3(kRecThreads), 3 * bins_lds, st, src, lv,
                         rb, p.nbins, zero_table, p.entries);
    else
      hipLaunchKernelGGL((bin_place_kernel<RecBF16, 1, kMaxPer>), dim3(p.nblk), dim3(kRecThreads), 3 * bins_lds, st, src,
                         lv, rb, p.nbins, zero_table, p.entries);
    hipLaunchKernelGGL(bin_reduce_kernel<RecBF16>, dim3(p.max_chunks), dim3(kReduceThreads), 0, st, rb, p.nbins,
                       p.entries, grad_table, overflow, overwrite);
  } else {
    if (p.nbins <= 2 * kRecThreads)
      hipLaunchKernelGGL((bin_place_kernel<RecF32, 1, 2>), dim3(p.nblk), dim3(kRecThreads), 3 * bins_lds, st, src, lv,
                         rb, p.nbins, zero_table, p.entries);
    else
      hipLaunchKernelGGL((bin_place_kernel<RecF32, 1, kMaxPer>), dim3(p.nblk), dim3(kRecThreads), 3 * bins_lds, st, src,
                         lv, rb, p.nbins, zero_table, p.entries);
    hipLaunchKernelGGL(bin_reduce_kernel<RecF32>, dim3(p.max_chunks), dim3(kReduceThreads), 0, st, rb, p.nbins,
                       p.entries, grad_table, overflow, overwrite);
  }
  return hipGetLastError();
}

}  // namespace nsl
