// Table-gradient accumulation without global atomics on the hot path.
//
// The gradient of a table entry is the sum, over every sample and every
// corner of its cell that lands on the entry, of the corner's trilinear
// weight times dL/de of that level (the chain rule through the encoding of
// Sec. 3.3).  Device-coherent atomics on gfx950 retire at roughly one lane
// per clock per XCD whatever the address pattern, and LDS float atomics at a
// third of a lane per clock per CU, so the sum is formed by a counting sort
// into bins of 2^13 consecutive entries of a level and an LDS reduction per
// bin:
//
//   (backward)  dL/de of every sample, level-major [level][sample]
//   count       per unit (256 consecutive samples of one level): records per
//               bin of the level (LDS integer atomics); or done by the
//               encoding kernel, which evaluates the same corners
//   scan        per bin, exclusive prefix over the level's units; bin totals
//               (bins.h; in the training step, beside the forward MLP)
//   start       exclusive prefix over bins; chunks of at most a chunk of
//               corner additions per bin (fewer when the table has few bins,
//               so that the records still spread over many workgroups; half
//               as many for bins that need several) (bins.h; in the step,
//               beside the compositing)
//   place       per unit, the records again, ordered by bin in LDS and stored
//               to their bins' slices
//   reduce      one workgroup per chunk: LDS accumulation of the bin with
//               64-bit compare-and-swap on (g0, g1) pairs, then grad += acc,
//               or grad = acc when the step clears its gradients (a bin of
//               one chunk owns its entries; chunks of a bin with several add
//               with atomics, one per touched entry)
//
// A record is (entry, w * dL/de_l0, w * dL/de_l1), the values in FP32, or in
// BF16 for the mixed-precision step (accumulated in FP32 all the same), whose
// records also carry the x-neighbour corner when its entry differs from the
// first in a run of low bits (pair_code).  Count and place generate the same
// records from the sample positions and dL/de: the 16 lanes of a row hold 16
// consecutive samples (mostly along one ray); neighbouring lanes in the same
// cell form a run, and each run gives eight corner values carrying the run's
// sums.  Both run over the units of a level on one XCD (see level_unit), so
// the slices that consecutive units place into a bin are adjacent and merge
// in that XCD's L2.
#include <algorithm>

#include "bins.h"
#include "field_common.h"

namespace nsl {

namespace {

constexpr int kUnitWaves = kUnitSamples / kWave;  // count and place: one sample per thread
constexpr int kReduceThreads = 1024;

// Record formats: FP32 values (key, g0, g1), one corner a record; or, for
// mixed precision, BF16 values (key, g0 | g1 << 16, g0' | g1' << 16) of a
// corner and, when pair_code joins them, of its x-neighbour too.  key = the
// bin's index in its level << 16 | p << 13 | the entry's offset in the bin,
// p being the pair code (0: one corner; else the partner's offset is the
// offset ^ (2^p - 1)).  In the sorted array a record keeps only the low 16
// bits of the key and its values (10 bytes a record either way: FP32
// (g0, g1), or the two BF16 pairs).  Either way the reduction accumulates in FP32.
static_assert(kBinShift <= 13, "in-bin offsets take 13 bits, the pair code 3");
static_assert((kReduceThreads & (kReduceThreads - 1)) == 0, "the scattered group order needs a power of two");
struct RecF32 {
  typedef uint3 T;
  static constexpr bool kPaired = false;
  // the placement takes a level's units one after another on an XCD (its
  // 10-byte records fill more partly written lines when two levels' bins
  // are written at once: 88 against 84 us interleaved)
  static constexpr bool kInterleaveLevels = false;
  static __device__ __forceinline__ T pack(uint32_t key, float a, float b) {
    return make_uint3(key, __float_as_uint(a), __float_as_uint(b));
  }
  static __device__ __forceinline__ T pack_pair(uint32_t key, float a, float b, float, float) { return pack(key, a, b); }
  // In the sorted array a record takes 10 bytes: the entry's 16-bit offset
  // in its bin (the bin is implied by the slot) and the two FP32 values.
  static __device__ __forceinline__ void store(const RecordBuffers& rb, uint32_t pos, const T& r) {
    static_cast<uint16_t*>(rb.sorted)[pos] = (uint16_t)(r.x & 0xFFFFu);
    reinterpret_cast<uint2*>(rb.sorted_vals)[pos] = make_uint2(r.y, r.z);
  }
  // the values of the four slots 4 gi .. 4 gi + 3 (x, y: the record's entry)
  static __device__ __forceinline__ void vals4(const RecordBuffers& rb, uint32_t gi, float4 (&v)[4]) {
    const uint4* p = reinterpret_cast<const uint4*>(rb.sorted_vals) + 2 * (size_t)gi;
    const uint4 a = p[0], b = p[1];
    v[0] = make_float4(__uint_as_float(a.x), __uint_as_float(a.y), 0.0f, 0.0f);
    v[1] = make_float4(__uint_as_float(a.z), __uint_as_float(a.w), 0.0f, 0.0f);
    v[2] = make_float4(__uint_as_float(b.x), __uint_as_float(b.y), 0.0f, 0.0f);
    v[3] = make_float4(__uint_as_float(b.z), __uint_as_float(b.w), 0.0f, 0.0f);
  }
  static __device__ __forceinline__ uint32_t key(const T& r) { return r.x; }
};
struct RecBF16 {
  typedef uint3 T;
  // x-neighbour corners share a record: the records of a step are about
  // half as many, at 10 bytes instead of twice 6
  static constexpr bool kPaired = true;
  // the placement alternates an XCD's levels unit by unit, so each sample's
  // t and ray index are fetched once for both of its levels
  static constexpr bool kInterleaveLevels = true;
  static __device__ __forceinline__ uint32_t bf2(float a, float b) {
    const __bf16 x = (__bf16)a, y = (__bf16)b;
    return (uint32_t)__builtin_bit_cast(uint16_t, x) | ((uint32_t)__builtin_bit_cast(uint16_t, y) << 16);
  }
  static __device__ __forceinline__ float lo(uint32_t w) { return __uint_as_float(w << 16); }
  static __device__ __forceinline__ float hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }
  static __device__ __forceinline__ T pack(uint32_t key, float a, float b) { return make_uint3(key, bf2(a, b), 0u); }
  static __device__ __forceinline__ T pack_pair(uint32_t key, float a, float b, float c, float d) {
    return make_uint3(key, bf2(a, b), bf2(c, d));
  }
  // In the sorted array a record takes 10 bytes: the low 16 bits of its key
  // (the bin is implied by the slot) and the two BF16 pairs.
  static __device__ __forceinline__ void store(const RecordBuffers& rb, uint32_t pos, const T& r) {
    static_cast<uint16_t*>(rb.sorted)[pos] = (uint16_t)(r.x & 0xFFFFu);
    reinterpret_cast<uint2*>(rb.sorted_vals)[pos] = make_uint2(r.y, r.z);
  }
  static __device__ __forceinline__ uint32_t key(const T& r) { return r.x; }
  // the values of the four slots 4 gi .. 4 gi + 3 (x, y: the record's entry;
  // z, w: its partner's)
  static __device__ __forceinline__ void vals4(const RecordBuffers& rb, uint32_t gi, float4 (&v)[4]) {
    const uint4* p = reinterpret_cast<const uint4*>(rb.sorted_vals) + 2 * (size_t)gi;
    const uint4 a = p[0], b = p[1];
    v[0] = make_float4(lo(a.x), hi(a.x), lo(a.y), hi(a.y));
    v[1] = make_float4(lo(a.z), hi(a.z), lo(a.w), hi(a.w));
    v[2] = make_float4(lo(b.x), hi(b.x), lo(b.y), hi(b.y));
    v[3] = make_float4(lo(b.z), hi(b.z), lo(b.w), hi(b.w));
  }
};

__device__ __forceinline__ int sample_count(const SampleSrc& src) { return src.n_dev ? (int)*src.n_dev : src.n; }

// Entries [e0, e0 + ne) of bin b (b over the whole table).
__device__ __forceinline__ void bin_entries(const BinLevels& bl, int b, uint32_t& e0, uint32_t& ne) {
  int l = 0;
  while (l + 1 < bl.levels && bl.first[l + 1] <= (uint32_t)b) ++l;
  const uint32_t k = ((uint32_t)b - bl.first[l]) << kBinShift;
  e0 = bl.offset[l] + k;
  ne = min((uint32_t)kBinEntries, bl.size[l] - k);
}

// This thread's sample of unit u of level l: its position (the cell centre of
// the unit cube for samples beyond the batch) and whether it is one.
__device__ __forceinline__ bool unit_sample(const SampleSrc& src, int u, int& s, float xn[3]) {
  s = u * kUnitSamples + (int)threadIdx.x;
  const bool valid = s < sample_count(src);
  xn[0] = xn[1] = xn[2] = 0.5f;
  if (valid) load_position(src, s, xn);
  return valid;
}

template <bool kPaired>
__global__ __launch_bounds__(kUnitSamples) void bin_count_kernel(SampleSrc src, LevelInfo lv, BinLevels bl,
                                                                uint32_t* __restrict__ hist) {
  extern __shared__ uint32_t cnt[];
  int l, u;
  level_unit(bl.levels, bl.nunits, l, u);
  for (int k = threadIdx.x; k < bl.max_level_bins; k += kUnitSamples) cnt[k] = 0u;
  __syncthreads();
  int s;
  float xn[3];
  const bool valid = unit_sample(src, u, s, xn);
  Corner8 c;
  corners(xn[0], xn[1], xn[2], lv.res[l], (lv.dense_bits >> l) & 1u, lv.table_mask, lv.offset[l], c);
  count_records<kPaired>(c, row_run_head(c.cell, valid), lv.offset[l], cnt);
  __syncthreads();
  write_counts(bl, l, u, cnt, hist);
}

__global__ __launch_bounds__(kColThreads) void bin_colscan_kernel(RecordBuffers rb, int nunits) {
  colscan_bin(rb, nunits, (int)blockIdx.x);
}

// The column scan of nbins bins, then (workgroups nbins onwards) the
// weight-gradient and loss sums of the step.
template <class N>
__global__ __launch_bounds__(kColThreads) void bin_colscan_dw_kernel(RecordBuffers rb, int nunits, int nbins,
                                                                    WeightSum ws) {
  static_assert(kColThreads == 256, "the weight-gradient sum takes 256-thread workgroups");
  if ((int)blockIdx.x < nbins) {
    colscan_bin(rb, nunits, (int)blockIdx.x);
    return;
  }
  __shared__ float lds[kSumScratchFloats];
  dw_reduce_block<N>(ws.partial, ws.nblocks, ws.wo, ws.grads, ws.overflow, ws.ls, (int)blockIdx.x - nbins,
                     (int)gridDim.x - nbins, lds);
}

__global__ __launch_bounds__(1024) void bin_start_kernel(RecordBuffers rb, int nbins, uint32_t chunk, bool split) {
  bin_start_block<1024>(rb, nbins, chunk, split);
}

// The unit's records (at most eight a sample), generated as in the count,
// ordered by bin in LDS (counting sort with LDS integer atomics) and stored
// so that the global stores of a wave cover runs of consecutive slots of a
// few bins instead of one cache line per lane.
//
// zero_table (overwriting reductions only, else null): the gradient entries of
// the bins that the reduction will not overwrite (bins with no records, or
// with several chunks, which add with atomics) are cleared here first.
//
// The first nsum workgroups (a prescanned step's) sum the weight gradients
// and the loss of ws instead (dw_reduce_block, in the stage's memory), beside
// the placement; the placement starts at workgroup nskip, a multiple of 8 not
// below nsum, so that its units keep their XCDs.
template <class R, class N>
__global__ __launch_bounds__(kUnitSamples) void bin_place_kernel(SampleSrc src, LevelInfo lv, BinLevels bl,
                                                                RecordBuffers rb, float* __restrict__ zero_table,
                                                                WeightSum ws, int nsum, int nskip) {
  typedef typename R::T Rec;
  // cnt: the unit's records per bin of the level; lst: its exclusive prefix;
  // base: the slot of the unit's record i of bin k is base[k] + i.
  extern __shared__ uint32_t bins_lds[];
  uint32_t* cnt = bins_lds;
  uint32_t* lst = bins_lds + bl.max_level_bins;
  uint32_t* base = bins_lds + 2 * bl.max_level_bins;
  __shared__ uint32_t wsum[kUnitWaves];
  // paired records are about four a sample: a stage of six a sample keeps
  // the workgroup's LDS under 20 KB (eight workgroups a CU); a unit with more
  // records stores them unstaged
  constexpr int kStage = kUnitSamples * (R::kPaired ? 6 : 8);
  __shared__ Rec stage[kStage];
  static_assert(sizeof(stage) >= kSumScratchFloats * sizeof(float), "the sums borrow the stage");
  if ((int)blockIdx.x < nskip) {
    if ((int)blockIdx.x < nsum)
      dw_reduce_block<N>(ws.partial, ws.nblocks, ws.wo, ws.grads, ws.overflow, ws.ls, (int)blockIdx.x, nsum,
                         reinterpret_cast<float*>(stage));
    return;
  }
  const uint32_t wg = blockIdx.x - (uint32_t)nskip;
  const int nplace = (int)gridDim.x - nskip;
  const int t = (int)threadIdx.x, wave = t / kWave, lane = lane_id();
  int l, u;
  if (R::kInterleaveLevels)
    level_unit_interleaved(bl.levels, bl.nunits, l, u, wg);
  else
    level_unit(bl.levels, bl.nunits, l, u, wg);
  const int nb = (int)(bl.first[l + 1] - bl.first[l]);
  for (int k = t; k < nb; k += kUnitSamples) cnt[k] = 0u;
  if (zero_table) {
    const int nbins = (int)bl.first[bl.levels];
    for (int b = (int)wg; b < nbins; b += nplace) {
      if (rb.chunk_start[b + 1] - rb.chunk_start[b] == 1u) continue;
      uint32_t e0, ne;
      bin_entries(bl, b, e0, ne);
      float2* g = reinterpret_cast<float2*>(zero_table) + e0;
      for (uint32_t e = t; e < ne; e += kUnitSamples) g[e] = make_float2(0.0f, 0.0f);
    }
  }
  int s;
  float xn[3];
  const bool valid = unit_sample(src, u, s, xn);
  float2 d = make_float2(0.0f, 0.0f);
  if (valid) {
    const size_t i = (size_t)l * rb.stride + s;
    if (rb.de_bf16) {
      const uint32_t w = reinterpret_cast<const uint32_t*>(rb.de)[i];
      d = make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xFFFF0000u));
    } else {
      d = rb.de[i];
    }
  }
  Corner8 c;
  const uint32_t loff = lv.offset[l];
  corners(xn[0], xn[1], xn[2], lv.res[l], (lv.dense_bits >> l) & 1u, lv.table_mask, loff, c);
  float v[16];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[2 * k] = c.w[k] * d.x;
    v[2 * k + 1] = c.w[k] * d.y;
  }
  const bool on = row_cell_runs<16>(c.cell, valid, v) && valid;
  // records k (and k + 1 unless the pair shares record k): the key is
  // the bin << 16 | pair code << 13 | in-bin offset
  Rec rec[8];
  uint32_t rank[8], pc[4];
#pragma unroll
  for (int k = 0; k < 8; k += 2) {
    const uint32_t e0 = c.idx[k] - loff, e1 = c.idx[k + 1] - loff;
    const uint32_t p = R::kPaired ? pair_code(e0, e1) : 0u;
    pc[k / 2] = p;
    const uint32_t k0 = ((e0 >> kBinShift) << 16) | (p << 13) | (e0 & (uint32_t)(kBinEntries - 1));
    const uint32_t k1 = ((e1 >> kBinShift) << 16) | (e1 & (uint32_t)(kBinEntries - 1));
    if (p != 0u) {
      rec[k] = R::pack_pair(k0, v[2 * k], v[2 * k + 1], v[2 * k + 2], v[2 * k + 3]);
      rec[k + 1] = rec[k];
    } else {
      rec[k] = R::pack(k0, v[2 * k], v[2 * k + 1]);
      rec[k + 1] = R::pack(k1, v[2 * k + 2], v[2 * k + 3]);
    }
  }
  __syncthreads();
  // ranks in the bins: a paired record takes one; two records of the
  // x-neighbour corners (k, k + 1) nearly always share a bin and then take
  // two consecutive ranks from one atomic
  if (on) {
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
      const uint32_t ba = R::key(rec[k]) >> 16, bb = R::key(rec[k + 1]) >> 16;
      if (pc[k / 2] != 0u) {
        rank[k] = atomicAdd(&cnt[ba], 1u);
      } else if (ba == bb) {
        rank[k] = atomicAdd(&cnt[ba], 2u);
        rank[k + 1] = rank[k] + 1u;
      } else {
        rank[k] = atomicAdd(&cnt[ba], 1u);
        rank[k + 1] = atomicAdd(&cnt[bb], 1u);
      }
    }
  }
  __syncthreads();
  // lst = exclusive prefix of cnt (per-thread runs of bins, a wave scan of
  // the thread totals, then the totals of the waves before); base from the
  // bin's first slot and the unit's offset in it
  const int per = (nb + kUnitSamples - 1) / kUnitSamples;
  const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
  uint32_t mine = 0;
  for (int k = b0; k < b1; ++k) mine += cnt[k];
  const uint32_t incl = wave_incl_scan_u32(mine);
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  uint32_t run = incl - mine, m = 0;
#pragma unroll
  for (int w = 0; w < kUnitWaves; ++w) {
    run += w < wave ? wsum[w] : 0u;
    m += wsum[w];
  }
  for (int k = b0; k < b1; ++k) {
    const uint32_t b = bl.first[l] + (uint32_t)k;
    lst[k] = run;
    base[k] = rb.bin_start[b] + rb.off[(size_t)b * bl.nunits + u] - run;
    run += cnt[k];
  }
  __syncthreads();
  if (m > (uint32_t)kStage) {  // (uniform) each record straight to its slot
    if (on) {
#pragma unroll
      for (int k = 0; k < 8; k += 2) {
        const uint32_t ba = R::key(rec[k]) >> 16, bb = R::key(rec[k + 1]) >> 16;
        R::store(rb, base[ba] + lst[ba] + rank[k], rec[k]);
        if (pc[k / 2] == 0u) R::store(rb, base[bb] + lst[bb] + rank[k + 1], rec[k + 1]);
      }
    }
    return;
  }
  if (on) {
    // two records that took consecutive ranks in one bin take consecutive
    // slots
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
      const uint32_t ba = R::key(rec[k]) >> 16, bb = R::key(rec[k + 1]) >> 16;
      const uint32_t sa = lst[ba] + rank[k];
      stage[sa] = rec[k];
      if (pc[k / 2] != 0u) continue;
      if (ba == bb)
        stage[sa + 1] = rec[k + 1];
      else
        stage[lst[bb] + rank[k + 1]] = rec[k + 1];
    }
  }
  __syncthreads();
  for (uint32_t i = t; i < m; i += kUnitSamples) {
    const Rec r = stage[i];
    R::store(rb, base[R::key(r) >> 16] + i, r);
  }
}

// overwrite: a bin of one chunk stores its sums over every entry (zeros
// included) instead of adding them to the gradient.
template <class R>
__global__ __launch_bounds__(kReduceThreads) void bin_reduce_kernel(RecordBuffers rb, BinLevels bl, uint32_t chunk,
                                                                    bool scattered, bool split,
                                                                    float* __restrict__ grad_table,
                                                                    float* __restrict__ overflow, bool overwrite) {
  // (g0, g1) of each entry as one 64-bit word: float pairs are added with
  // LDS 64-bit compare-and-swap, which retires far faster than LDS float
  // atomics on this architecture
  __shared__ unsigned long long acc[kBinEntries];
  const int nbins = (int)bl.first[bl.levels];
  const uint32_t c = blockIdx.x;
  if (c >= rb.chunk_start[nbins]) return;
  const int b = (int)rb.chunk_bin[c];
  const uint32_t nch = rb.chunk_start[b + 1] - rb.chunk_start[b];
  const uint32_t csz = chunk_size_of(rb.bin_start[b + 1] - rb.bin_start[b], chunk, split);
  const uint32_t first = rb.bin_start[b] + (c - rb.chunk_start[b]) * csz;
  const uint32_t last = min(rb.bin_start[b + 1], first + csz);
  for (int i = threadIdx.x; i < kBinEntries; i += kReduceThreads) acc[i] = 0ull;
  __syncthreads();
  uint32_t e0, ne;
  bin_entries(bl, b, e0, ne);
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
  // With small chunks (tables of few bins, whose coarse levels put runs of
  // records of one entry next to each other), the threads take the groups
  // in a scattered order (t -> 29 t mod 1024), so that the lanes of a wave
  // meet different entries in their compare-and-swap instead of queueing on
  // one; with full chunks they read consecutive groups, coalesced.
  const uint32_t tp = scattered ? (threadIdx.x * 29u) & (kReduceThreads - 1) : threadIdx.x;
  for (uint32_t gb = g0; gb < g1; gb += kReduceThreads * 2) {
    uint2 kk[2];
    float4 vv[2][4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint32_t gi = gb + j * kReduceThreads + tp;
      const uint32_t gc = gi < g1 ? gi : g0;  // a group of this chunk either way
      kk[j] = keys[gc];
      R::vals4(rb, gc, vv[j]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint32_t p0 = 4 * (gb + j * kReduceThreads + tp);
      const uint32_t k4[4] = {kk[j].x & 0xFFFFu, kk[j].x >> 16, kk[j].y & 0xFFFFu, kk[j].y >> 16};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (p0 + u < first || p0 + u >= last) continue;
        const uint32_t o = k4[u] & (uint32_t)(kBinEntries - 1);
        add(o, vv[j][u].x, vv[j][u].y);
        if (R::kPaired) {
          const uint32_t pc = k4[u] >> 13;
          if (pc != 0u) add(o ^ ((1u << pc) - 1u), vv[j][u].z, vv[j][u].w);
        }
      }
    }
  }
  __syncthreads();
  // every gradient value written is checked for the loss-scale overflow flag
  // (for the atomic adds, the value each add leaves)
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

BinPlan bin_plan(const LevelInfo& lv, uint32_t entries, int64_t max_samples) {
  BinPlan p{};
  p.entries = entries;
  p.levels = lv.levels;
  p.stride = (int)max_samples;
  p.nunits = (int)((max_samples + kUnitSamples - 1) / kUnitSamples);
  BinLevels& bl = p.bl;
  bl.levels = lv.levels;
  bl.nunits = p.nunits;
  uint32_t nb = 0;
  for (int l = 0; l < lv.levels; ++l) {
    const uint32_t end = l + 1 < lv.levels ? lv.offset[l + 1] : entries;
    bl.offset[l] = lv.offset[l];
    bl.size[l] = end - lv.offset[l];
    bl.first[l] = nb;
    const int k = (int)((bl.size[l] + kBinEntries - 1) >> kBinShift);
    nb += (uint32_t)k;
    bl.max_level_bins = std::max(bl.max_level_bins, k);
  }
  bl.first[lv.levels] = nb;
  p.nbins = (int)nb;
  p.max_records = max_samples * 8 * lv.levels;
  // a table of few bins (the tiny field has four) would leave a few huge
  // chunks: there the chunk shrinks (to a power of two of at least 4096) so
  // that a full batch of records makes up to about 8192 chunks; their sums
  // then meet in the gradient through atomics, one per touched entry and chunk
  p.chunk = kChunk;
  if (p.nbins < 256) {
    uint32_t c = 4096;
    while (c < kChunk && (int64_t)c * 2 * 8192 <= p.max_records) c *= 2;
    p.chunk = c;
  }
  // paired records (two corner additions each) are cut into chunks of half
  // as many, and, unless the table has few bins, bins that take several
  // chunks into chunks of half the size (bin_split)
  const uint32_t smallest = bin_split(p) ? p.chunk / 4 : p.chunk / 2;
  p.max_chunks = (int)(p.nbins + (p.max_records + smallest - 1) / smallest);
  return p;
}

// Tables of few bins already cut small chunks.
bool bin_split(const BinPlan& p) { return p.chunk >= kChunk; }

uint32_t bin_chunk(const BinPlan& p, bool bf16_values) {
  // a chunk holds at most p.chunk corner additions: as many records, or half
  // as many paired ones
  return bf16_values && RecBF16::kPaired ? p.chunk / 2 : p.chunk;
}

namespace {

template <class R, class N>
void launch_place(const BinPlan& p, const RecordBuffers& rb, const SampleSrc& src, const LevelInfo& lv,
                  float* zero_table, const WeightSum* sums, hipStream_t st) {
  const int nplace = p.levels * p.nunits;
  const int nsum = sums ? dw_reduce_blocks<N>(sums->ls.loss != nullptr) : 0;
  const int nskip = (nsum + 7) / 8 * 8;
  const size_t level_lds = (size_t)p.bl.max_level_bins * sizeof(uint32_t);
  hipLaunchKernelGGL((bin_place_kernel<R, N>), dim3(nskip + nplace), dim3(kUnitSamples), 3 * level_lds, st, src, lv,
                     p.bl, rb, zero_table, sums ? *sums : WeightSum{}, nsum, nskip);
}

template <class R>
void place_and_reduce(const BinPlan& p, const RecordBuffers& rb, const SampleSrc& src, const LevelInfo& lv,
                      bool overwrite, float* grad_table, float* overflow, const WeightSum* sums, hipStream_t st) {
  float* zero_table = overwrite ? grad_table : nullptr;
  if (sums && sums->shape == kShapeTiny)
    launch_place<R, NetTiny>(p, rb, src, lv, zero_table, sums, st);
  else
    launch_place<R, NetFull>(p, rb, src, lv, zero_table, sums, st);
  // the small chunks of tables of few bins read their record groups in a
  // scattered order
  const bool scattered = p.chunk < kChunk;
  hipLaunchKernelGGL(bin_reduce_kernel<R>, dim3(p.max_chunks), dim3(kReduceThreads), 0, st, rb, p.bl,
                     bin_chunk(p, R::kPaired), scattered, bin_split(p), grad_table, overflow, overwrite);
}

}  // namespace

hipError_t bin_scatter(const BinPlan& p, const RecordBuffers& rb, const SampleSrc& src, const LevelInfo& lv,
                       bool bf16_values, bool overwrite, float* grad_table, float* overflow, hipStream_t st,
                       bool counted, const WeightSum* ws, bool prescanned) {
  if (p.nbins == 0 || p.nunits == 0) {
    return ws ? field_dw_reduce(ws->shape, ws->partial, ws->nblocks, ws->wo, ws->grads, ws->overflow,
                                ws->ls.loss ? &ws->ls : nullptr, st)
              : hipSuccess;
  }
  if (!prescanned) {
    const dim3 grid(p.levels * p.nunits);
    const size_t level_lds = (size_t)p.bl.max_level_bins * sizeof(uint32_t);
    if (!counted) {
      if (bf16_values)
        hipLaunchKernelGGL(bin_count_kernel<RecBF16::kPaired>, grid, dim3(kUnitSamples), level_lds, st, src, lv,
                           p.bl, rb.hist);
      else
        hipLaunchKernelGGL(bin_count_kernel<RecF32::kPaired>, grid, dim3(kUnitSamples), level_lds, st, src, lv,
                           p.bl, rb.hist);
    }
    if (ws) {
      const bool loss = ws->ls.loss != nullptr;
      if (ws->shape == kShapeTiny)
        hipLaunchKernelGGL(bin_colscan_dw_kernel<NetTiny>, dim3(p.nbins + dw_reduce_blocks<NetTiny>(loss)),
                           dim3(kColThreads), 0, st, rb, p.nunits, p.nbins, *ws);
      else
        hipLaunchKernelGGL(bin_colscan_dw_kernel<NetFull>, dim3(p.nbins + dw_reduce_blocks<NetFull>(loss)),
                           dim3(kColThreads), 0, st, rb, p.nunits, p.nbins, *ws);
    } else {
      hipLaunchKernelGGL(bin_colscan_kernel, dim3(p.nbins), dim3(kColThreads), 0, st, rb, p.nunits);
    }
    hipLaunchKernelGGL(bin_start_kernel, dim3(1), dim3(1024), 0, st, rb, p.nbins, bin_chunk(p, bf16_values),
                       bin_split(p));
  }
  // with the scans done earlier, the weight and loss sums ride along the
  // placement
  const WeightSum* sums = prescanned ? ws : nullptr;
  if (bf16_values)
    place_and_reduce<RecBF16>(p, rb, src, lv, overwrite, grad_table, overflow, sums, st);
  else
    place_and_reduce<RecF32>(p, rb, src, lv, overwrite, grad_table, overflow, sums, st);
  return hipGetLastError();
}

}  // namespace nsl
