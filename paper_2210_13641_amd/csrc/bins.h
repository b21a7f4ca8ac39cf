// The two small scans of the table-gradient counting sort (csrc/scatter.hip):
// per bin, the exclusive prefix of its record counts over the units; over
// the bins, their first slots and chunks.  They are block functions, so that
// the training step can run them as extra workgroups of launches that do
// not depend on them (the forward MLP and the compositing), off the
// table-gradient chain.
#pragma once
#include "kernels.h"

namespace nsl {

constexpr int kColThreads = 256;

// off[b][u] = sum over units u' < u of hist[b][u']; total[b] = sum over all
// units.  One workgroup per bin; a thread takes four consecutive units.
__device__ __forceinline__ void colscan_bin(const RecordBuffers& rb, int nunits, int b) {
  __shared__ uint32_t wsum[kColThreads / kWave];
  const int t = (int)threadIdx.x, wave = t / kWave, lane = lane_id();
  const uint32_t* __restrict__ h = rb.hist + (size_t)b * nunits;
  uint32_t* __restrict__ o = rb.off + (size_t)b * nunits;
  uint32_t carry = 0;
  for (int seg = 0; seg < nunits; seg += 4 * kColThreads) {
    const int i0 = seg + 4 * t;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = i0 + k < nunits ? h[i0 + k] : 0u;
      sum += v[k];
    }
    const uint32_t incl = wave_incl_scan_u32(sum);
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    uint32_t run = carry + incl - sum, all = 0;
#pragma unroll
    for (int w = 0; w < kColThreads / kWave; ++w) {
      run += w < wave ? wsum[w] : 0u;
      all += wsum[w];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (i0 + k < nunits) o[i0 + k] = run;
      run += v[k];
    }
    carry += all;
    __syncthreads();
  }
  if (t == 0) rb.bin_total[b] = carry;
}

// The records of each chunk of a bin of n records, and its chunks: one chunk
// when the bin fits; with split, a bin that does not fit takes chunks of half
// the size.  Such bins are the heavy bins of the coarse dense levels, whose
// chunks also meet the most compare-and-swap retries in the reduction, so
// they are spread over more workgroups.
__host__ __device__ __forceinline__ uint32_t chunk_size_of(uint32_t n, uint32_t chunk, bool split) {
  return split && n > chunk ? chunk / 2 : chunk;
}
__host__ __device__ __forceinline__ uint32_t chunks_of(uint32_t n, uint32_t chunk, bool split) {
  const uint32_t c = chunk_size_of(n, chunk, split);
  return (n + c - 1) / c;
}

// bin_start = exclusive prefix of the totals, chunk_start = exclusive prefix
// of the chunks per bin; both with the grand total at [nbins].
// One workgroup of THREADS threads.
constexpr int kMaxStartBins = (int)(kMaxTableEntries / kBinEntries) + kMaxLevels;  // bins of any table
template <int THREADS>
__device__ __forceinline__ void bin_start_block(const RecordBuffers& rb, int nbins, uint32_t chunk, bool split) {
  __shared__ uint32_t w_rec[THREADS / kWave], w_chk[THREADS / kWave];
  const int t = threadIdx.x;
  const int per = (nbins + THREADS - 1) / THREADS;
  const int b0 = min(nbins, t * per), b1 = min(nbins, b0 + per);
  uint32_t rec = 0, chk = 0;
  for (int b = b0; b < b1; ++b) {
    const uint32_t n = rb.bin_total[b];
    rec += n;
    chk += chunks_of(n, chunk, split);
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
  for (int w = 0; w < THREADS / kWave; ++w) {
    run_r += w < wave ? w_rec[w] : 0u;
    run_c += w < wave ? w_chk[w] : 0u;
    all_r += w_rec[w];
    all_c += w_chk[w];
  }
  // the chunk starts also go to LDS, where every thread then finds the bin of
  // chunks t, t + THREADS, ... by binary search (a bin of many chunks would
  // otherwise leave one thread writing all of its entries)
  __shared__ uint32_t cs[kMaxStartBins + 1];
  for (int b = b0; b < b1; ++b) {
    const uint32_t n = rb.bin_total[b];
    rb.bin_start[b] = run_r;
    rb.chunk_start[b] = run_c;
    cs[b] = run_c;
    run_r += n;
    run_c += chunks_of(n, chunk, split);
  }
  if (t == THREADS - 1) {
    rb.bin_start[nbins] = all_r;
    rb.chunk_start[nbins] = all_c;
    cs[nbins] = all_c;
  }
  __syncthreads();
  for (uint32_t c = t; c < all_c; c += THREADS) {
    int lo = 0, hi = nbins;  // the last bin b with cs[b] <= c (bins of no chunks are skipped)
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (cs[mid] <= c) lo = mid;
      else hi = mid;
    }
    rb.chunk_bin[c] = (uint32_t)lo;
  }
}


}  // namespace nsl
