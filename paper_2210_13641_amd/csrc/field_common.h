// Device helpers shared by the FP32 and mixed-precision field kernels:
// per-sample inputs, grid corners and trilinear encoding, SH, row scans.
#pragma once
#include "kernels.h"
#include "net.h"

namespace nsl {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Per-sample inputs
// ---------------------------------------------------------------------------

// Normalised position of sample s (the direction is not read).
__device__ __forceinline__ void load_position(const SampleSrc& src, int s, float xn[3]) {
  if (src.t) {
    const uint32_t r = src.ray[s];
    const float t = src.t[s];
    const float4 o = src.rays[2 * r];
    const float4 dd = src.rays[2 * r + 1];
    xn[0] = normalise_axis(pos_axis(o.x, dd.x, t), src.box.lo[0], src.box.inv[0]);
    xn[1] = normalise_axis(pos_axis(o.y, dd.y, t), src.box.lo[1], src.box.inv[1]);
    xn[2] = normalise_axis(pos_axis(o.z, dd.z, t), src.box.lo[2], src.box.inv[2]);
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i) xn[i] = fminf(fmaxf(src.xn[3 * s + i], 0.0f), 1.0f);
  }
}

// View direction of sample s.
__device__ __forceinline__ void load_direction(const SampleSrc& src, int s, float d[3]) {
  if (src.t) {
    const float4 dd = src.rays[2 * src.ray[s] + 1];
    d[0] = dd.x; d[1] = dd.y; d[2] = dd.z;
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i) d[i] = src.dir[3 * s + i];
  }
}

__device__ __forceinline__ void load_sample(const SampleSrc& src, int s, float xn[3],
                                            float d[3]) {
  load_position(src, s, xn);
  load_direction(src, s, d);
}

// Per-lane level constants (levels g, g+4, ... of this lane group).
template <class N>
struct LaneLevels {
  int res[N::LPL];
  uint32_t off[N::LPL];
  bool dense[N::LPL];
};

template <class N>
__device__ __forceinline__ void lane_levels(const LevelInfo& lv, int g, LaneLevels<N>& ll) {
#pragma unroll
  for (int q = 0; q < N::LPL; ++q) {
    const int l = g + 4 * q;
    ll.res[q] = lv.res[l];
    ll.off[q] = lv.offset[l];
    ll.dense[q] = (lv.dense_bits >> l) & 1u;
  }
}

struct Corner8 {
  uint32_t idx[8];
  float w[8];
  uint32_t cell[3];  // integer coordinates of the cell's lower corner
};

__device__ __forceinline__ void corners(float x, float y, float z, int n, bool dense,
                                        uint32_t mask, uint32_t off, Corner8& c) {
  float fx, fy, fz, ux, uy, uz;
  const uint32_t ix = (uint32_t)cell_floor(x, n, fx, ux);
  const uint32_t iy = (uint32_t)cell_floor(y, n, fy, uy);
  const uint32_t iz = (uint32_t)cell_floor(z, n, fz, uz);
  c.cell[0] = ix;
  c.cell[1] = iy;
  c.cell[2] = iz;
  const float gx[2] = {ux, fx}, gy[2] = {uy, fy}, gz[2] = {uz, fz};
  // grid_index per corner, with the per-axis terms formed once: a dense
  // index is x + m y + m^2 z, a hashed one (x ^ P1 y ^ P2 z) & mask, and the
  // upper corner's term is the lower one's plus m, m^2, P1 or P2 (all mod 2^32)
  uint32_t ty[2], tz[2];
  if (dense) {
    const uint32_t m = (uint32_t)n + 1u, m2 = m * m;
    ty[0] = iy * m;
    tz[0] = iz * m2;
    ty[1] = ty[0] + m;
    tz[1] = tz[0] + m2;
  } else {
    ty[0] = iy * kPrime1;
    tz[0] = iz * kPrime2;
    ty[1] = ty[0] + kPrime1;
    tz[1] = tz[0] + kPrime2;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t cx = k & 1, cy = (k >> 1) & 1, cz = (k >> 2) & 1;
    c.idx[k] = off + (dense ? (ix + cx) + ty[cy] + tz[cz] : ((ix + cx) ^ ty[cy] ^ tz[cz]) & mask);
    c.w[k] = (gx[cx] * gy[cy]) * gz[cz];
  }
}

// Two features of table entry idx as floats (FP32 or FP16 storage).
__device__ __forceinline__ float2 load_entry(const float* __restrict__ t, uint32_t idx) {
  return *reinterpret_cast<const float2*>(t + 2 * (size_t)idx);
}
__device__ __forceinline__ float2 load_entry(const _Float16* __restrict__ t, uint32_t idx) {
  const h2 v = *reinterpret_cast<const h2*>(t + 2 * (size_t)idx);
  return make_float2((float)v[0], (float)v[1]);
}

// The trilinear blend of a cell's eight corners, in corner order.
template <class T>
__device__ __forceinline__ float2 blend_corners(const T* __restrict__ table, const Corner8& c) {
  float2 v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = load_entry(table, c.idx[k]);
  float a0 = 0.0f, a1 = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a0 += c.w[k] * v[k].x;
    a1 += c.w[k] * v[k].y;
  }
  return make_float2(a0, a1);
}

// Trilinear blend of one level's two features at xn.
template <class T>
__device__ __forceinline__ float2 encode_level(const T* __restrict__ table, uint32_t mask, int res, bool dense,
                                               uint32_t off, const float xn[3]) {
  Corner8 c;
  corners(xn[0], xn[1], xn[2], res, dense, mask, off, c);
  return blend_corners(table, c);
}

template <class N, class T>
__device__ __forceinline__ void encode(const T* __restrict__ table, uint32_t mask,
                                       const LaneLevels<N>& ll, const float xn[3],
                                       float e[N::NSLOT]) {
#pragma unroll
  for (int q = 0; q < N::LPL; ++q) {
    const float2 v = encode_level(table, mask, ll.res[q], ll.dense[q], ll.off[q], xn);
    e[2 * q] = v.x;
    e[2 * q + 1] = v.y;
  }
}

// The kept encoding, level-major [level][ecache_stride]: FP32 pairs, or BF16
// pairs (as the mixed-precision MLP consumes them) packed in 32 bits.
__device__ __forceinline__ void store_encoding(float2* out, float2 v) { *out = v; }
__device__ __forceinline__ void store_encoding(uint32_t* out, float2 v) {
  const __bf16 a = (__bf16)v.x, b = (__bf16)v.y;
  *out = (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}
__device__ __forceinline__ float2 load_encoding(const float2* in) { return *in; }
__device__ __forceinline__ float2 load_encoding(const uint32_t* in) {
  const uint32_t w = *in;
  return make_float2((float)__builtin_bit_cast(__bf16, (uint16_t)(w & 0xFFFFu)),
                     (float)__builtin_bit_cast(__bf16, (uint16_t)(w >> 16)));
}

// This lane's encoding slots (levels g + 4q of sample s) from the kept
// encoding; zero for samples beyond the batch.
template <class N, class E>
__device__ __forceinline__ void read_encoding(const E* __restrict__ ec, int stride, int g, int s, bool valid,
                                              float e[N::NSLOT]) {
#pragma unroll
  for (int q = 0; q < N::LPL; ++q) {
    const float2 v = valid ? load_encoding(ec + (size_t)(g + 4 * q) * stride + s) : make_float2(0.0f, 0.0f);
    e[2 * q] = v.x;
    e[2 * q + 1] = v.y;
  }
}

// The encoding of every sample, written level-major for the MLP kernels.
// One workgroup per kEncodeUnits consecutive units of one level (units of
// 256 samples, see level_unit), a thread taking one sample of each, so that
// the dependent loads of its samples (ray index and t, the ray, the corners)
// are in flight together.  Workgroups are dispatched round-robin over the 8
// XCDs, in order; with 16 levels, the workgroups of XCD x evaluate level x
// for every sample and then level x + 8, so at any time each XCD's L2 holds
// the table slice of one level (2 MB in FP16) instead of seeing the whole
// table, and the random corner reads hit in L2.
constexpr int kEncodeUnits = 2;
template <class N>
__host__ __device__ constexpr int encode_grid(int max_samples) {
  return N::L * ((max_samples + 256 * kEncodeUnits - 1) / (256 * kEncodeUnits));
}

// Workgroup -> (level l, unit u) of the level-major kernels (the encoding
// with 16 levels, the record counting and placement), unit u being samples
// [u * kUnitSamples, (u + 1) * kUnitSamples) of level l.  Workgroups are
// dispatched round-robin over the 8 XCDs, in order: with a multiple of 8
// levels, XCD x takes level x for every unit, then level x + 8, and so on, so
// that consecutive units of a level run on one XCD; with other level counts
// consecutive workgroups take consecutive levels.
// wg: the workgroup's index among those of the kernel (a launch that puts
// other work in its first workgroups passes blockIdx.x less a multiple of 8).
__device__ __forceinline__ void level_unit(int levels, int nunits, int& l, int& u, uint32_t wg) {
  if (levels % 8 == 0) {
    const int x = (int)(wg % 8u), j = (int)(wg / 8u);
    l = x + 8 * (j / nunits);
    u = j % nunits;
  } else {
    l = (int)(wg % (uint32_t)levels);
    u = (int)(wg / (uint32_t)levels);
  }
}
__device__ __forceinline__ void level_unit(int levels, int nunits, int& l, int& u) {
  level_unit(levels, nunits, l, u, blockIdx.x);
}

// As level_unit, but with a multiple of 8 levels the workgroups of XCD x
// alternate between its levels x, x + 8, ... unit by unit, so that the
// samples' inputs that every level reads are fetched into that XCD's L2
// once for all of its levels (for kernels that gather no table, whose L2
// need not hold one level's slice at a time).
__device__ __forceinline__ void level_unit_interleaved(int levels, int nunits, int& l, int& u, uint32_t wg) {
  if (levels % 8 == 0) {
    const int m = levels / 8;
    const int x = (int)(wg % 8u), j = (int)(wg / 8u);
    l = x + 8 * (j % m);
    u = j / m;
  } else {
    level_unit(levels, nunits, l, u, wg);
  }
}

// The x-neighbour corners k, k + 1 (k even) of a cell lie at in-level
// offsets e0 and e1 that nearly always differ in low bits only: a hashed
// level multiplies x by 1, and a dense one stores x + 1 next to x, so that
// e1 = e0 ^ (2^p - 1) with p the carry length of the increment.  When
// 1 <= p <= 7 (the bin is the same, since bins are 2^13 entries) the two
// corners can travel as one paired record; returns p, else 0.
__device__ __forceinline__ uint32_t pair_code(uint32_t e0, uint32_t e1) {
  const uint32_t d = e0 ^ e1;
  return (d != 0u && d < 128u && (d & (d + 1u)) == 0u) ? 32u - (uint32_t)__clz((int)d) : 0u;
}

// The table-gradient records of a lane that starts a run (see row_cell_runs:
// one record per corner, for the first sample of each run of consecutive
// samples of an aligned group of 16 that share a cell), counted per bin of
// the level in cnt (LDS): the bin of entry idx is (idx - level_off) >>
// kBinShift.  The two x-neighbour corners (k, k + 1) nearly always share a
// bin, and then one atomic counts both; with kPaired, two corners that
// pair_code joins take one slot.
template <bool kPaired>
__device__ __forceinline__ void count_records(const Corner8& c, bool head, uint32_t level_off, uint32_t* cnt) {
  if (!head) return;
#pragma unroll
  for (int k = 0; k < 8; k += 2) {
    const uint32_t e0 = c.idx[k] - level_off, e1 = c.idx[k + 1] - level_off;
    const uint32_t ba = e0 >> kBinShift, bb = e1 >> kBinShift;
    if (kPaired && pair_code(e0, e1) != 0u) {
      atomicAdd(&cnt[ba], 1u);
    } else if (ba == bb) {
      atomicAdd(&cnt[ba], 2u);
    } else {
      atomicAdd(&cnt[ba], 1u);
      atomicAdd(&cnt[bb], 1u);
    }
  }
}

// The workgroup's counts of level l, unit u into hist[bin][unit].
__device__ __forceinline__ void write_counts(const BinLevels& bl, int l, int u, const uint32_t* cnt,
                                             uint32_t* __restrict__ hist) {
  const int nb = (int)(bl.first[l + 1] - bl.first[l]);
  for (int k = threadIdx.x; k < nb; k += blockDim.x) hist[(size_t)(bl.first[l] + k) * bl.nunits + u] = cnt[k];
}

// With hist set, the kernel also counts the table-gradient records of its
// unit per bin exactly as the scatter's counting pass would, and writes them
// to hist[bin][unit] (every workgroup writes its row, so hist needs no
// clearing).  The counting pass of the scatter is then skipped.  The
// mixed-precision step (FP16 table) places its records in x-neighbour pairs,
// the FP32 step one corner a record.
template <class N, class T, class E>
__global__ __launch_bounds__(256) void encode_levels_kernel(LevelInfo lv, const T* __restrict__ table, SampleSrc src,
                                                            E* __restrict__ out, int stride,
                                                            uint32_t* __restrict__ hist, BinLevels bl) {
  static_assert(kUnitSamples == 256, "one sample of each unit per thread");
  constexpr int U = kEncodeUnits;
  const int S = src.n_dev ? (int)*src.n_dev : src.n;
  int l, ug;
  level_unit(N::L, (int)(gridDim.x / (uint32_t)N::L), l, ug);
  const bool dense = (lv.dense_bits >> l) & 1u;
  int s[U];
  bool valid[U];
  float xn[U][3];
#pragma unroll
  for (int k = 0; k < U; ++k) {
    s[k] = (ug * U + k) * 256 + (int)threadIdx.x;
    valid[k] = s[k] < S;
    xn[k][0] = xn[k][1] = xn[k][2] = 0.5f;
    if (valid[k]) load_position(src, s[k], xn[k]);
  }
  Corner8 c[U];
#pragma unroll
  for (int k = 0; k < U; ++k) corners(xn[k][0], xn[k][1], xn[k][2], lv.res[l], dense, lv.table_mask, lv.offset[l], c[k]);
#pragma unroll
  for (int k = 0; k < U; ++k)
    if (valid[k]) store_encoding(out + (size_t)l * stride + s[k], blend_corners(table, c[k]));
  if (!hist) return;
  __shared__ uint32_t cnt[U][kEncodeLevelBins];
  for (int i = threadIdx.x; i < U * kEncodeLevelBins; i += 256) (&cnt[0][0])[i] = 0u;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < U; ++k)
    count_records<sizeof(T) == 2>(c[k], row_run_head(c[k].cell, valid[k]), lv.offset[l], cnt[k]);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < U; ++k)
    if (ug * U + k < bl.nunits) write_counts(bl, l, ug * U + k, cnt[k], hist);
}

// Real orthonormal SH coefficients 4g..4g+3 of direction d (0 beyond NSH).
template <class N>
__device__ __forceinline__ void sh_lane(const float d[3], int g, float out[4]) {
  const float x = d[0], y = d[1], z = d[2];
  float Y[16];
  Y[0] = 0.28209479177387814f;
  Y[1] = 0.4886025119029199f * y;
  Y[2] = 0.4886025119029199f * z;
  Y[3] = 0.4886025119029199f * x;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = 1.0925484305920792f * x * y;
  Y[5] = 1.0925484305920792f * y * z;
  Y[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);
  Y[7] = 1.0925484305920792f * x * z;
  Y[8] = 0.5462742152960396f * (xx - yy);
  if (N::SHB > 3) {
    Y[9] = 0.5900435899266435f * y * (3.0f * xx - yy);
    Y[10] = 2.890611442640554f * x * y * z;
    Y[11] = 0.4570457994644658f * y * (5.0f * zz - 1.0f);
    Y[12] = 0.3731763325901154f * z * (5.0f * zz - 3.0f);
    Y[13] = 0.4570457994644658f * x * (5.0f * zz - 1.0f);
    Y[14] = 1.445305721320277f * z * (xx - yy);
    Y[15] = 0.5900435899266435f * x * (xx - 3.0f * yy);
  } else {
#pragma unroll
    for (int k = 9; k < 16; ++k) Y[k] = 0.0f;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
    out[r] = g == 0 ? Y[r] : g == 1 ? Y[4 + r] : g == 2 ? Y[8 + r] : Y[12 + r];
}

__device__ __forceinline__ f4 relu4(f4 v) {
  return f4{fmaxf(v[0], 0.0f), fmaxf(v[1], 0.0f), fmaxf(v[2], 0.0f), fmaxf(v[3], 0.0f)};
}


__device__ __forceinline__ void wave_lds_fence() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// Inclusive prefix sum within each 16-lane row.
__device__ __forceinline__ float row_incl_scan(float v) {
  v += __int_as_float(row_from_below<1>(__float_as_int(v)));
  v += __int_as_float(row_from_below<2>(__float_as_int(v)));
  v += __int_as_float(row_from_below<4>(__float_as_int(v)));
  v += __int_as_float(row_from_below<8>(__float_as_int(v)));
  return v;
}

__device__ __forceinline__ float row_sum(float v) {
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 16);
  return v;
}

// Weight-gradient tile set of one layer (KIN x KOUT, padded to 16 x 16
// tiles), kept as MFMA accumulators in registers across all tiles a wave
// processes: tile (m, n), lane (gk, i) holds dW[16m + 4gk + r][16n + i].
template <int KIN, int KOUT>
struct DWAcc {
  static constexpr int MI = (KIN + 15) / 16, NJ = (KOUT + 15) / 16;
  f4 v[MI * NJ];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int t = 0; t < MI * NJ; ++t) v[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  // dW (LDS, row-major KIN x KOUT) += this wave's sums; plain read-modify-
  // write, so the waves of a workgroup call it one at a time.
  __device__ __forceinline__ void flush(float* dW, int lane) const {
    const int gk = lane >> 4, i = lane & 15;
#pragma unroll
    for (int m = 0; m < MI; ++m)
#pragma unroll
      for (int n = 0; n < NJ; ++n) {
        const int col = 16 * n + i;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * m + 4 * gk + r;
          if (row < KIN && col < KOUT) dW[row * KOUT + col] += v[m * NJ + n][r];
        }
      }
  }
};

// LDS scratch of the sums below (floats), passed in by the kernel, which may
// lend memory it uses otherwise.
constexpr int kSumScratchFloats = 512;

// The loss of a step from its per-ray shares, summed in a fixed order by one
// 256-thread workgroup: loss = (L_rgb + lambda_d L_D, L_rgb, L_D).
__device__ __forceinline__ void loss_sum_block(const LossSum& ls, float* lds) {
  float* s0 = lds;
  float* s1 = lds + 256;
  const int t = threadIdx.x;
  const float2* __restrict__ p2 = reinterpret_cast<const float2*>(ls.parts);
  float a = 0.0f, b = 0.0f;
  for (int r0 = 0; r0 < ls.R; r0 += 256 * 16) {
    float2 v[16];  // sixteen loads in flight, added in ray order
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int r = r0 + 256 * k + t;
      v[k] = r < ls.R ? p2[r] : make_float2(0.0f, 0.0f);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      a += v[k].x;
      b += v[k].y;
    }
  }
  s0[t] = a;
  s1[t] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      s0[t] += s0[t + o];
      s1[t] += s1[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    ls.loss[0] = s0[0] + ls.lambda_d * s1[0];
    ls.loss[1] = s0[0];
    ls.loss[2] = s1[0];
  }
}

// grads[weights] += sum over blocks of the per-block weight gradients, in a
// fixed order: a workgroup takes 16 weights, each of its 16 thread groups
// sums every 16th partial (all loads of a thread in flight at once), and the
// 16 sums are added in LDS.  With ls.loss set, one more workgroup sums the
// loss of the step.  Workgroup b of nb (256 threads) of such a launch.
template <class N>
constexpr int dw_reduce_blocks(bool with_loss) {
  return (N::NWEIGHTS + 15) / 16 + (with_loss ? 1 : 0);
}

template <class N>
__device__ __forceinline__ void dw_reduce_block(const float* __restrict__ partial, int nblocks, const WOffsets& wo,
                                                float* __restrict__ grads, float* __restrict__ overflow,
                                                const LossSum& ls, int b, int nb, float* lds) {
  if (ls.loss && b == nb - 1) {
    loss_sum_block(ls, lds);
    return;
  }
  float(*red)[16] = reinterpret_cast<float(*)[16]>(lds);
  const int wl = threadIdx.x & 15, pg = threadIdx.x >> 4;
  const int i = b * 16 + wl;
  float acc = 0.0f;
  if (i < N::NWEIGHTS) {
    for (int b0 = pg; b0 < nblocks; b0 += 256) {
      float v[16];  // sixteen loads in flight, added in block order
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int bb = b0 + 16 * k;
        v[k] = bb < nblocks ? partial[(size_t)bb * N::NWEIGHTS + i] : 0.0f;
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) acc += v[k];
    }
  }
  red[pg][wl] = acc;
  __syncthreads();
  if (pg != 0 || i >= N::NWEIGHTS) return;
  float sum = 0.0f;
#pragma unroll
  for (int k = 0; k < 16; ++k) sum += red[k][wl];
  int j = 0;
  while (j + 1 < N::NW && i >= N::woff(j + 1)) ++j;
  float* g = grads + wo.off[j] + (i - N::woff(j));
  const float r = *g + sum;
  *g = r;
  if (overflow && !isfinite(r)) *overflow = 1.0f;
}

template <class N>
__global__ __launch_bounds__(256) void dw_reduce_kernel(const float* __restrict__ partial, int nblocks, WOffsets wo,
                                                        float* __restrict__ grads, float* __restrict__ overflow,
                                                        LossSum ls) {
  __shared__ float lds[kSumScratchFloats];
  dw_reduce_block<N>(partial, nblocks, wo, grads, overflow, ls, (int)blockIdx.x, (int)gridDim.x, lds);
}

template <class N>
__host__ inline hipError_t launch_dw_reduce(const float* partial, int nblocks, const WOffsets& wo, float* grads,
                                           float* overflow, const LossSum* ls, hipStream_t st) {
  const LossSum none{};
  hipLaunchKernelGGL(dw_reduce_kernel<N>, dim3(dw_reduce_blocks<N>(ls != nullptr)), dim3(256), 0, st, partial,
                     nblocks, wo, grads, overflow, ls ? *ls : none);
  return hipGetLastError();
}

template <class N>
__device__ __forceinline__ void load_operands(float* dst, const float* __restrict__ src, int n) {
  for (int i = threadIdx.x * 4; i < n; i += blockDim.x * 4)
    *reinterpret_cast<float4*>(dst + i) = *reinterpret_cast<const float4*>(src + i);
}

}  // namespace nsl
