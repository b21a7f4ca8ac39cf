// Mixed-precision hash-grid field on gfx950: FP16 tables, BF16 weights and
// activations on v_mfma_f32_16x16x32_bf16 with FP32 accumulation (weight
// gradients too, with samples on the contraction axis, on 32x32x16 tiles
// where a layer's widths allow),
// FP32 trilinear blending, FP32 table-gradient accumulation.
//
// Operand layouts follow the FP32 kernels (features as rows, 16 samples as
// columns): a 16x16x32 k-step takes 8 consecutive k-slots per lane group,
// filled from two 16-row output tiles of the previous layer (rows 4g..4g+3
// of each), and the weights are laid out for that permutation.
#include "bins.h"
#include "field_common.h"
#include "march_common.h"

namespace nsl {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f4 mfma32(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

typedef float f16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f16v mfma32x32(bf8 a, bf8 b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef short s8v __attribute__((ext_vector_type(8)));

// Two floats as BF16 (round to nearest even), a in the low half; one
// v_cvt_pk_bf16_f32.
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  const bf2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ bf8 pack8(f4 lo, f4 hi) {
  return __builtin_bit_cast(bf8, make_uint4(bf16_pair(lo[0], lo[1]), bf16_pair(lo[2], lo[3]),
                                            bf16_pair(hi[0], hi[1]), bf16_pair(hi[2], hi[3])));
}

// Element u of a as 16 bits.  The whole vector is reinterpreted first: the
// gfx950 compiler lowers a bit cast of one extracted __bf16 element to
// element 0 whatever the index.
__device__ __forceinline__ uint32_t bf_bits(bf8 a, int u) {
  return (uint32_t)(uint16_t)__builtin_bit_cast(s8v, a)[u];
}

// Layout of the BF16 operands (one block = 64 lanes x 8 values per (m, k-step)).
template <class N>
struct Mixed {
  static_assert(N::HD % 32 == 0 && N::HC % 32 == 0, "hidden widths must be multiples of 32");
  static constexpr int BLK = kWave * 8;
  static constexpr int fks(int j) { return j == 0 || j == 2 ? 1 : j == 1 ? N::HD / 32 : N::HC / 32; }
  static constexpr int fsize(int j) { return fks(j) * N::fmt(j) * BLK; }
  static constexpr int foff(int j) {
    int o = 0;
    for (int i = 0; i < j; ++i) o += fsize(i);
    return o;
  }
  static constexpr int FWD = foff(N::NW);
  static constexpr int bks(int j) { return j == N::NW - 1 || j == 1 ? 1 : j == 0 ? N::HD / 32 : N::HC / 32; }
  static constexpr int bsize(int j) { return bks(j) * N::bmt(j) * BLK; }
  static constexpr int boff(int j) {
    int o = 0;
    for (int i = 0; i < j; ++i) o += bsize(i);
    return o;
  }
  static constexpr int BWD = boff(N::NW);
};

// Input feature of forward k-slot (s, lane group g, value u) of layer j; -1 = pad.
template <class N>
__host__ __device__ constexpr int mixed_fwd_feature(int j, int s, int g, int u) {
  if (j == 0) return u < N::NSLOT ? 2 * (g + 4 * (u >> 1)) + (u & 1) : -1;
  if (j == 2) {
    if (u < 4) return 4 * g + u;
    const int k = 4 * g + (u - 4);
    return k < N::NSH ? N::GEO + k : -1;
  }
  return 32 * s + 16 * (u >> 2) + 4 * g + (u & 3);
}

// Output feature consumed by backward k-slot (s, g, u) of layer j; -1 = pad.
template <class N>
__host__ __device__ constexpr int mixed_bwd_kfeature(int j, int s, int g, int u) {
  if (j == N::NW - 1 || j == 1) return u < 4 ? 4 * g + u : -1;
  return 32 * s + 16 * (u >> 2) + 4 * g + (u & 3);
}

// Element idx of the BF16 operand arrays (forward, then backward).
template <class N>
__device__ __forceinline__ void prep_operand(const float* __restrict__ params, const WOffsets& wo,
                                             __bf16* __restrict__ out, int idx) {
  using M = Mixed<N>;
  if (idx >= M::FWD + M::BWD) return;
  float v = 0.0f;
  const bool fwd = idx < M::FWD;
  const int r0 = fwd ? idx : idx - M::FWD;
  int j = 0;
  if (fwd) {
    while (j + 1 < N::NW && r0 >= M::foff(j + 1)) ++j;
  } else {
    while (j + 1 < N::NW && r0 >= M::boff(j + 1)) ++j;
  }
  const int r = r0 - (fwd ? M::foff(j) : M::boff(j));
  const int u = r % 8, lane = (r / 8) % kWave, ms = r / M::BLK;
  const int ks = fwd ? M::fks(j) : M::bks(j);
  const int s = ms % ks, m = ms / ks;
  const int g = lane >> 4, i = lane & 15;
  int row, col;
  if (fwd) {
    row = mixed_fwd_feature<N>(j, s, g, u);
    col = 16 * m + i;
  } else {
    row = bwd_row_feature<N>(j, m, i);
    col = mixed_bwd_kfeature<N>(j, s, g, u);
  }
  if (row >= 0 && col >= 0 && row < N::kin(j) && col < N::kout(j)) v = params[wo.off[j] + row * N::kout(j) + col];
  out[idx] = (__bf16)v;
}

// FP16 copy of the FP32 table (tf floats), eight values [i, i + 8) per
// thread; with g set, the same pass clears the gradient vector from tf
// rounded down to a multiple of 8 up to total.
__device__ __forceinline__ void table_to_half(const float* __restrict__ t, _Float16* __restrict__ h, int64_t tf,
                                              float* __restrict__ g, int64_t total, int64_t i) {
  typedef _Float16 h8 __attribute__((ext_vector_type(8)));
  if (i + 8 <= tf) {
    const float4 a = reinterpret_cast<const float4*>(t + i)[0];
    const float4 b = reinterpret_cast<const float4*>(t + i)[1];
    const h8 o = {(_Float16)a.x, (_Float16)a.y, (_Float16)a.z, (_Float16)a.w,
                  (_Float16)b.x, (_Float16)b.y, (_Float16)b.z, (_Float16)b.w};
    *reinterpret_cast<h8*>(h + i) = o;
  } else {
    for (int64_t k = i; k < tf; ++k) h[k] = (_Float16)t[k];
  }
  if (g && i >= (tf & ~(int64_t)7)) {
    if (i + 8 <= total) {
      reinterpret_cast<float4*>(g + i)[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      reinterpret_cast<float4*>(g + i)[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    } else {
      for (int64_t k = i; k < total; ++k) g[k] = 0.0f;
    }
  }
}

// One launch prepares a mixed-precision step: workgroups [0, tblocks) copy
// the table to FP16 (and clear the gradient tail), the rest lay out the BF16
// weight operands; clear_flag (may be null), the loss-scale overflow flag, is
// reset by the first thread.  Workgroup b of the preparation.
template <class N>
__device__ __forceinline__ void prepare_block(const float* __restrict__ params, const WOffsets& wo,
                                              __bf16* __restrict__ ops, _Float16* __restrict__ t16, int64_t tf,
                                              float* __restrict__ g, int64_t total, int tblocks,
                                              float* __restrict__ clear_flag, int b) {
  if (clear_flag && b == 0 && threadIdx.x == 0) *clear_flag = 0.0f;
  if (b < tblocks)
    table_to_half(params, t16, tf, g, total, ((int64_t)b * 256 + threadIdx.x) * 8);
  else
    prep_operand<N>(params, wo, ops, (b - tblocks) * 256 + (int)threadIdx.x);
}

template <class N>
__global__ __launch_bounds__(256) void mixed_prepare_kernel(const float* __restrict__ params, WOffsets wo,
                                                            __bf16* __restrict__ ops, _Float16* __restrict__ t16,
                                                            int64_t tf, float* __restrict__ g, int64_t total,
                                                            int tblocks, float* __restrict__ clear_flag) {
  prepare_block<N>(params, wo, ops, t16, tf, g, total, tblocks, clear_flag, (int)blockIdx.x);
}

// The step's first launch: workgroups [0, ncount) set up the candidate rays
// and count their samples, the rest prepare the step as above.  The two are
// independent, so the latency-bound marching overlaps the streaming table
// copy instead of following it.
template <class N>
__global__ __launch_bounds__(256) void mixed_prepare_count_kernel(
    const float* __restrict__ params, WOffsets wo, __bf16* __restrict__ ops, _Float16* __restrict__ t16, int64_t tf,
    float* __restrict__ g, int64_t total, int tblocks, float* __restrict__ clear_flag, KeyframeStore kf,
    MarchParams mp, const uint32_t* __restrict__ ids, int n, RayBuffers rb, int ncount) {
  if ((int)blockIdx.x < ncount) {
    march_detail::rays_count_block(kf, mp, ids, n, rb, (int)blockIdx.x);
    return;
  }
  prepare_block<N>(params, wo, ops, t16, tf, g, total, tblocks, clear_flag, (int)blockIdx.x - ncount);
}

template <class N>
__device__ __forceinline__ bf8 lds_bf8(const __bf16* A, int block, int lane) {
  return *reinterpret_cast<const bf8*>(A + (size_t)block * Mixed<N>::BLK + lane * 8);
}

template <class N>
__device__ __forceinline__ void load_bf16(__bf16* dst, const __bf16* __restrict__ src, int n) {
  for (int i = threadIdx.x * 8; i < n; i += blockDim.x * 8)
    *reinterpret_cast<float4*>(dst + i) = *reinterpret_cast<const float4*>(src + i);
}

// ---------------------------------------------------------------------------
// Pieces shared by the forward and backward kernels: the activations of a
// tile (kept by the backward as the BF16 operands the next layer consumed),
// its inputs, and the forward of T tiles interleaved layer by layer.
// ---------------------------------------------------------------------------

template <class N>
struct PActs {
  bf8 e;                   // layer-0 operand: encoding slots (zero beyond NSLOT)
  bf8 h1[N::HD / 32];      // ReLU outputs of layer 0, as layer-1 operands
  f4 o;                    // geometry output, FP32
  bf8 osh;                 // layer-2 operand: geometry rows 4g.., SH 4g..
  bf8 h3[N::HC / 32];
  bf8 h4[N::HC / 32];      // second colour hidden layer (NCH == 2)
  f4 z;                    // colour logits (rows 0..2 in lane group 0)
};

// Inputs of one tile: encoding slots, view direction, upstream gradients.
template <class N>
struct TileIn {
  uint32_t e[N::LPL];      // BF16 pairs of levels g + 4q
  float d[3];
  float ds, dr[3];
};

// acc[r] where the ReLU output (element 4*half + r of p) is positive, else 0.
typedef short s16x2 __attribute__((ext_vector_type(2)));

// ReLU of eight BF16 values on their bits: a BF16 value is below zero exactly
// when its bit pattern is negative as a 16-bit integer (and -0 becomes +0).
// Rounding keeps the sign, so this equals rounding the FP32 ReLU.
__device__ __forceinline__ bf8 relu8(bf8 v) {
  uint4 u = __builtin_bit_cast(uint4, v);
  const s16x2 z = {0, 0};
  u.x = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, u.x), z));
  u.y = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, u.y), z));
  u.z = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, u.z), z));
  u.w = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, u.w), z));
  return __builtin_bit_cast(bf8, u);
}

// The BF16 gradient g where the ReLU output p (bits of a value >= +0) is
// above zero, else 0: the same values as masking in FP32 and rounding after.
// (two packed 16-bit instructions: keep = min(p, 1), g * keep; written out
// because the compiler otherwise selects each half apart, after converting
// each value on its own)
__device__ __forceinline__ uint32_t relu_mask2(uint32_t g, uint32_t p) {
  uint32_t keep, r;
  asm("v_pk_min_u16 %0, %1, %2" : "=v"(keep) : "v"(p), "v"(0x00010001u));
  asm("v_pk_mul_lo_u16 %0, %1, %2" : "=v"(r) : "v"(g), "v"(keep));
  return r;
}
__device__ __forceinline__ bf8 relu_mask8(bf8 g, bf8 p) {
  uint4 a = __builtin_bit_cast(uint4, g);
  const uint4 b = __builtin_bit_cast(uint4, p);
  a.x = relu_mask2(a.x, b.x);
  a.y = relu_mask2(a.y, b.y);
  a.z = relu_mask2(a.z, b.z);
  a.w = relu_mask2(a.w, b.w);
  return __builtin_bit_cast(bf8, a);
}


// Sigmoid through the hardware reciprocal (1 ulp) rather than an IEEE
// division: in the backward the colour gradient it enters is rounded to BF16
// right after, and in the forward it is far below the BF16 network's error.
__device__ __forceinline__ float sigmoid_rcp(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

template <class N, bool KEEP>
__device__ __forceinline__ void fetch_tile(const SampleSrc& src, const _Float16* __restrict__ table,
                                           const LevelInfo& lv, const LaneLevels<N>& ll,
                                           const float* __restrict__ dsigma, const float* __restrict__ drgb, int s,
                                           bool valid, int g, uint32_t ridx, TileIn<N>& in) {
  in.d[0] = 0.0f; in.d[1] = 0.0f; in.d[2] = 1.0f;
  if constexpr (KEEP) {
    const uint32_t* ec = static_cast<const uint32_t*>(src.ecache);
#pragma unroll
    for (int q = 0; q < N::LPL; ++q) in.e[q] = valid ? ec[(size_t)(g + 4 * q) * src.ecache_stride + s] : 0u;
    if (valid) {
      if (src.t) {
        const float4 dd = src.rays[2 * ridx + 1];
        in.d[0] = dd.x; in.d[1] = dd.y; in.d[2] = dd.z;
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) in.d[i] = src.dir[3 * s + i];
      }
    }
  } else {
    float xn[3] = {0.5f, 0.5f, 0.5f};
    if (valid) load_sample(src, s, xn, in.d);
    float e[N::NSLOT];
    encode<N>(table, lv.table_mask, ll, xn, e);
#pragma unroll
    for (int q = 0; q < N::LPL; ++q) in.e[q] = valid ? bf16_pair(e[2 * q], e[2 * q + 1]) : 0u;
  }
  in.ds = 0.0f;
  in.dr[0] = in.dr[1] = in.dr[2] = 0.0f;
  if (dsigma && g == 0 && valid) {
    in.ds = dsigma[s];
#pragma unroll
    for (int r = 0; r < 3; ++r) in.dr[r] = drgb[3 * s + r];
  }
}

template <class N>
__device__ __forceinline__ uint32_t ray_of(const SampleSrc& src, int s, int S) {
  return src.t && s < S ? src.ray[s] : 0u;
}

// K consecutive weight-operand blocks of one layer.
template <class N, int K>
__device__ __forceinline__ void load_ops(const __bf16* A, int lane, bf8 (&w)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) w[k] = lds_bf8<N>(A, k, lane);
}

// Forward of T tiles, interleaved layer by layer; each layer's weight
// operands are read from LDS one layer ahead, so the reads overlap the
// previous layer's MFMAs instead of each waiting in front of its own.
template <class N, int T>
__device__ __forceinline__ void fwd_tiles(const __bf16* __restrict__ Af, int lane, const f4 (&sh)[T],
                                          PActs<N> (&a)[T]) {
  using M = Mixed<N>;
  constexpr f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  constexpr int K3 = N::NCH == 2 ? (N::HC / 16) * (N::HC / 32) : 1;
  bf8 w0[N::HD / 16], w1[N::HD / 32], w2[N::HC / 16], w3[K3], w4[N::HC / 32];
  load_ops<N>(Af + M::foff(0), lane, w0);
  load_ops<N>(Af + M::foff(1), lane, w1);
  {
    f4 h[T][N::HD / 16];
#pragma unroll
    for (int m = 0; m < N::HD / 16; ++m)
#pragma unroll
      for (int t = 0; t < T; ++t) h[t][m] = mfma32(w0[m], a[t].e, zero);
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int s = 0; s < N::HD / 32; ++s) a[t].h1[s] = relu8(pack8(h[t][2 * s], h[t][2 * s + 1]));
  }
  load_ops<N>(Af + M::foff(2), lane, w2);
  {
    f4 acc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = zero;
#pragma unroll
    for (int s = 0; s < N::HD / 32; ++s)
#pragma unroll
      for (int t = 0; t < T; ++t) acc[t] = mfma32(w1[s], a[t].h1[s], acc[t]);
#pragma unroll
    for (int t = 0; t < T; ++t) {
      a[t].o = acc[t];
      a[t].osh = pack8(acc[t], sh[t]);
    }
  }
  if constexpr (N::NCH == 2) load_ops<N>(Af + M::foff(3), lane, w3);
  else load_ops<N>(Af + M::foff(N::NW - 1), lane, w4);
  {
    f4 h[T][N::HC / 16];
#pragma unroll
    for (int m = 0; m < N::HC / 16; ++m)
#pragma unroll
      for (int t = 0; t < T; ++t) h[t][m] = mfma32(w2[m], a[t].osh, zero);
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int s = 0; s < N::HC / 32; ++s) a[t].h3[s] = relu8(pack8(h[t][2 * s], h[t][2 * s + 1]));
  }
  if constexpr (N::NCH == 2) {
    load_ops<N>(Af + M::foff(N::NW - 1), lane, w4);
    f4 acc[T][N::HC / 16];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int m = 0; m < N::HC / 16; ++m) acc[t][m] = zero;
#pragma unroll
    for (int s = 0; s < N::HC / 32; ++s)
#pragma unroll
      for (int m = 0; m < N::HC / 16; ++m)
#pragma unroll
        for (int t = 0; t < T; ++t) acc[t][m] = mfma32(w3[m * (N::HC / 32) + s], a[t].h3[s], acc[t][m]);
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int s = 0; s < N::HC / 32; ++s) a[t].h4[s] = relu8(pack8(acc[t][2 * s], acc[t][2 * s + 1]));
  }
  {
    f4 acc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = zero;
#pragma unroll
    for (int s = 0; s < N::HC / 32; ++s)
#pragma unroll
      for (int t = 0; t < T; ++t) acc[t] = mfma32(w4[s], N::NCH == 2 ? a[t].h4[s] : a[t].h3[s], acc[t]);
#pragma unroll
    for (int t = 0; t < T; ++t) a[t].z = acc[t];
  }
}

// Layer-0 operand (encoding slots, zero beyond NSLOT) and SH coefficients of
// one tile.
template <class N>
__device__ __forceinline__ void tile_operands(const TileIn<N>& in, int g, PActs<N>& a, f4& sh) {
  uint32_t w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) w[q] = q < N::LPL ? in.e[q < N::LPL ? q : 0] : 0u;
  a.e = __builtin_bit_cast(bf8, make_uint4(w[0], w[1], w[2], w[3]));
  float shv[4];
  sh_lane<N>(in.d, g, shv);
  sh = f4{shv[0], shv[1], shv[2], shv[3]};
}

// ---------------------------------------------------------------------------
// Backward, eight waves a workgroup (two per SIMD).  Each wave runs the
// forward recompute and the input-gradient chain of one 16-sample tile; the
// 128 samples of the workgroup's step are staged into a shared
// [feature][sample] buffer, two or one layers at a time (three groups a tile;
// two buffers, used alternately, so one barrier a group suffices), and each
// wave adds the products of its share of the group's weight-gradient tiles
// over the 128 samples.  A wave then holds
// a few weight-gradient tiles instead of all of them, which leaves room for
// two waves on a SIMD.
// ---------------------------------------------------------------------------
constexpr int kBwdWaves8 = 8;
constexpr int kStepSamples = 16 * kBwdWaves8;  // samples of a workgroup step
constexpr int kSRow = kStepSamples + 8;        // bf16 per staged row (the pad staggers rows over the banks)

// The weight-gradient tiles of layer J (16x16, numbered m * NJ + n) go
// round-robin over the waves, continuing from the tiles of the layers that
// come before J in backward order, so that every wave owns about as many.
template <class N, int J>
struct OwnAcc {
  static constexpr int MI = (N::kin(J) + 15) / 16, NJ = (N::kout(J) + 15) / 16, TILES = MI * NJ;
  static constexpr int before() {
    int o = 0;
    for (int i = N::NW - 1; i > J; --i) o += ((N::kin(i) + 15) / 16) * ((N::kout(i) + 15) / 16);
    return o;
  }
  static constexpr int SLOTS = (TILES + kBwdWaves8 - 1) / kBwdWaves8;
  f4 v[SLOTS];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < SLOTS; ++k) v[k] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  // tile of slot k of wave w, or -1
  static __device__ __forceinline__ int tile(int w, int k) {
    const int t = (w - before() % kBwdWaves8 + kBwdWaves8) % kBwdWaves8 + k * kBwdWaves8;
    return t < TILES ? t : -1;
  }
  // v += X^T dY over the staged samples, for the tiles wave w owns
  __device__ __forceinline__ void add(const __bf16* Xs, const __bf16* Ys, int w, int lane) {
    const int gk = lane >> 4, i = lane & 15;
#pragma unroll
    for (int k = 0; k < SLOTS; ++k) {
      const int t = tile(w, k);
      if (t < 0) continue;
      const int m = t / NJ, n = t % NJ;
      const __bf16* xr = Xs + (16 * m + i) * kSRow + 8 * gk;
      const __bf16* yr = Ys + (16 * n + i) * kSRow + 8 * gk;
#pragma unroll
      for (int c = 0; c < kStepSamples / 32; ++c)
        v[k] = mfma32(*reinterpret_cast<const bf8*>(xr + 32 * c), *reinterpret_cast<const bf8*>(yr + 32 * c), v[k]);
    }
  }
  static constexpr int SPLIT = 1;
  // dW (LDS, row-major kin x kout, zeroed) += the owned tiles (disjoint over
  // the waves, so all waves write at once, in phase 0)
  __device__ __forceinline__ void flush(float* dW, int w, int lane, int phase) const {
    if (phase != 0) return;
    const int gk = lane >> 4, i = lane & 15;
#pragma unroll
    for (int k = 0; k < SLOTS; ++k) {
      const int t = tile(w, k);
      if (t < 0) continue;
      const int m = t / NJ, n = t % NJ, col = 16 * n + i;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * m + 4 * gk + r;
        if (row < N::kin(J) && col < N::kout(J)) dW[row * N::kout(J) + col] += v[k][r];
      }
    }
  }
};

// The weight-gradient products of a layer whose input and output widths are
// multiples of 32, on 32x32x16 tiles: each tile goes to kBwdWaves8 / TILES
// waves, each of which adds the products over its own share of the staged
// samples (the operand reads per product are half those of 16x16 tiles).
template <class N, int J>
struct OwnAcc32 {
  static constexpr int MI = N::kin(J) / 32, NJ = N::kout(J) / 32, TILES = MI * NJ;
  static constexpr int SPLIT = kBwdWaves8 / TILES, KSTEPS = kStepSamples / SPLIT / 16;
  f16v v;
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = 0.0f;
  }
  __device__ __forceinline__ void add(const __bf16* Xs, const __bf16* Ys, int w, int lane) {
    const int t = w % TILES, sp = w / TILES, m = t / NJ, n = t % NJ;
    const int i = lane & 31, c0 = sp * (kStepSamples / SPLIT) + 8 * (lane >> 5);
    const __bf16* xr = Xs + (32 * m + i) * kSRow + c0;
    const __bf16* yr = Ys + (32 * n + i) * kSRow + c0;
#pragma unroll
    for (int c = 0; c < KSTEPS; ++c)
      v = mfma32x32(*reinterpret_cast<const bf8*>(xr + 16 * c), *reinterpret_cast<const bf8*>(yr + 16 * c), v);
  }
  // dW += this wave's partial tile; the waves sharing a tile write in
  // different phases
  __device__ __forceinline__ void flush(float* dW, int w, int lane, int phase) const {
    const int t = w % TILES, sp = w / TILES, m = t / NJ, n = t % NJ;
    if (sp != phase) return;
    const int col = 32 * n + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 32 * m + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      dW[row * N::kout(J) + col] += v[r];
    }
  }
};

template <class N, int J>
constexpr bool kWideTiles = N::kin(J) % 32 == 0 && N::kout(J) % 32 == 0 &&
                            kBwdWaves8 % ((N::kin(J) / 32) * (N::kout(J) / 32)) == 0;
template <class N, int J>
using LayerAcc = typename std::conditional<kWideTiles<N, J>, OwnAcc32<N, J>, OwnAcc<N, J>>::type;

template <class N>
struct OwnAll {
  LayerAcc<N, 0> w0;
  LayerAcc<N, 1> w1;
  LayerAcc<N, 2> w2;
  LayerAcc<N, N::NCH == 2 ? 3 : 2> w3;  // second colour hidden layer (unused with one)
  LayerAcc<N, N::NW - 1> wl;
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int PHASES =
      cmax(cmax(LayerAcc<N, 0>::SPLIT, LayerAcc<N, 1>::SPLIT),
           cmax(cmax(LayerAcc<N, 2>::SPLIT, LayerAcc<N, N::NCH == 2 ? 3 : 2>::SPLIT), LayerAcc<N, N::NW - 1>::SPLIT));
};

// One tile's staged values: rows 16m + 4g + r of column c (lane group g).
template <int MB>
__device__ __forceinline__ void stage1_packed(uint16_t* S, const bf8* a, int g, int c) {
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) S[(16 * m + 4 * g + r) * kSRow + c] = (uint16_t)bf_bits(a[m >> 1], 4 * (m & 1) + r);
}

// dL/de of one tile held back one step, stored after the next tile's
// forward; as BF16 pairs (the table-gradient records it feeds are BF16 too).
template <class N>
struct PendingDe1 {
  f4 de[N::bmt(0)];
  int s;
  bool valid;
  __device__ __forceinline__ void store(const RecordBuffers& rec, int g) const {
    if (!valid) return;
#pragma unroll
    for (int q = 0; q < N::LPL; ++q) {
      const int k0 = 2 * q, k1 = 2 * q + 1;
      reinterpret_cast<uint32_t*>(rec.de)[(size_t)(g + 4 * q) * rec.stride + s] =
          bf16_pair(de[k0 >> 2][k0 & 3], de[k1 >> 2][k1 & 3]);
    }
  }
};

// Staging groups: the layers whose weight-gradient products follow one
// barrier together (the colour layers; the geometry-feature layer and the
// second density layer; the first density layer).  Within a group each layer
// has its X rows (16 per input tile) and then its dY rows (16 per output
// tile), layers in backward order; a buffer holds the largest group.
template <class N>
struct StageRows {
  static constexpr int xr(int j) { return (N::kin(j) + 15) / 16 * 16; }
  static constexpr int yr(int j) { return (N::kout(j) + 15) / 16 * 16; }
  static constexpr int group(int j) { return j >= 3 || j == N::NW - 1 ? 0 : j >= 1 ? 1 : 2; }
  static constexpr int x(int j) {
    int o = 0;
    for (int i = N::NW - 1; i > j; --i)
      if (group(i) == group(j)) o += xr(i) + yr(i);
    return o;
  }
  static constexpr int y(int j) { return x(j) + xr(j); }
  static constexpr int rows(int gr) {
    int o = 0;
    for (int i = 0; i < N::NW; ++i)
      if (group(i) == gr) o += xr(i) + yr(i);
    return o;
  }
  static constexpr int ROWS = N::cmax(rows(0), N::cmax(rows(1), rows(2)));
};

// Row r of staging buffer b.
template <class N>
__device__ __forceinline__ __bf16* srow(__bf16* stage, int b, int r) {
  return stage + (b * StageRows<N>::ROWS + r) * kSRow;
}
template <class N>
__device__ __forceinline__ uint16_t* srow16(__bf16* stage, int b, int r) {
  return reinterpret_cast<uint16_t*>(srow<N>(stage, b, r));
}

// Forward recompute, backward chain and dL/de of this wave's tile (samples
// s = 128 p + 16 w + jc), with the workgroup's weight-gradient products of
// each staging group in between; the previous tile's dL/de (pend) is stored after the
// forward and replaced by this tile's.
template <class N>
__device__ __forceinline__ void bwd_tile8(const __bf16* __restrict__ Af, const __bf16* __restrict__ Ab,
                                          __bf16* stage, int& buf, const TileIn<N>& in, int s, bool valid,
                                          const RecordBuffers& rec, OwnAll<N>& dw, PendingDe1<N>& pend, int w,
                                          int lane) {
  using M = Mixed<N>;
  constexpr f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  const int g = lane >> 4, jc = lane & 15, c = 16 * w + jc;
  PActs<N> a[1];
  f4 sh[1];
  tile_operands<N>(in, g, a[0], sh[0]);
  fwd_tiles<N, 1>(Af, lane, sh, a);
  pend.store(rec, g);

  f4 dz = zero;
  if (g == 0) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const float cc = sigmoid_rcp(a[0].z[r]);
      dz[r] = in.dr[r] * cc * (1.0f - cc);
    }
  }
  constexpr int K3 = N::NCH == 2 ? (N::HC / 16) * (N::HC / 32) : 1;
  constexpr int MT0 = N::bmt(0);
  bf8 w4[N::HC / 16], w3[K3], w2[N::HC / 32], w1[N::HD / 16], w0[MT0 * (N::HD / 32)];
  using SR = StageRows<N>;
  load_ops<N>(Ab + M::boff(N::NW - 1), lane, w4);
  const bf8* hl = N::NCH == 2 ? a[0].h4 : a[0].h3;
  // colour layers: the last one, then (with two) the second hidden one
  // the hidden-layer gradients are used only as BF16 (MFMA operands and
  // staged values), so they are rounded once and masked on their bits
  bf8 dhl[N::HC / 32];
  const bf8 dzp = pack8(dz, zero);
  {
    f4 raw[N::HC / 16];
#pragma unroll
    for (int m = 0; m < N::HC / 16; ++m) raw[m] = mfma32(w4[m], dzp, zero);
#pragma unroll
    for (int k = 0; k < N::HC / 32; ++k) dhl[k] = relu_mask8(pack8(raw[2 * k], raw[2 * k + 1]), hl[k]);
  }
  if constexpr (N::NCH == 2) load_ops<N>(Ab + M::boff(3), lane, w3);
  else load_ops<N>(Ab + M::boff(2), lane, w2);
  stage1_packed<N::HC / 16>(srow16<N>(stage, buf, SR::x(N::NW - 1)), hl, g, c);
  stage1_packed<1>(srow16<N>(stage, buf, SR::y(N::NW - 1)), &dzp, g, c);
  bf8 dh3[N::HC / 32];
  if constexpr (N::NCH == 2) {
    f4 acc[N::HC / 16];
#pragma unroll
    for (int m = 0; m < N::HC / 16; ++m) acc[m] = zero;
#pragma unroll
    for (int k = 0; k < N::HC / 32; ++k)
#pragma unroll
      for (int m = 0; m < N::HC / 16; ++m) acc[m] = mfma32(w3[m * (N::HC / 32) + k], dhl[k], acc[m]);
#pragma unroll
    for (int k = 0; k < N::HC / 32; ++k) dh3[k] = relu_mask8(pack8(acc[2 * k], acc[2 * k + 1]), a[0].h3[k]);
    load_ops<N>(Ab + M::boff(2), lane, w2);
    stage1_packed<N::HC / 16>(srow16<N>(stage, buf, SR::x(3)), a[0].h3, g, c);
    stage1_packed<N::HC / 16>(srow16<N>(stage, buf, SR::y(3)), dhl, g, c);
  } else {
#pragma unroll
    for (int k = 0; k < N::HC / 32; ++k) dh3[k] = dhl[k];
  }
  __syncthreads();
  dw.wl.add(srow<N>(stage, buf, SR::x(N::NW - 1)), srow<N>(stage, buf, SR::y(N::NW - 1)), w, lane);
  if constexpr (N::NCH == 2) dw.w3.add(srow<N>(stage, buf, SR::x(3)), srow<N>(stage, buf, SR::y(3)), w, lane);
  buf ^= 1;
  // first colour layer (gradient of the geometry features), second density layer
  f4 dgeo = zero;
#pragma unroll
  for (int k = 0; k < N::HC / 32; ++k) dgeo = mfma32(w2[k], dh3[k], dgeo);
  load_ops<N>(Ab + M::boff(1), lane, w1);
  stage1_packed<2>(srow16<N>(stage, buf, SR::x(2)), &a[0].osh, g, c);
  stage1_packed<N::HC / 16>(srow16<N>(stage, buf, SR::y(2)), dh3, g, c);
  if (g == 0) dgeo[0] += __expf(a[0].o[0]) * in.ds;  // rounded to BF16 next
  bf8 dh1[N::HD / 32];
  const bf8 dgp = pack8(dgeo, zero);
  {
    f4 raw[N::HD / 16];
#pragma unroll
    for (int m = 0; m < N::HD / 16; ++m) raw[m] = mfma32(w1[m], dgp, zero);
#pragma unroll
    for (int k = 0; k < N::HD / 32; ++k) dh1[k] = relu_mask8(pack8(raw[2 * k], raw[2 * k + 1]), a[0].h1[k]);
  }
  load_ops<N>(Ab + M::boff(0), lane, w0);
  stage1_packed<N::HD / 16>(srow16<N>(stage, buf, SR::x(1)), a[0].h1, g, c);
  stage1_packed<1>(srow16<N>(stage, buf, SR::y(1)), &dgp, g, c);
  __syncthreads();
  dw.w2.add(srow<N>(stage, buf, SR::x(2)), srow<N>(stage, buf, SR::y(2)), w, lane);
  dw.w1.add(srow<N>(stage, buf, SR::x(1)), srow<N>(stage, buf, SR::y(1)), w, lane);
  buf ^= 1;
  // first density layer: dL/de
  f4 de[MT0];
#pragma unroll
  for (int m = 0; m < MT0; ++m) de[m] = zero;
#pragma unroll
  for (int k = 0; k < N::HD / 32; ++k)
#pragma unroll
    for (int m = 0; m < MT0; ++m) de[m] = mfma32(w0[m * (N::HD / 32) + k], dh1[k], de[m]);
  {
    uint16_t* X = srow16<N>(stage, buf, SR::x(0));
#pragma unroll
    for (int k = 0; k < N::NSLOT; ++k) X[fwd_in_feature<N>(0, k, g) * kSRow + c] = (uint16_t)bf_bits(a[0].e, k);
    if constexpr (N::ENC < 16) {
#pragma unroll
      for (int k = 0; k < 2; ++k) X[(N::ENC + 2 * g + k) * kSRow + c] = 0;
    }
  }
  stage1_packed<N::HD / 16>(srow16<N>(stage, buf, SR::y(0)), dh1, g, c);
  __syncthreads();
  dw.w0.add(srow<N>(stage, buf, SR::x(0)), srow<N>(stage, buf, SR::y(0)), w, lane);
  buf ^= 1;
  pend.s = s;
  pend.valid = valid;
#pragma unroll
  for (int m = 0; m < MT0; ++m) pend.de[m] = de[m];
}

// kBwdWaves8 waves per workgroup, two per SIMD; the workgroup takes steps
// (128 samples) blockIdx.x, blockIdx.x + gridDim.x, ...  With the kept
// encoding, a wave fetches its next tile's inputs while it computes the
// current one (ray indices two steps ahead).
template <class N>
__global__ __launch_bounds__(kBwdWaves8 * kWave, 1) void mixed_bwd8_kernel(
    LevelInfo lv, const _Float16* __restrict__ table, const __bf16* __restrict__ prep, SampleSrc src,
    const float* __restrict__ dsigma, const float* __restrict__ drgb, RecordBuffers rec,
    float* __restrict__ dw_partial) {
  using M = Mixed<N>;
  constexpr int SBUF = StageRows<N>::ROWS * kSRow;
  static_assert(2 * SBUF * (int)sizeof(__bf16) >= N::NWEIGHTS * (int)sizeof(float),
                "the weight-gradient sums reuse the staging buffers");
  __shared__ __attribute__((aligned(16))) __bf16 Af[M::FWD];
  __shared__ __attribute__((aligned(16))) __bf16 Ab[M::BWD];
  __shared__ __attribute__((aligned(16))) __bf16 stage[2 * SBUF];
  load_bf16<N>(Af, prep, M::FWD);
  load_bf16<N>(Ab, prep + M::FWD, M::BWD);
  __syncthreads();

  const int S = src.n_dev ? (int)*src.n_dev : src.n;
  const int w = threadIdx.x / kWave, lane = lane_id(), g = lane >> 4, jc = lane & 15;
  OwnAll<N> dw;
  dw.w0.zero(); dw.w1.zero(); dw.w2.zero(); dw.wl.zero();
  if constexpr (N::NCH == 2) dw.w3.zero();
  LaneLevels<N> ll;
  lane_levels<N>(lv, g, ll);
  PendingDe1<N> pend;
  pend.valid = false;
  pend.s = 0;
  int buf = 0;
  const int nsteps = (S + kStepSamples - 1) / kStepSamples, step = gridDim.x;
  const int off = 16 * w + jc;
  if (src.ecache) {
    const int p0 = blockIdx.x;
    TileIn<N> cur;
    const int s0 = kStepSamples * p0 + off;
    fetch_tile<N, true>(src, table, lv, ll, dsigma, drgb, s0, s0 < S, g, ray_of<N>(src, s0, S), cur);
    uint32_t rid1 = ray_of<N>(src, kStepSamples * (p0 + step) + off, S);
    for (int p = p0; p < nsteps; p += step) {
      const int s = kStepSamples * p + off;
      TileIn<N> nxt;
      const int s1 = s + kStepSamples * step;
      fetch_tile<N, true>(src, table, lv, ll, dsigma, drgb, s1, s1 < S, g, rid1, nxt);
      const uint32_t rid2 = ray_of<N>(src, s1 + kStepSamples * step, S);
      bwd_tile8<N>(Af, Ab, stage, buf, cur, s, s < S, rec, dw, pend, w, lane);
      cur = nxt;
      rid1 = rid2;
    }
  } else {
    for (int p = blockIdx.x; p < nsteps; p += step) {
      const int s = kStepSamples * p + off;
      TileIn<N> cur;
      fetch_tile<N, false>(src, table, lv, ll, dsigma, drgb, s, s < S, g, 0u, cur);
      bwd_tile8<N>(Af, Ab, stage, buf, cur, s, s < S, rec, dw, pend, w, lane);
    }
  }
  pend.store(rec, g);
  // the workgroup's weight-gradient sums, in the staging space
  __syncthreads();
  float* dW = reinterpret_cast<float*>(stage);
  for (int i = threadIdx.x; i < N::NWEIGHTS; i += blockDim.x) dW[i] = 0.0f;
  __syncthreads();
  for (int ph = 0; ph < OwnAll<N>::PHASES; ++ph) {
    dw.w0.flush(dW + N::woff(0), w, lane, ph);
    dw.w1.flush(dW + N::woff(1), w, lane, ph);
    dw.w2.flush(dW + N::woff(2), w, lane, ph);
    if constexpr (N::NCH == 2) dw.w3.flush(dW + N::woff(3), w, lane, ph);
    dw.wl.flush(dW + N::woff(N::NW - 1), w, lane, ph);
    __syncthreads();
  }
  float* out = dw_partial + (size_t)blockIdx.x * N::NWEIGHTS;
  for (int i = threadIdx.x; i < N::NWEIGHTS; i += blockDim.x) out[i] = dW[i];
}

// Forward: density and colour of 16-sample tiles, one tile per wave at a
// time (four waves per SIMD stay resident, which hides latency better than
// pairing tiles here; the register budget is held to four waves, without
// which the compiler takes 136 registers, three waves, and the fixed grid
// needs a second round).  The grid is a fixed number of workgroups, so the
// weight operands are staged into LDS once per workgroup rather than once per
// four tiles; with the kept encoding, a wave fetches its next tile's inputs
// while it computes the current one (ray indices two tiles ahead).
constexpr int kMixedFwdGrid = 1024;

template <class N>
__device__ __forceinline__ void fwd_store(const PActs<N>& a, int g, int s, bool valid, float* __restrict__ sigma_out,
                                          float* __restrict__ rgb_out) {
  if (g == 0 && valid) {
    sigma_out[s] = expf(a.o[0]);
    rgb_out[3 * s + 0] = sigmoid_rcp(a.z[0]);
    rgb_out[3 * s + 1] = sigmoid_rcp(a.z[1]);
    rgb_out[3 * s + 2] = sigmoid_rcp(a.z[2]);
  }
}

//
// Workgroups past the MLP's (bp.nbins of them) run the table-gradient column
// scan (bins.h), which needs only the record counts of the encoding.
template <class N>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void mixed_fwd_kernel(
    LevelInfo lv, const _Float16* __restrict__ table, const __bf16* __restrict__ prep, SampleSrc src,
    float* __restrict__ sigma_out, float* __restrict__ rgb_out, BinPrep bp) {
  using M = Mixed<N>;
  const int G = (int)gridDim.x - bp.nbins;  // the MLP's workgroups
  if ((int)blockIdx.x >= G) {
    colscan_bin(bp.rb, bp.nunits, (int)blockIdx.x - G);
    return;
  }
  __shared__ __attribute__((aligned(16))) __bf16 Af[M::FWD];
  load_bf16<N>(Af, prep, M::FWD);
  __syncthreads();
  const int S = src.n_dev ? (int)*src.n_dev : src.n;
  const int ntiles = (S + 15) / 16;
  const int lane = lane_id(), g = lane >> 4, jc = lane & 15;
  const int first = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  const int step = G * (blockDim.x / kWave);
  if (first >= ntiles) return;
  LaneLevels<N> ll;
  lane_levels<N>(lv, g, ll);
  if (src.ecache) {
    TileIn<N> cur;
    const int s0 = 16 * first + jc;
    fetch_tile<N, true>(src, table, lv, ll, nullptr, nullptr, s0, s0 < S, g, ray_of<N>(src, s0, S), cur);
    uint32_t rid1 = ray_of<N>(src, 16 * (first + step) + jc, S);
    for (int tile = first; tile < ntiles; tile += step) {
      const int s = 16 * tile + jc, s1 = s + 16 * step;
      TileIn<N> nxt;
      fetch_tile<N, true>(src, table, lv, ll, nullptr, nullptr, s1, s1 < S, g, rid1, nxt);
      rid1 = ray_of<N>(src, s1 + 16 * step, S);
      PActs<N> a[1];
      f4 sh[1];
      tile_operands<N>(cur, g, a[0], sh[0]);
      fwd_tiles<N, 1>(Af, lane, sh, a);
      fwd_store<N>(a[0], g, s, s < S, sigma_out, rgb_out);
      cur = nxt;
    }
  } else {
    for (int tile = first; tile < ntiles; tile += step) {
      const int s = 16 * tile + jc;
      TileIn<N> in;
      fetch_tile<N, false>(src, table, lv, ll, nullptr, nullptr, s, s < S, g, 0u, in);
      PActs<N> a[1];
      f4 sh[1];
      tile_operands<N>(in, g, a[0], sh[0]);
      fwd_tiles<N, 1>(Af, lane, sh, a);
      fwd_store<N>(a[0], g, s, s < S, sigma_out, rgb_out);
    }
  }
}

// ---------------------------------------------------------------------------
// Host launchers.  Shadow buffer: BF16 operands (forward, then backward),
// padded to 256 bytes, then the FP16 table (same entry layout as FP32).
// ---------------------------------------------------------------------------

template <class N>
constexpr size_t mixed_ops_bytes() {
  return ((size_t)(Mixed<N>::FWD + Mixed<N>::BWD) * 2 + 255) / 256 * 256;
}

size_t mixed_shadow_bytes(int shape, int64_t table_floats) {
  const size_t ops = shape == kShapeTiny ? mixed_ops_bytes<NetTiny>() : mixed_ops_bytes<NetFull>();
  return ops + ((size_t)table_floats * 2 + 255) / 256 * 256;
}

// With kf set, the same launch also sets up the n candidate rays and counts
// their samples.
template <class N>
static hipError_t prep_impl(const float* params, const WOffsets& wo, int64_t table_floats, void* shadow,
                            float* zero_grads, int64_t total, float* clear_flag, const KeyframeStore* kf,
                            const MarchParams* mp, const uint32_t* ids, int n, const RayBuffers* rb,
                            hipStream_t st) {
  using M = Mixed<N>;
  const int nops = M::FWD + M::BWD;
  _Float16* t16 = reinterpret_cast<_Float16*>(static_cast<char*>(shadow) + mixed_ops_bytes<N>());
  const int64_t span = zero_grads && total > table_floats ? total : table_floats;
  const int tblocks = (int)((span + 2047) / 2048);
  const int oblocks = (nops + 255) / 256;
  if (kf) {
    const int ncount = (int)march_block_count(n);
    hipLaunchKernelGGL(mixed_prepare_count_kernel<N>, dim3(ncount + tblocks + oblocks), dim3(256), 0, st, params,
                       wo, static_cast<__bf16*>(shadow), t16, table_floats, zero_grads, total, tblocks, clear_flag,
                       *kf, *mp, ids, n, *rb, ncount);
  } else {
    hipLaunchKernelGGL(mixed_prepare_kernel<N>, dim3(tblocks + oblocks), dim3(256), 0, st, params, wo,
                       static_cast<__bf16*>(shadow), t16, table_floats, zero_grads, total, tblocks, clear_flag);
  }
  return hipGetLastError();
}

template <class N>
static hipError_t fwd_impl(const LevelInfo& lv, const void* shadow, const SampleSrc& src, int max_samples,
                           float* sigma, float* rgb, hipStream_t st, const BinPrep* bp) {
  const int tiles = (max_samples + 15) / 16;
  const __bf16* ops = static_cast<const __bf16*>(shadow);
  const _Float16* t16 = reinterpret_cast<const _Float16*>(static_cast<const char*>(shadow) + mixed_ops_bytes<N>());
  const int grid = (tiles + 3) / 4 < kMixedFwdGrid ? (tiles + 3) / 4 : kMixedFwdGrid;
  const BinPrep none{};
  const BinPrep& b = bp ? *bp : none;
  if (grid + b.nbins > 0)
    hipLaunchKernelGGL(mixed_fwd_kernel<N>, dim3(grid + b.nbins), dim3(256), 0, st, lv, t16, ops, src, sigma, rgb,
                       b);
  return hipGetLastError();
}

template <class N>
static hipError_t bwd_impl(const LevelInfo& lv, const void* shadow, const SampleSrc& src, int nblocks,
                           const float* dsigma, const float* drgb, const RecordBuffers& rec, float* partial,
                           const WOffsets& wo, float* grads, hipStream_t st) {
  const __bf16* ops = static_cast<const __bf16*>(shadow);
  const _Float16* t16 = reinterpret_cast<const _Float16*>(static_cast<const char*>(shadow) + mixed_ops_bytes<N>());
  hipLaunchKernelGGL(mixed_bwd8_kernel<N>, dim3(nblocks), dim3(kBwdWaves8 * kWave), 0, st, lv, t16, ops, src,
                     dsigma, drgb, rec, partial);
  return hipGetLastError();
}

template <class N>
static hipError_t encode_impl(const LevelInfo& lv, const void* shadow, const SampleSrc& src, int max_samples,
                              uint32_t* hist, const BinLevels& bl, hipStream_t st) {
  const _Float16* t16 = reinterpret_cast<const _Float16*>(static_cast<const char*>(shadow) + mixed_ops_bytes<N>());
  const int grid = encode_grid<N>(max_samples);
  if (grid > 0)
    hipLaunchKernelGGL((encode_levels_kernel<N, _Float16, uint32_t>), dim3(grid), dim3(256), 0, st, lv, t16, src,
                       static_cast<uint32_t*>(src.ecache), src.ecache_stride, hist, bl);
  return hipGetLastError();
}

hipError_t mixed_encode(int shape, const LevelInfo& lv, const void* shadow, const SampleSrc& src, int max_samples,
                        uint32_t* hist, const BinLevels& bl, hipStream_t st) {
  return shape == kShapeTiny ? encode_impl<NetTiny>(lv, shadow, src, max_samples, hist, bl, st)
                             : encode_impl<NetFull>(lv, shadow, src, max_samples, hist, bl, st);
}

hipError_t mixed_prepare(int shape, const float* params, const WOffsets& wo, int64_t table_floats, void* shadow,
                         float* zero_grads, int64_t total, float* clear_flag, hipStream_t st) {
  return shape == kShapeTiny ? prep_impl<NetTiny>(params, wo, table_floats, shadow, zero_grads, total, clear_flag,
                                                   nullptr, nullptr, nullptr, 0, nullptr, st)
                             : prep_impl<NetFull>(params, wo, table_floats, shadow, zero_grads, total, clear_flag,
                                                   nullptr, nullptr, nullptr, 0, nullptr, st);
}

hipError_t mixed_prepare_count(int shape, const float* params, const WOffsets& wo, int64_t table_floats,
                               void* shadow, float* zero_grads, int64_t total, float* clear_flag,
                               const KeyframeStore& kf, const MarchParams& mp, const uint32_t* ids, int n,
                               const RayBuffers& rb, hipStream_t st) {
  return shape == kShapeTiny ? prep_impl<NetTiny>(params, wo, table_floats, shadow, zero_grads, total, clear_flag,
                                                   &kf, &mp, ids, n, &rb, st)
                             : prep_impl<NetFull>(params, wo, table_floats, shadow, zero_grads, total, clear_flag,
                                                   &kf, &mp, ids, n, &rb, st);
}

hipError_t mixed_forward(int shape, const LevelInfo& lv, const void* shadow, const SampleSrc& src, int max_samples,
                         float* sigma, float* rgb, hipStream_t st, const BinPrep* bp) {
  return shape == kShapeTiny ? fwd_impl<NetTiny>(lv, shadow, src, max_samples, sigma, rgb, st, bp)
                             : fwd_impl<NetFull>(lv, shadow, src, max_samples, sigma, rgb, st, bp);
}

hipError_t mixed_backward(int shape, const LevelInfo& lv, const void* shadow, const SampleSrc& src, int nblocks,
                          const float* dsigma, const float* drgb, const RecordBuffers& rec, float* partial,
                          const WOffsets& wo, float* grads, hipStream_t st) {
  return shape == kShapeTiny
             ? bwd_impl<NetTiny>(lv, shadow, src, nblocks, dsigma, drgb, rec, partial, wo, grads, st)
             : bwd_impl<NetFull>(lv, shadow, src, nblocks, dsigma, drgb, rec, partial, wo, grads, st);
}

}  // namespace nsl
