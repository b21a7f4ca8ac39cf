// Mixed-precision hash-grid field on gfx950: FP16 tables, BF16 weights and
// activations on v_mfma_f32_16x16x32_bf16 with FP32 accumulation, weight
// gradients on v_mfma_f32_16x16x16_bf16 (samples on the contraction axis),
// FP32 trilinear blending, FP32 table-gradient accumulation.
//
// Operand layouts follow the FP32 kernels (features as rows, 16 samples as
// columns): a 16x16x32 k-step takes 8 consecutive k-slots per lane group,
// filled from two 16-row output tiles of the previous layer (rows 4g..4g+3
// of each), and the weights are laid out for that permutation.
#include "field_common.h"

namespace nsl {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma32(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf8 pack8(f4 lo, f4 hi) {
  bf8 r;
  r[0] = (__bf16)lo[0]; r[1] = (__bf16)lo[1]; r[2] = (__bf16)lo[2]; r[3] = (__bf16)lo[3];
  r[4] = (__bf16)hi[0]; r[5] = (__bf16)hi[1]; r[6] = (__bf16)hi[2]; r[7] = (__bf16)hi[3];
  return r;
}

__device__ __forceinline__ short bf16_bits(float x) {
  const __bf16 b = (__bf16)x;
  return __builtin_bit_cast(short, b);
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
  static constexpr int SROW = 20;  // bf16 per staged row (16 samples + pad)
  static constexpr int STAGE = (N::XROWS + N::YROWS) * SROW;
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

template <class N>
__global__ void mixed_prep_kernel(const float* __restrict__ params, WOffsets wo, __bf16* __restrict__ out) {
  using M = Mixed<N>;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
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

__global__ void table_to_half_kernel(const float* __restrict__ t, _Float16* __restrict__ h, int64_t n2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n2) return;
  const float2 v = reinterpret_cast<const float2*>(t)[i];
  h2 o;
  o[0] = (_Float16)v.x;
  o[1] = (_Float16)v.y;
  reinterpret_cast<h2*>(h)[i] = o;
}

template <class N>
struct MActs {
  float e[N::NSLOT];
  f4 h1[N::HD / 16];
  f4 o;
  float sh[4];
  f4 h3[N::HC / 16];
  f4 h4[N::HC / 16];
  f4 z;
};

template <class N>
__device__ __forceinline__ bf8 lds_bf8(const __bf16* A, int block, int lane) {
  return *reinterpret_cast<const bf8*>(A + (size_t)block * Mixed<N>::BLK + lane * 8);
}

template <class N>
__device__ __forceinline__ void mlp_fwd_mixed(const __bf16* __restrict__ Af, int lane, MActs<N>& a) {
  using M = Mixed<N>;
  constexpr f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  {
    bf8 b;
#pragma unroll
    for (int u = 0; u < 8; ++u) b[u] = (__bf16)(u < N::NSLOT ? a.e[u < N::NSLOT ? u : 0] : 0.0f);
    const __bf16* A = Af + M::foff(0);
#pragma unroll
    for (int m = 0; m < N::HD / 16; ++m) a.h1[m] = relu4(mfma32(lds_bf8<N>(A, m, lane), b, zero));
  }
  {
    const __bf16* A = Af + M::foff(1);
    f4 acc = zero;
#pragma unroll
    for (int s = 0; s < N::HD / 32; ++s) acc = mfma32(lds_bf8<N>(A, s, lane), pack8(a.h1[2 * s], a.h1[2 * s + 1]), acc);
    a.o = acc;
  }
  {
    const f4 shv = {a.sh[0], a.sh[1], a.sh[2], a.sh[3]};
    const bf8 b = pack8(a.o, shv);
    const __bf16* A = Af + M::foff(2);
#pragma unroll
    for (int m = 0; m < N::HC / 16; ++m) a.h3[m] = relu4(mfma32(lds_bf8<N>(A, m, lane), b, zero));
  }
  const f4* hl = a.h3;
  if constexpr (N::NCH == 2) {
    const __bf16* A = Af + M::foff(3);
    f4 acc[N::HC / 16];
#pragma unroll
    for (int m = 0; m < N::HC / 16; ++m) acc[m] = zero;
#pragma unroll
    for (int s = 0; s < N::HC / 32; ++s) {
      const bf8 b = pack8(a.h3[2 * s], a.h3[2 * s + 1]);
#pragma unroll
      for (int m = 0; m < N::HC / 16; ++m) acc[m] = mfma32(lds_bf8<N>(A, m * (N::HC / 32) + s, lane), b, acc[m]);
    }
#pragma unroll
    for (int m = 0; m < N::HC / 16; ++m) a.h4[m] = relu4(acc[m]);
    hl = a.h4;
  }
  {
    const __bf16* A = Af + M::foff(N::NW - 1);
    f4 acc = zero;
#pragma unroll
    for (int s = 0; s < N::HC / 32; ++s) acc = mfma32(lds_bf8<N>(A, s, lane), pack8(hl[2 * s], hl[2 * s + 1]), acc);
    a.z = acc;
  }
}

template <class N>
__device__ __forceinline__ void load_bf16(__bf16* dst, const __bf16* __restrict__ src, int n) {
  for (int i = threadIdx.x * 8; i < n; i += blockDim.x * 8)
    *reinterpret_cast<float4*>(dst + i) = *reinterpret_cast<const float4*>(src + i);
}

template <class N>
__global__ __launch_bounds__(256) void mixed_fwd_kernel(LevelInfo lv, const _Float16* __restrict__ table,
                                                        const __bf16* __restrict__ prep, SampleSrc src,
                                                        float* __restrict__ sigma_out, float* __restrict__ rgb_out) {
  using M = Mixed<N>;
  __shared__ __attribute__((aligned(16))) __bf16 Af[M::FWD];
  load_bf16<N>(Af, prep, M::FWD);
  __syncthreads();
  const int S = src.n_dev ? (int)*src.n_dev : src.n;
  const int lane = lane_id(), g = lane >> 4, jc = lane & 15;
  const int tile = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  const int s = tile * 16 + jc;
  if (tile * 16 >= S) return;
  const bool valid = s < S;
  LaneLevels<N> ll;
  lane_levels<N>(lv, g, ll);
  MActs<N> act;
  float xn[3] = {0.5f, 0.5f, 0.5f}, d[3] = {0.0f, 0.0f, 1.0f};
  if (valid) load_sample(src, s, xn, d);
  if (src.ecache)
    read_encoding<N>(static_cast<const uint32_t*>(src.ecache), src.ecache_stride, g, s, valid, act.e);
  else
    encode<N>(table, lv.table_mask, ll, xn, act.e);
  sh_lane<N>(d, g, act.sh);
  mlp_fwd_mixed<N>(Af, lane, act);
  if (g == 0 && valid) {
    sigma_out[s] = expf(act.o[0]);
    rgb_out[3 * s + 0] = sigmoidf(act.z[0]);
    rgb_out[3 * s + 1] = sigmoidf(act.z[1]);
    rgb_out[3 * s + 2] = sigmoidf(act.z[2]);
  }
}

// Stage a D-layout block as bf16 rows [feature][sample].
template <class N, int TILES>
__device__ __forceinline__ void stage_bf(__bf16* S, const f4* v, int g, int jc) {
#pragma unroll
  for (int m = 0; m < TILES; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) S[(16 * m + 4 * g + r) * Mixed<N>::SROW + jc] = (__bf16)v[m][r];
}

template <class N, int KIN, int KOUT>
__device__ __forceinline__ void dw_mixed(const __bf16* Xs, const __bf16* Ys, DWAcc<KIN, KOUT>& acc, int lane) {
  constexpr int MI = DWAcc<KIN, KOUT>::MI, NJ = DWAcc<KIN, KOUT>::NJ, SR = Mixed<N>::SROW;
  const int gk = lane >> 4, i = lane & 15;
  s4 xa[MI], yb[NJ];
#pragma unroll
  for (int m = 0; m < MI; ++m) xa[m] = *reinterpret_cast<const s4*>(Xs + (16 * m + i) * SR + 4 * gk);
#pragma unroll
  for (int n = 0; n < NJ; ++n) yb[n] = *reinterpret_cast<const s4*>(Ys + (16 * n + i) * SR + 4 * gk);
#pragma unroll
  for (int m = 0; m < MI; ++m)
#pragma unroll
    for (int n = 0; n < NJ; ++n) acc.v[m * NJ + n] = mfma16(xa[m], yb[n], acc.v[m * NJ + n]);
}

// kMixedBwdWaves waves per workgroup, one per SIMD: the weight-gradient
// accumulators of a wave live in registers for the whole kernel.
template <class N>
__global__ __launch_bounds__(kMixedBwdWaves * kWave, 1) void mixed_bwd_kernel(LevelInfo lv, const _Float16* __restrict__ table,
                                                           const __bf16* __restrict__ prep, SampleSrc src,
                                                           const float* __restrict__ dsigma,
                                                           const float* __restrict__ drgb, RecordBuffers rec,
                                                           float* __restrict__ dw_partial) {
  using M = Mixed<N>;
  __shared__ __attribute__((aligned(16))) __bf16 Af[M::FWD];
  __shared__ __attribute__((aligned(16))) __bf16 Ab[M::BWD];
  __shared__ __attribute__((aligned(16))) float dW[N::NWEIGHTS];
  __shared__ __attribute__((aligned(16))) __bf16 stage_all[kMixedBwdWaves * M::STAGE];
  load_bf16<N>(Af, prep, M::FWD);
  load_bf16<N>(Ab, prep + M::FWD, M::BWD);
  for (int i = threadIdx.x; i < N::NWEIGHTS; i += blockDim.x) dW[i] = 0.0f;
  __syncthreads();

  const int S = src.n_dev ? (int)*src.n_dev : src.n;
  const int ntiles = (S + 15) / 16;
  const int wave = threadIdx.x / kWave;
  const int lane = lane_id(), g = lane >> 4, jc = lane & 15;
  __bf16* Xs = stage_all + wave * M::STAGE;
  __bf16* Ys = Xs + N::XROWS * M::SROW;
  LaneLevels<N> ll;
  lane_levels<N>(lv, g, ll);
  constexpr f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  const int region = blockIdx.x * kMixedBwdWaves + wave;
  DWAcc<N::ENC, N::HD> dw0;
  DWAcc<N::HD, 16> dw1;
  DWAcc<N::CIN, N::HC> dw2;
  DWAcc<N::HC, N::HC> dw3;  // second colour hidden layer (unused with one)
  DWAcc<N::HC, 3> dwl;
  dw0.zero(); dw1.zero(); dw2.zero(); dwl.zero();
  if constexpr (N::NCH == 2) dw3.zero();

  for (int tile = region; tile < ntiles; tile += gridDim.x * kMixedBwdWaves) {
    const int s = tile * 16 + jc;
    const bool valid = s < S;
    float xn[3] = {0.5f, 0.5f, 0.5f}, d[3] = {0.0f, 0.0f, 1.0f};
    if (valid) load_sample(src, s, xn, d);
    MActs<N> act;
    if (src.ecache) {
      read_encoding<N>(static_cast<const uint32_t*>(src.ecache), src.ecache_stride, g, s, valid, act.e);
    } else {
      encode<N>(table, lv.table_mask, ll, xn, act.e);
      if (!valid) {
#pragma unroll
        for (int k = 0; k < N::NSLOT; ++k) act.e[k] = 0.0f;
      }
    }
    sh_lane<N>(d, g, act.sh);
    mlp_fwd_mixed<N>(Af, lane, act);

    float ds = 0.0f;
    f4 dz = zero;
    if (g == 0 && valid) {
      ds = dsigma[s];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const float c = sigmoidf(act.z[r]);
        dz[r] = drgb[3 * s + r] * c * (1.0f - c);
      }
    }
    const f4* hl = (N::NCH == 2) ? act.h4 : act.h3;
    f4 dhl[N::HC / 16];
    {
      const bf8 b = pack8(dz, zero);
      const __bf16* A = Ab + M::boff(N::NW - 1);
#pragma unroll
      for (int m = 0; m < N::HC / 16; ++m) {
        f4 acc = mfma32(lds_bf8<N>(A, m, lane), b, zero);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = hl[m][r] > 0.0f ? acc[r] : 0.0f;
        dhl[m] = acc;
      }
    }
    stage_bf<N, N::HC / 16>(Xs, hl, g, jc);
    stage_bf<N, 1>(Ys, &dz, g, jc);
    wave_lds_fence();
    dw_mixed<N, N::HC, 3>(Xs, Ys, dwl, lane);
    wave_lds_fence();

    f4 dh3[N::HC / 16];
    if constexpr (N::NCH == 2) {
      const __bf16* A = Ab + M::boff(3);
      f4 acc[N::HC / 16];
#pragma unroll
      for (int m = 0; m < N::HC / 16; ++m) acc[m] = zero;
#pragma unroll
      for (int k = 0; k < N::HC / 32; ++k) {
        const bf8 b = pack8(dhl[2 * k], dhl[2 * k + 1]);
#pragma unroll
        for (int m = 0; m < N::HC / 16; ++m) acc[m] = mfma32(lds_bf8<N>(A, m * (N::HC / 32) + k, lane), b, acc[m]);
      }
#pragma unroll
      for (int m = 0; m < N::HC / 16; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[m][r] = act.h3[m][r] > 0.0f ? acc[m][r] : 0.0f;
        dh3[m] = acc[m];
      }
      stage_bf<N, N::HC / 16>(Xs, act.h3, g, jc);
      stage_bf<N, N::HC / 16>(Ys, dhl, g, jc);
      wave_lds_fence();
      dw_mixed<N, N::HC, N::HC>(Xs, Ys, dw3, lane);
      wave_lds_fence();
    } else {
#pragma unroll
      for (int m = 0; m < N::HC / 16; ++m) dh3[m] = dhl[m];
    }
    f4 dgeo = zero;
    {
      const __bf16* A = Ab + M::boff(2);
#pragma unroll
      for (int k = 0; k < N::HC / 32; ++k) dgeo = mfma32(lds_bf8<N>(A, k, lane), pack8(dh3[2 * k], dh3[2 * k + 1]), dgeo);
    }
    stage_bf<N, 1>(Xs, &act.o, g, jc);
#pragma unroll
    for (int r = 0; r < 4; ++r) Xs[(16 + 4 * g + r) * M::SROW + jc] = (__bf16)act.sh[r];
    stage_bf<N, N::HC / 16>(Ys, dh3, g, jc);
    wave_lds_fence();
    dw_mixed<N, N::CIN, N::HC>(Xs, Ys, dw2, lane);
    wave_lds_fence();
    if (g == 0) dgeo[0] += expf(act.o[0]) * ds;
    f4 dh1[N::HD / 16];
    {
      const bf8 b = pack8(dgeo, zero);
      const __bf16* A = Ab + M::boff(1);
#pragma unroll
      for (int m = 0; m < N::HD / 16; ++m) {
        f4 acc = mfma32(lds_bf8<N>(A, m, lane), b, zero);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = act.h1[m][r] > 0.0f ? acc[r] : 0.0f;
        dh1[m] = acc;
      }
    }
    stage_bf<N, N::HD / 16>(Xs, act.h1, g, jc);
    stage_bf<N, 1>(Ys, &dgeo, g, jc);
    wave_lds_fence();
    dw_mixed<N, N::HD, 16>(Xs, Ys, dw1, lane);
    wave_lds_fence();
    constexpr int MT0 = N::bmt(0);
    f4 de[MT0];
    {
      const __bf16* A = Ab + M::boff(0);
#pragma unroll
      for (int m = 0; m < MT0; ++m) de[m] = zero;
#pragma unroll
      for (int k = 0; k < N::HD / 32; ++k) {
        const bf8 b = pack8(dh1[2 * k], dh1[2 * k + 1]);
#pragma unroll
        for (int m = 0; m < MT0; ++m) de[m] = mfma32(lds_bf8<N>(A, m * (N::HD / 32) + k, lane), b, de[m]);
      }
    }
#pragma unroll
    for (int k = 0; k < N::NSLOT; ++k) Xs[fwd_in_feature<N>(0, k, g) * M::SROW + jc] = (__bf16)act.e[k];
    if constexpr (N::ENC < 16) {
#pragma unroll
      for (int k = 0; k < 2; ++k) Xs[(N::ENC + 2 * g + k) * M::SROW + jc] = (__bf16)0.0f;
    }
    stage_bf<N, N::HD / 16>(Ys, dh1, g, jc);
    wave_lds_fence();
    dw_mixed<N, N::ENC, N::HD>(Xs, Ys, dw0, lane);
    wave_lds_fence();
    // dL/de of this lane's levels g + 4q, level-major: the 16 lanes of a row
    // store 16 consecutive samples of one level
    if (valid) {
#pragma unroll
      for (int q = 0; q < N::LPL; ++q) {
        const int k0 = 2 * q, k1 = 2 * q + 1;
        rec.de[(size_t)(g + 4 * q) * rec.stride + s] = make_float2(de[k0 >> 2][k0 & 3], de[k1 >> 2][k1 & 3]);
      }
    }
  }
  for (int w = 0; w < kMixedBwdWaves; ++w) {
    __syncthreads();
    if (wave == w) {
      dw0.flush(dW + N::woff(0), lane);
      dw1.flush(dW + N::woff(1), lane);
      dw2.flush(dW + N::woff(2), lane);
      if constexpr (N::NCH == 2) dw3.flush(dW + N::woff(3), lane);
      dwl.flush(dW + N::woff(N::NW - 1), lane);
    }
  }
  __syncthreads();
  float* out = dw_partial + (size_t)blockIdx.x * N::NWEIGHTS;
  for (int i = threadIdx.x; i < N::NWEIGHTS; i += blockDim.x) out[i] = dW[i];
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

template <class N>
static hipError_t prep_impl(const float* params, const WOffsets& wo, int64_t table_floats, void* shadow,
                            hipStream_t st) {
  using M = Mixed<N>;
  const int n = M::FWD + M::BWD;
  hipLaunchKernelGGL(mixed_prep_kernel<N>, dim3((n + 255) / 256), dim3(256), 0, st, params, wo,
                     static_cast<__bf16*>(shadow));
  _Float16* t16 = reinterpret_cast<_Float16*>(static_cast<char*>(shadow) + mixed_ops_bytes<N>());
  const int64_t n2 = table_floats / 2;
  if (n2 > 0)
    hipLaunchKernelGGL(table_to_half_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, params, t16, n2);
  return hipGetLastError();
}

template <class N>
static hipError_t fwd_impl(const LevelInfo& lv, const void* shadow, const SampleSrc& src, int max_samples,
                           float* sigma, float* rgb, hipStream_t st) {
  const int tiles = (max_samples + 15) / 16;
  if (tiles == 0) return hipSuccess;
  const __bf16* ops = static_cast<const __bf16*>(shadow);
  const _Float16* t16 = reinterpret_cast<const _Float16*>(static_cast<const char*>(shadow) + mixed_ops_bytes<N>());
  hipLaunchKernelGGL(mixed_fwd_kernel<N>, dim3((tiles + 3) / 4), dim3(256), 0, st, lv, t16, ops, src, sigma, rgb);
  return hipGetLastError();
}

template <class N>
static hipError_t bwd_impl(const LevelInfo& lv, const void* shadow, const SampleSrc& src, int nblocks,
                           const float* dsigma, const float* drgb, const RecordBuffers& rec, float* partial,
                           const WOffsets& wo, float* grads, hipStream_t st) {
  const __bf16* ops = static_cast<const __bf16*>(shadow);
  const _Float16* t16 = reinterpret_cast<const _Float16*>(static_cast<const char*>(shadow) + mixed_ops_bytes<N>());
  hipLaunchKernelGGL(mixed_bwd_kernel<N>, dim3(nblocks), dim3(kMixedBwdWaves * kWave), 0, st, lv, t16, ops, src,
                     dsigma, drgb, rec, partial);
  return hipGetLastError();
}

template <class N>
static hipError_t encode_impl(const LevelInfo& lv, const void* shadow, const SampleSrc& src, int max_samples,
                              hipStream_t st) {
  const _Float16* t16 = reinterpret_cast<const _Float16*>(static_cast<const char*>(shadow) + mixed_ops_bytes<N>());
  const int grid = encode_grid<N>(max_samples);
  if (grid > 0)
    hipLaunchKernelGGL((encode_levels_kernel<N, _Float16, uint32_t>), dim3(grid), dim3(256), 0, st, lv, t16, src,
                       static_cast<uint32_t*>(src.ecache), src.ecache_stride);
  return hipGetLastError();
}

hipError_t mixed_encode(int shape, const LevelInfo& lv, const void* shadow, const SampleSrc& src, int max_samples,
                        hipStream_t st) {
  return shape == kShapeTiny ? encode_impl<NetTiny>(lv, shadow, src, max_samples, st)
                             : encode_impl<NetFull>(lv, shadow, src, max_samples, st);
}

hipError_t mixed_prepare(int shape, const float* params, const WOffsets& wo, int64_t table_floats, void* shadow,
                         hipStream_t st) {
  return shape == kShapeTiny ? prep_impl<NetTiny>(params, wo, table_floats, shadow, st)
                             : prep_impl<NetFull>(params, wo, table_floats, shadow, st);
}

hipError_t mixed_forward(int shape, const LevelInfo& lv, const void* shadow, const SampleSrc& src, int max_samples,
                         float* sigma, float* rgb, hipStream_t st) {
  return shape == kShapeTiny ? fwd_impl<NetTiny>(lv, shadow, src, max_samples, sigma, rgb, st)
                             : fwd_impl<NetFull>(lv, shadow, src, max_samples, sigma, rgb, st);
}

hipError_t mixed_backward(int shape, const LevelInfo& lv, const void* shadow, const SampleSrc& src, int nblocks,
                          const float* dsigma, const float* drgb, const RecordBuffers& rec, float* partial,
                          const WOffsets& wo, float* grads, hipStream_t st) {
  return shape == kShapeTiny
             ? bwd_impl<NetTiny>(lv, shadow, src, nblocks, dsigma, drgb, rec, partial, wo, grads, st)
             : bwd_impl<NetFull>(lv, shadow, src, nblocks, dsigma, drgb, rec, partial, wo, grads, st);
}

}  // namespace nsl
