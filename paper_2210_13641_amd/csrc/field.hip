// Hash-grid field on gfx950: fused encode + density/colour MLP forward, and
// the recompute adjoint (encode, MLP forward again, MLP backward with
// weight gradients, scatter into the table gradient).
//
// One wave evaluates 16 samples: lane (g, j) = (lane/16, lane%16) gathers
// levels g, g+4, ... of sample j, which are exactly its B-operand slots of
// the first MFMA layer (net.h).  Nothing but sigma and colour leaves the
// forward kernel; the backward kernel re-derives every activation from the
// sample position instead of reading stored activations.
#include "bins.h"
#include "field_common.h"

namespace nsl {

// ---------------------------------------------------------------------------
// MLP forward (activations kept for the adjoint)
// ---------------------------------------------------------------------------

template <class N>
struct Acts {
  float e[N::NSLOT];
  f4 h1[N::HD / 16];
  f4 o;
  float sh[4];
  f4 h3[N::HC / 16];
  f4 h4[N::HC / 16];
  f4 z;
};

template <class N>
__device__ __forceinline__ void mlp_fwd(const float* __restrict__ Af, int lane, Acts<N>& a) {
  constexpr f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  // layer 0: encoding -> h1
  {
    const float* A = Af + N::foff(0) + lane;
    f4 acc[N::HD / 16];
#pragma unroll
    for (int m = 0; m < N::HD / 16; ++m) acc[m] = zero;
#pragma unroll
    for (int s = 0; s < N::fks(0); ++s)
#pragma unroll
      for (int m = 0; m < N::HD / 16; ++m) acc[m] = mfma4(A[(m * N::fks(0) + s) * kWave], a.e[s], acc[m]);
#pragma unroll
    for (int m = 0; m < N::HD / 16; ++m) a.h1[m] = relu4(acc[m]);
  }
  // layer 1: h1 -> o (geometry, 16)
  {
    const float* A = Af + N::foff(1) + lane;
    f4 acc = zero;
#pragma unroll
    for (int s = 0; s < N::fks(1); ++s) acc = mfma4(A[s * kWave], a.h1[s >> 2][s & 3], acc);
    a.o = acc;
  }
  // layer 2: [o, sh] -> h3
  {
    const float* A = Af + N::foff(2) + lane;
    f4 acc[N::HC / 16];
#pragma unroll
    for (int m = 0; m < N::HC / 16; ++m) acc[m] = zero;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const float b = s < 4 ? a.o[s & 3] : a.sh[s & 3];
#pragma unroll
      for (int m = 0; m < N::HC / 16; ++m) acc[m] = mfma4(A[(m * 8 + s) * kWave], b, acc[m]);
    }
#pragma unroll
    for (int m = 0; m < N::HC / 16; ++m) a.h3[m] = relu4(acc[m]);
  }
  const f4* hl = a.h3;
  if constexpr (N::NCH == 2) {
    const float* A = Af + N::foff(3) + lane;
    f4 acc[N::HC / 16];
#pragma unroll
    for (int m = 0; m < N::HC / 16; ++m) acc[m] = zero;
#pragma unroll
    for (int s = 0; s < N::HC / 4; ++s)
#pragma unroll
      for (int m = 0; m < N::HC / 16; ++m)
        acc[m] = mfma4(A[(m * (N::HC / 4) + s) * kWave], a.h3[s >> 2][s & 3], acc[m]);
#pragma unroll
    for (int m = 0; m < N::HC / 16; ++m) a.h4[m] = relu4(acc[m]);
    hl = a.h4;
  }
  // last layer -> z (rows 0..2 valid, held by lane group 0)
  {
    const float* A = Af + N::foff(N::NW - 1) + lane;
    f4 acc = zero;
#pragma unroll
    for (int s = 0; s < N::HC / 4; ++s) acc = mfma4(A[s * kWave], hl[s >> 2][s & 3], acc);
    a.z = acc;
  }
}

// ---------------------------------------------------------------------------
// Weight-operand preparation (once per step from the FP32 parameters)
// ---------------------------------------------------------------------------

template <class N>
__global__ void prep_weights_kernel(const float* __restrict__ params, WOffsets wo,
                                    float* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N::FWD_FLOATS + N::BWD_FLOATS) return;
  float v = 0.0f;
  if (idx < N::FWD_FLOATS) {
    int j = 0;
    while (j + 1 < N::NW && idx >= N::foff(j + 1)) ++j;
    const int r = idx - N::foff(j);
    const int lane = r % kWave, ms = r / kWave;
    const int s = ms % N::fks(j), m = ms / N::fks(j);
    const int g = lane >> 4, i = lane & 15;
    const int row = fwd_in_feature<N>(j, s, g), col = 16 * m + i;
    if (row >= 0 && row < N::kin(j) && col < N::kout(j)) v = params[wo.off[j] + row * N::kout(j) + col];
  } else {
    const int b = idx - N::FWD_FLOATS;
    int j = 0;
    while (j + 1 < N::NW && b >= N::boff(j + 1)) ++j;
    const int r = b - N::boff(j);
    const int lane = r % kWave, ms = r / kWave;
    const int s = ms % N::bks(j), m = ms / N::bks(j);
    const int g = lane >> 4, i = lane & 15;
    const int row = bwd_row_feature<N>(j, m, i), col = bwd_k_feature<N>(j, s, g);
    if (row >= 0 && row < N::kin(j) && col < N::kout(j)) v = params[wo.off[j] + row * N::kout(j) + col];
  }
  out[idx] = v;
}

// ---------------------------------------------------------------------------
// Forward: sigma and colour per sample
// ---------------------------------------------------------------------------

// Inputs of one sample for the MLP from the kept encoding: this lane's
// encoding slots and the ray direction (ray index ridx, fetched earlier).
template <class N>
__device__ __forceinline__ void fetch_kept(const SampleSrc& src, int g, int s, bool valid, uint32_t ridx,
                                           float e[N::NSLOT], float d[3]) {
  read_encoding<N>(static_cast<const float2*>(src.ecache), src.ecache_stride, g, s, valid, e);
  d[0] = 0.0f; d[1] = 0.0f; d[2] = 1.0f;
  if (valid) {
    if (src.t) {
      const float4 dd = src.rays[2 * ridx + 1];
      d[0] = dd.x; d[1] = dd.y; d[2] = dd.z;
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i) d[i] = src.dir[3 * s + i];
    }
  }
}

template <class N>
__device__ __forceinline__ void fwd_tile_out(const float* Af, int lane, int g, int s, bool valid, Acts<N>& act,
                                             const float d[3], float* __restrict__ sigma_out,
                                             float* __restrict__ rgb_out) {
  sh_lane<N>(d, g, act.sh);
  mlp_fwd<N>(Af, lane, act);
  if (g == 0 && valid) {
    sigma_out[s] = __expf(act.o[0]) ;
    rgb_out[3 * s + 0] = sigmoidf(act.z[0]);
    rgb_out[3 * s + 1] = sigmoidf(act.z[1]);
    rgb_out[3 * s + 2] = sigmoidf(act.z[2]);
  }
}

// Forward of 16-sample tiles, one per wave at a time, on a fixed grid (the
// weight operands are staged into LDS once per workgroup); with the kept
// encoding a wave fetches its next tile's inputs while it computes the
// current one (ray indices two tiles ahead).
constexpr int kFieldFwdGrid = 768;
constexpr bool kFieldFwdPrefetch = true;

// Workgroups past the MLP's (bp.nbins of them) run the table-gradient column
// scan (bins.h), which needs only the record counts of the encoding.
template <class N>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void field_fwd_kernel(FieldArgs a, SampleSrc src,
                                                        float* __restrict__ sigma_out,
                                                        float* __restrict__ rgb_out, BinPrep bp) {
  const int G = (int)gridDim.x - bp.nbins;  // the MLP's workgroups
  if ((int)blockIdx.x >= G) {
    colscan_bin(bp.rb, bp.nunits, (int)blockIdx.x - G);
    return;
  }
  __shared__ __attribute__((aligned(16))) float Af[N::FWD_FLOATS];
  load_operands<N>(Af, a.wprep, N::FWD_FLOATS);
  __syncthreads();
  const int S = src.n_dev ? (int)*src.n_dev : src.n;
  const int ntiles = (S + 15) / 16;
  const int lane = lane_id(), g = lane >> 4, jc = lane & 15;
  const int first = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  const int step = G * (blockDim.x / kWave);
  if (first >= ntiles) return;
  if (kFieldFwdPrefetch && src.ecache) {
    auto rid = [&](int s) -> uint32_t { return src.t && s < S ? src.ray[s] : 0u; };
    float e[N::NSLOT], d[3];
    const int s0 = 16 * first + jc;
    fetch_kept<N>(src, g, s0, s0 < S, rid(s0), e, d);
    uint32_t rid1 = rid(s0 + 16 * step);
    for (int tile = first; tile < ntiles; tile += step) {
      const int s = 16 * tile + jc, s1 = s + 16 * step;
      float en[N::NSLOT], dn[3];
      fetch_kept<N>(src, g, s1, s1 < S, rid1, en, dn);
      rid1 = rid(s1 + 16 * step);
      Acts<N> act;
#pragma unroll
      for (int k = 0; k < N::NSLOT; ++k) act.e[k] = e[k];
      fwd_tile_out<N>(Af, lane, g, s, s < S, act, d, sigma_out, rgb_out);
#pragma unroll
      for (int k = 0; k < N::NSLOT; ++k) e[k] = en[k];
#pragma unroll
      for (int i = 0; i < 3; ++i) d[i] = dn[i];
    }
  } else {
    LaneLevels<N> ll;
    lane_levels<N>(a.lv, g, ll);
    for (int tile = first; tile < ntiles; tile += step) {
      const int s = 16 * tile + jc;
      const bool valid = s < S;
      Acts<N> act;
      float xn[3] = {0.5f, 0.5f, 0.5f}, d[3] = {0.0f, 0.0f, 1.0f};
      if (valid) load_sample(src, s, xn, d);
      if (src.ecache)
        read_encoding<N>(static_cast<const float2*>(src.ecache), src.ecache_stride, g, s, valid, act.e);
      else
        encode<N>(a.table, a.lv.table_mask, ll, xn, act.e);
      fwd_tile_out<N>(Af, lane, g, s, valid, act, d, sigma_out, rgb_out);
    }
  }
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------

// acc[in][out] += sum over the wave's 16 samples of X[in] * dY[out], with X
// and dY staged [feature][sample] (stride SROW) in this wave's LDS area.
template <class N, int KIN, int KOUT>
__device__ __forceinline__ void dw_accumulate(const float* Xs, const float* Ys, DWAcc<KIN, KOUT>& acc, int lane) {
  constexpr int MI = DWAcc<KIN, KOUT>::MI, NJ = DWAcc<KIN, KOUT>::NJ;
  const int gk = lane >> 4, i = lane & 15;
  f4 xa[MI], yb[NJ];
#pragma unroll
  for (int m = 0; m < MI; ++m) xa[m] = *reinterpret_cast<const f4*>(Xs + (16 * m + i) * N::SROW + 4 * gk);
#pragma unroll
  for (int n = 0; n < NJ; ++n) yb[n] = *reinterpret_cast<const f4*>(Ys + (16 * n + i) * N::SROW + 4 * gk);
#pragma unroll
  for (int m = 0; m < MI; ++m)
#pragma unroll
    for (int n = 0; n < NJ; ++n)
#pragma unroll
      for (int s = 0; s < 4; ++s) acc.v[m * NJ + n] = mfma4(xa[m][s], yb[n][s], acc.v[m * NJ + n]);
}

// Stage a D-layout activation block (tiles of 16 rows) as rows [row0, ...).
template <class N, int TILES>
__device__ __forceinline__ void stage_d(float* S, const f4* v, int g, int jc) {
#pragma unroll
  for (int m = 0; m < TILES; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) S[(16 * m + 4 * g + r) * N::SROW + jc] = v[m][r];
}

template <class N>
__global__ __launch_bounds__(kFieldBwdWaves * kWave, 1) void field_bwd_kernel(FieldArgs a, SampleSrc src,
                                                           const float* __restrict__ dsigma,
                                                           const float* __restrict__ drgb, RecordBuffers rec,
                                                           float* __restrict__ dw_partial) {
  __shared__ __attribute__((aligned(16))) float Af[N::FWD_FLOATS];
  __shared__ __attribute__((aligned(16))) float Ab[N::BWD_FLOATS];
  __shared__ __attribute__((aligned(16))) float dW[N::NWEIGHTS];
  __shared__ __attribute__((aligned(16))) float stage_all[kFieldBwdWaves * N::STAGE_FLOATS];
  load_operands<N>(Af, a.wprep, N::FWD_FLOATS);
  load_operands<N>(Ab, a.wprep + N::FWD_FLOATS, N::BWD_FLOATS);
  for (int i = threadIdx.x; i < N::NWEIGHTS; i += blockDim.x) dW[i] = 0.0f;
  __syncthreads();

  const int S = src.n_dev ? (int)*src.n_dev : src.n;
  const int ntiles = (S + 15) / 16;
  const int wave = threadIdx.x / kWave;
  const int lane = lane_id(), g = lane >> 4, jc = lane & 15;
  float* Xs = stage_all + wave * N::STAGE_FLOATS;
  float* Ys = Xs + N::XROWS * N::SROW;
  LaneLevels<N> ll;
  lane_levels<N>(a.lv, g, ll);
  constexpr f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  const int region = blockIdx.x * kFieldBwdWaves + wave;
  // weight gradients of the wave, summed over its tiles in registers
  DWAcc<N::ENC, N::HD> dw0;
  DWAcc<N::HD, 16> dw1;
  DWAcc<N::CIN, N::HC> dw2;
  DWAcc<N::HC, N::HC> dw3;  // second colour hidden layer (unused with one)
  DWAcc<N::HC, 3> dwl;
  dw0.zero(); dw1.zero(); dw2.zero(); dwl.zero();
  if constexpr (N::NCH == 2) dw3.zero();

  for (int tile = region; tile < ntiles; tile += gridDim.x * kFieldBwdWaves) {
    const int s = tile * 16 + jc;
    const bool valid = s < S;
    float xn[3] = {0.5f, 0.5f, 0.5f}, d[3] = {0.0f, 0.0f, 1.0f};
    if (valid) {
      if (src.ecache)
        load_direction(src, s, d);  // the position is not needed with the encoding given
      else
        load_sample(src, s, xn, d);
    }
    Acts<N> act;
    if (src.ecache) {
      read_encoding<N>(static_cast<const float2*>(src.ecache), src.ecache_stride, g, s, valid, act.e);
    } else {
      encode<N>(a.table, a.lv.table_mask, ll, xn, act.e);
      if (!valid) {
#pragma unroll
        for (int k = 0; k < N::NSLOT; ++k) act.e[k] = 0.0f;
      }
    }
    sh_lane<N>(d, g, act.sh);
    mlp_fwd<N>(Af, lane, act);

    // seeds: dz = dc * c (1 - c) and dsigma, on lane group 0
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
    // last layer: dh_last = W_last dz, masked
    const f4* hl = (N::NCH == 2) ? act.h4 : act.h3;
    f4 dhl[N::HC / 16];
    {
      const float* A = Ab + N::boff(N::NW - 1) + lane;
#pragma unroll
      for (int m = 0; m < N::HC / 16; ++m) {
        f4 acc = zero;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc = mfma4(A[(m * 3 + k) * kWave], dz[k], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = hl[m][r] > 0.0f ? acc[r] : 0.0f;
        dhl[m] = acc;
      }
    }
    // dW of the last layer
    stage_d<N, N::HC / 16>(Xs, hl, g, jc);
    stage_d<N, 1>(Ys, &dz, g, jc);
    wave_lds_fence();
    dw_accumulate<N, N::HC, 3>(Xs, Ys, dwl, lane);
    wave_lds_fence();

    f4 dh3[N::HC / 16];
    if constexpr (N::NCH == 2) {
      const float* A = Ab + N::boff(3) + lane;
#pragma unroll
      for (int m = 0; m < N::HC / 16; ++m) {
        f4 acc = zero;
#pragma unroll
        for (int k = 0; k < N::HC / 4; ++k) acc = mfma4(A[(m * (N::HC / 4) + k) * kWave], dhl[k >> 2][k & 3], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = act.h3[m][r] > 0.0f ? acc[r] : 0.0f;
        dh3[m] = acc;
      }
      stage_d<N, N::HC / 16>(Xs, act.h3, g, jc);
      stage_d<N, N::HC / 16>(Ys, dhl, g, jc);
      wave_lds_fence();
      dw_accumulate<N, N::HC, N::HC>(Xs, Ys, dw3, lane);
      wave_lds_fence();
    } else {
#pragma unroll
      for (int m = 0; m < N::HC / 16; ++m) dh3[m] = dhl[m];
    }
    // colour input layer: d(geo) = W3[geo rows] dh3; dW3 with X = [o, sh]
    f4 dgeo = zero;
    {
      const float* A = Ab + N::boff(2) + lane;
#pragma unroll
      for (int k = 0; k < N::HC / 4; ++k) dgeo = mfma4(A[k * kWave], dh3[k >> 2][k & 3], dgeo);
    }
    stage_d<N, 1>(Xs, &act.o, g, jc);
#pragma unroll
    for (int r = 0; r < 4; ++r) Xs[(16 + 4 * g + r) * N::SROW + jc] = act.sh[r];
    stage_d<N, N::HC / 16>(Ys, dh3, g, jc);
    wave_lds_fence();
    dw_accumulate<N, N::CIN, N::HC>(Xs, Ys, dw2, lane);
    wave_lds_fence();
    // density output: do = dgeo, do_0 += sigma * dsigma
    if (g == 0) dgeo[0] += __expf(act.o[0]) * ds;
    f4 dh1[N::HD / 16];
    {
      const float* A = Ab + N::boff(1) + lane;
#pragma unroll
      for (int m = 0; m < N::HD / 16; ++m) {
        f4 acc = zero;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc = mfma4(A[(m * 4 + k) * kWave], dgeo[k], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = act.h1[m][r] > 0.0f ? acc[r] : 0.0f;
        dh1[m] = acc;
      }
    }
    stage_d<N, N::HD / 16>(Xs, act.h1, g, jc);
    stage_d<N, 1>(Ys, &dgeo, g, jc);
    wave_lds_fence();
    dw_accumulate<N, N::HD, 16>(Xs, Ys, dw1, lane);
    wave_lds_fence();
    // encoding gradient: de = W1 dh1 (rows = this lane group's slots)
    constexpr int MT0 = N::bmt(0);
    f4 de[MT0];
    {
      const float* A = Ab + N::boff(0) + lane;
#pragma unroll
      for (int m = 0; m < MT0; ++m) {
        f4 acc = zero;
#pragma unroll
        for (int k = 0; k < N::HD / 4; ++k) acc = mfma4(A[(m * (N::HD / 4) + k) * kWave], dh1[k >> 2][k & 3], acc);
        de[m] = acc;
      }
    }
    // dW1 with X = e (slots -> features)
#pragma unroll
    for (int k = 0; k < N::NSLOT; ++k) Xs[fwd_in_feature<N>(0, k, g) * N::SROW + jc] = act.e[k];
    if constexpr (N::ENC < 16) {
#pragma unroll
      for (int k = 0; k < 2; ++k) Xs[(N::ENC + 2 * g + k) * N::SROW + jc] = 0.0f;
    }
    stage_d<N, N::HD / 16>(Ys, dh1, g, jc);
    wave_lds_fence();
    dw_accumulate<N, N::ENC, N::HD>(Xs, Ys, dw0, lane);
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
  // workgroup sum of the weight gradients: waves add in turn (no atomics)
  for (int w = 0; w < kFieldBwdWaves; ++w) {
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
// Fused rendering: one wave per ray, 16 consecutive samples of the ray per
// MFMA tile, compositing by a row scan of the 16 sample lanes, and an early
// exit once the transmittance left for the ray is below stop_T.
// ---------------------------------------------------------------------------

// The weight and t of every composited sample wait in LDS (per wave, the
// samples of its current ray) for the second pass of V*, so a ray may take up
// to kRenderMaxSamples samples.
template <class N>
__global__ __launch_bounds__(256) void render_kernel(LevelInfo lv, Aabb box, const nsl_render_request* __restrict__ reqs,
                                                     int n_req, const nsl_render_tile* __restrict__ tiles,
                                                     RenderParams rp) {
  __shared__ __attribute__((aligned(16))) float Af[N::FWD_FLOATS];
  extern __shared__ float2 wt_lds[];  // [4 waves][16 * ntiles] (w, t), written by the lanes of row 0
  nsl_render_tile tile;
  if (tiles) {
    tile = tiles[blockIdx.x];
  } else {
    tile.request = 0;
    tile.first_pixel = blockIdx.x * NSL_RENDER_TILE;
    tile.n_pixels = NSL_RENDER_TILE;
  }
  if (tile.request < 0 || tile.request >= n_req) return;
  const nsl_render_request& rq = reqs[tile.request];
  const int npix = rq.H * rq.W;
  const int first = max(tile.first_pixel, 0);
  const int last = min(tile.first_pixel + min(tile.n_pixels, NSL_RENDER_TILE), npix);
  if (first >= last) return;
  load_operands<N>(Af, reinterpret_cast<const float*>(rq.prepared), N::FWD_FLOATS);
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = lane_id(), g = lane >> 4, jc = lane & 15;
  LaneLevels<N> ll;
  lane_levels<N>(lv, g, ll);
  const int ntiles = (rp.n_samples + 15) / 16;
  float2* wt = wt_lds + (size_t)wave * 16 * ntiles;
  for (int px = first + wave; px < last; px += 4) {
    const int v = px / rq.W, u = px - v * rq.W;
    float o[3], d[3], s;
    camera_ray(rq.pose, rq.intr, u, v, o, d, s);
    Acts<N> act;
    sh_lane<N>(d, g, act.sh);
    float carry = 0.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, D = 0.0f, A = 0.0f;
    int used = 0;  // tiles composited (the rest of the ray is not)
    wave_lds_fence();  // the previous ray's V* reads are done before this ray's writes
    for (int ti = 0; ti < ntiles; ++ti) {
      const int j = ti * 16 + jc;
      const bool valid = j < rp.n_samples;
      float t;
      {
#pragma clang fp contract(off)
        t = rp.t_near + ((float)j + 0.5f) * rp.dt;
      }
      float xn[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) xn[i] = normalise_axis(pos_axis(o[i], d[i], t), box.lo[i], box.inv[i]);
      encode<N>(rq.params, lv.table_mask, ll, xn, act.e);
      mlp_fwd<N>(Af, lane, act);
      // lanes of row 0 hold sample jc's density and colour
      const float tau = valid ? expf(act.o[0]) * rp.dt : 0.0f;
      const float incl = row_incl_scan(tau);
      const float T = expf(-(carry + (incl - tau)));
      const bool on = valid && !(rp.stop_T > 0.0f && T < rp.stop_T);
      const float w = on ? T * -expm1f(-tau) : 0.0f;
      if (g == 0) wt[j] = make_float2(w, t);
      used = ti + 1;
      C0 += w * sigmoidf(act.z[0]);
      C1 += w * sigmoidf(act.z[1]);
      C2 += w * sigmoidf(act.z[2]);
      D += w * t;
      A += w;
      carry += __shfl(incl, 15, kWave);
      if (rp.stop_T > 0.0f && expf(-carry) < rp.stop_T) break;
    }
    C0 = row_sum(C0);
    C1 = row_sum(C1);
    C2 = row_sum(C2);
    D = row_sum(D);
    A = row_sum(A);
    // V* = sum w (t - d*)^2, d* of row 0, over the composited samples
    const float Dr = __shfl(D, 0, kWave);
    wave_lds_fence();
    float V = 0.0f;
    for (int i = lane; i < 16 * used; i += kWave) {
      const float2 p = wt[i];
      V += p.x * (p.y - Dr) * (p.y - Dr);
    }
#pragma unroll
    for (int o2 = 1; o2 < kWave; o2 <<= 1) V += __shfl_xor(V, o2, kWave);
    if (lane == 0) {
      rq.rgb[3 * (size_t)px] = C0;
      rq.rgb[3 * (size_t)px + 1] = C1;
      rq.rgb[3 * (size_t)px + 2] = C2;
      rq.depth_z[px] = D / s;
      rq.var_z[px] = V / (s * s);
      if (rq.opacity) rq.opacity[px] = A;
    }
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

template <class N>
static hipError_t launch_prep(const float* params, const WOffsets& wo, float* out, hipStream_t st) {
  const int n = N::FWD_FLOATS + N::BWD_FLOATS;
  hipLaunchKernelGGL(prep_weights_kernel<N>, dim3((n + 255) / 256), dim3(256), 0, st, params, wo, out);
  return hipGetLastError();
}

template <class N>
static hipError_t launch_fwd(const FieldArgs& a, const SampleSrc& src, int max_samples,
                             float* sigma, float* rgb, hipStream_t st, const BinPrep* bp) {
  const int tiles = (max_samples + 15) / 16;
  const int grid = (tiles + 3) / 4 < kFieldFwdGrid ? (tiles + 3) / 4 : kFieldFwdGrid;
  const BinPrep none{};
  const BinPrep& b = bp ? *bp : none;
  if (grid + b.nbins > 0)
    hipLaunchKernelGGL(field_fwd_kernel<N>, dim3(grid + b.nbins), dim3(256), 0, st, a, src, sigma, rgb, b);
  return hipGetLastError();
}

template <class N>
static hipError_t launch_bwd(const FieldArgs& a, const SampleSrc& src, int nblocks,
                             const float* dsigma, const float* drgb, const RecordBuffers& rec,
                             float* partial, const WOffsets& wo, float* grads, hipStream_t st) {
  hipLaunchKernelGGL(field_bwd_kernel<N>, dim3(nblocks), dim3(kFieldBwdWaves * kWave), 0, st, a, src, dsigma, drgb,
                     rec, partial);
  return hipGetLastError();
}

template <class N>
static hipError_t launch_render(const LevelInfo& lv, const Aabb& box, const nsl_render_request* reqs, int n_req,
                                const nsl_render_tile* tiles, int n_tiles, const RenderParams& rp, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  const size_t lds = (size_t)4 * 16 * ((rp.n_samples + 15) / 16) * sizeof(float2);
  hipLaunchKernelGGL(render_kernel<N>, dim3(n_tiles), dim3(256), lds, st, lv, box, reqs, n_req, tiles, rp);
  return hipGetLastError();
}

hipError_t render_tiles(int shape, const LevelInfo& lv, const Aabb& box, const nsl_render_request* reqs,
                        int n_req, const nsl_render_tile* tiles, int n_tiles, const RenderParams& rp,
                        hipStream_t st) {
  return shape == kShapeTiny ? launch_render<NetTiny>(lv, box, reqs, n_req, tiles, n_tiles, rp, st)
                             : launch_render<NetFull>(lv, box, reqs, n_req, tiles, n_tiles, rp, st);
}

template <class N>
static hipError_t launch_encode(const FieldArgs& a, const SampleSrc& src, int max_samples, uint32_t* hist,
                                const BinLevels& bl, hipStream_t st) {
  const int grid = encode_grid<N>(max_samples);
  if (grid > 0)
    hipLaunchKernelGGL((encode_levels_kernel<N, float, float2>), dim3(grid), dim3(256), 0, st, a.lv, a.table, src,
                       static_cast<float2*>(src.ecache), src.ecache_stride, hist, bl);
  return hipGetLastError();
}

hipError_t field_encode(int shape, const FieldArgs& a, const SampleSrc& src, int max_samples, uint32_t* hist,
                        const BinLevels& bl, hipStream_t st) {
  return shape == kShapeTiny ? launch_encode<NetTiny>(a, src, max_samples, hist, bl, st)
                             : launch_encode<NetFull>(a, src, max_samples, hist, bl, st);
}

__global__ __launch_bounds__(256) void loss_sum_kernel(LossSum ls) {
  __shared__ float lds[kSumScratchFloats];
  loss_sum_block(ls, lds);
}

hipError_t loss_sum(const LossSum& ls, hipStream_t st) {
  hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(256), 0, st, ls);
  return hipGetLastError();
}

hipError_t field_dw_reduce(int shape, const float* partial, int nblocks, const WOffsets& wo, float* grads,
                           float* overflow, const LossSum* ls, hipStream_t st) {
  return shape == kShapeTiny ? launch_dw_reduce<NetTiny>(partial, nblocks, wo, grads, overflow, ls, st)
                             : launch_dw_reduce<NetFull>(partial, nblocks, wo, grads, overflow, ls, st);
}

size_t field_fwd_floats(int shape) { return shape == kShapeTiny ? NetTiny::FWD_FLOATS : NetFull::FWD_FLOATS; }

size_t field_prep_floats(int shape) {
  return shape == kShapeTiny ? NetTiny::FWD_FLOATS + NetTiny::BWD_FLOATS
                             : NetFull::FWD_FLOATS + NetFull::BWD_FLOATS;
}
size_t field_nweights(int shape) {
  return shape == kShapeTiny ? NetTiny::NWEIGHTS : NetFull::NWEIGHTS;
}

hipError_t field_prep(int shape, const float* params, const WOffsets& wo, float* out, hipStream_t st) {
  return shape == kShapeTiny ? launch_prep<NetTiny>(params, wo, out, st)
                             : launch_prep<NetFull>(params, wo, out, st);
}

hipError_t field_forward(int shape, const FieldArgs& a, const SampleSrc& src, int max_samples,
                         float* sigma, float* rgb, hipStream_t st, const BinPrep* bp) {
  return shape == kShapeTiny ? launch_fwd<NetTiny>(a, src, max_samples, sigma, rgb, st, bp)
                             : launch_fwd<NetFull>(a, src, max_samples, sigma, rgb, st, bp);
}

hipError_t field_backward(int shape, const FieldArgs& a, const SampleSrc& src, int nblocks,
                          const float* dsigma, const float* drgb, const RecordBuffers& rec,
                          float* partial, const WOffsets& wo, float* grads, hipStream_t st) {
  return shape == kShapeTiny
             ? launch_bwd<NetTiny>(a, src, nblocks, dsigma, drgb, rec, partial, wo, grads, st)
             : launch_bwd<NetFull>(a, src, nblocks, dsigma, drgb, rec, partial, wo, grads, st);
}

}  // namespace nsl
