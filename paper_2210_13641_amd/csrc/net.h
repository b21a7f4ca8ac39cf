// Network shapes and MFMA operand layouts of the radiance field.
//
// The MLP runs on v_mfma_f32_16x16x4_f32 in the "features as rows" form
// Y^T = W^T X^T: samples are the 16 MFMA columns, so a layer's output (the D
// operand: lane (g, j) = (lane/16, lane%16) holds rows 4g..4g+3 of column j)
// feeds the next layer's B operand (lane (g, j) holds row k-slot g of column
// j) without moving data: the contraction index is permuted instead, k-step
// s taking feature 16*(s/4) + 4g + (s%4) from register s%4 of tile s/4.
// The weight (A) operands are laid out for that permutation once per step
// by a prep kernel; per (layer, m-tile, k-step) they are 64 contiguous
// floats, one per lane.
//
// Encoding: lane group g evaluates levels g, g+4, ..., so its 2*L/4 values
// are exactly its B-operand slots of the first layer (slot s: level
// g + 4*(s/2), feature s%2).
#pragma once
#include "common.h"

namespace nsl {

template <int L_, int HD_, int NCH_, int HC_, int SHB_>
struct Net {
  static constexpr int L = L_;
  static constexpr int LPL = L_ / 4;     // levels per lane group
  static constexpr int ENC = 2 * L_;     // encoding width
  static constexpr int NSLOT = 2 * LPL;  // encoding slots per lane
  static constexpr int HD = HD_;
  static constexpr int GEO = 16;
  static constexpr int NSH = SHB_ * SHB_;
  static constexpr int SHB = SHB_;
  static constexpr int NCH = NCH_;
  static constexpr int HC = HC_;
  static constexpr int NW = 3 + NCH_;    // weight matrices
  static constexpr int CIN = GEO + NSH;  // true colour input width
  static_assert(L_ % 4 == 0 && HD_ % 16 == 0 && HC_ % 16 == 0 && NSH <= 16, "shape");
  static_assert(NCH_ == 1 || NCH_ == 2, "colour hidden layers");

  // true matrix shapes
  static constexpr int kin(int j) {
    return j == 0 ? ENC : j == 1 ? HD : j == 2 ? CIN : HC;
  }
  static constexpr int kout(int j) {
    return j == 0 ? HD : j == 1 ? GEO : j == NW - 1 ? 3 : HC;
  }
  // forward products: k-steps and m-tiles
  static constexpr int fks(int j) {
    return j == 0 ? NSLOT : j == 1 ? HD / 4 : j == 2 ? 8 : HC / 4;
  }
  static constexpr int fmt(int j) { return j == 1 || j == NW - 1 ? 1 : (j == 0 ? HD : HC) / 16; }
  static constexpr int fsize(int j) { return fks(j) * fmt(j) * kWave; }
  static constexpr int foff(int j) {
    int o = 0;
    for (int i = 0; i < j; ++i) o += fsize(i);
    return o;
  }
  static constexpr int FWD_FLOATS = foff(NW - 1) + fsize(NW - 1);

  // backward (input-gradient) products, indexed by the layer they undo
  static constexpr int bks(int j) { return j == NW - 1 ? 3 : j == 1 ? 4 : j == 0 ? HD / 4 : HC / 4; }
  static constexpr int bmt(int j) {
    return j == NW - 1 ? HC / 16 : j == 2 ? 1 : j == 1 ? HD / 16 : j == 0 ? (NSLOT + 3) / 4 : HC / 16;
  }
  static constexpr int bsize(int j) { return bks(j) * bmt(j) * kWave; }
  static constexpr int boff(int j) {
    int o = 0;
    for (int i = 0; i < j; ++i) o += bsize(i);
    return o;
  }
  static constexpr int BWD_FLOATS = boff(NW - 1) + bsize(NW - 1);

  // compact dW layout (true shapes, [in][out] row-major per layer)
  static constexpr int wsize(int j) { return kin(j) * kout(j); }
  static constexpr int woff(int j) {
    int o = 0;
    for (int i = 0; i < j; ++i) o += wsize(i);
    return o;
  }
  static constexpr int NWEIGHTS = woff(NW - 1) + wsize(NW - 1);

  // staging rows for the dW transposes (X rows then dY rows), 20-float stride
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int XROWS = cmax(cmax((ENC + 15) / 16 * 16, HD), cmax(32, HC));
  static constexpr int YROWS = cmax(HD, HC);
  static constexpr int SROW = 20;
  static constexpr int STAGE_FLOATS = (XROWS + YROWS) * SROW;
};

using NetTiny = Net<4, 32, 1, 32, 3>;
using NetFull = Net<16, 64, 2, 64, 4>;

// Input feature feeding forward k-step s of layer j at lane group g; -1 = pad.
template <class N>
__host__ __device__ constexpr int fwd_in_feature(int j, int s, int g) {
  if (j == 0) return 2 * (g + 4 * (s >> 1)) + (s & 1);
  if (j == 2) {
    if (s < 4) return 4 * g + s;
    const int k = 4 * g + (s - 4);
    return k < N::NSH ? N::GEO + k : -1;
  }
  return 16 * (s >> 2) + 4 * g + (s & 3);
}

// Row (input feature) of output row i of m-tile m of the backward product of
// layer j; -1 = pad.
template <class N>
__host__ __device__ constexpr int bwd_row_feature(int j, int m, int i) {
  if (j == 0) {
    const int gg = i >> 2, jj = 4 * m + (i & 3);
    return jj < N::NSLOT ? 2 * (gg + 4 * (jj >> 1)) + (jj & 1) : -1;
  }
  if (j == 2) return i;  // geometry rows only
  return 16 * m + i;
}

// Output feature consumed by backward k-step s of layer j at lane group g.
template <class N>
__host__ __device__ constexpr int bwd_k_feature(int j, int s, int g) {
  if (j == N::NW - 1) return 4 * g + s;  // z slots
  if (j == 1) return 4 * g + s;          // geometry slots
  return 16 * (s >> 2) + 4 * g + (s & 3);
}

}  // namespace nsl
