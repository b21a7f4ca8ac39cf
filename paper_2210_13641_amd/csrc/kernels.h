// Internal interface between the C ABI (api.cpp) and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nsl.h"
#include "common.h"

namespace nsl {

enum { kShapeTiny = 0, kShapeFull = 1 };

struct WOffsets {
  int off[8];  // float offset of each weight matrix in the parameter vector
};

struct FieldArgs {
  const float* table;  // parameter vector (the tables start at 0)
  const float* wprep;  // MFMA-ready weight operands (field_prep output)
  LevelInfo lv;
};

// Where the field's samples come from: either compacted march samples
// (t, ray) with per-ray records rays[2r] = (o, s), rays[2r+1] = (d, 0), or
// explicit normalised positions and directions.  The sample count is n, or
// *n_dev when n_dev is set (known on the device only).
struct SampleSrc {
  const float* t;
  const uint32_t* ray;
  const float4* rays;
  const float* xn;
  const float* dir;
  Aabb box;
  const uint32_t* n_dev;
  int n;
  // Optional kept encoding, level-major [level][ecache_stride]: FP32 pairs
  // (float2), or BF16 pairs packed in 32 bits in mixed precision.  When set,
  // the forward and backward MLP kernels read it instead of gathering the
  // table (it is written by field_encode / mixed_encode).
  void* ecache;
  int ecache_stride;
};

// The loss of a step from the per-ray shares parts[R][2] (L_rgb, L_D) that
// composite_loss_backward leaves: loss[0..2] = (L_rgb + lambda_d L_D, L_rgb,
// L_D), summed in a fixed order (loss_sum_block).
struct LossSum {
  const float* parts;
  int R;
  float lambda_d;
  float* loss;
};

// scatter.hip: table-gradient records and their binned reduction.
constexpr int kBinShift = 13;                 // 2^13 entries (64 KB of FP32 pairs) per bin
constexpr int kBinEntries = 1 << kBinShift;
constexpr uint32_t kChunk = 65536;            // corner additions per reduce workgroup (at most)
constexpr int64_t kMaxTableEntries = (int64_t)1 << 25;  // all levels together
constexpr int kUnitSamples = 256;             // samples of one level per counting / placement workgroup
constexpr int kEncodeLevelBins = 128;         // bins of a level the counting encoding supports (2^20 entries)

// The bins of the table: level l's entries [offset[l], offset[l] + size[l])
// are cut into bins of kBinEntries entries from the level's first entry (the
// last one shorter), numbered first[l] .. first[l + 1] - 1 over the table,
// so no bin spans two levels.  Records are counted and placed per unit of
// kUnitSamples consecutive samples of one level (nunits units per level).
struct BinLevels {
  int levels, nunits, max_level_bins;
  uint32_t first[kMaxLevels + 1];
  uint32_t offset[kMaxLevels];
  uint32_t size[kMaxLevels];
};

struct RecordBuffers {
  float2* de;             // [levels][stride] dL/de of every sample (two features per level): FP32
                          // pairs, or with de_bf16 the BF16 pairs (g0 | g1 << 16, 32 bits) the
                          // mixed-precision backward stores
  int stride;             // samples per level row of de
  bool de_bf16;
  uint32_t* hist;         // [nbins][nunits] records per bin and unit (unit u of the bin's level)
  uint32_t* off;          // [nbins][nunits] exclusive prefix of hist over the units
  uint32_t* bin_total;    // [nbins]
  uint32_t* bin_start;    // [nbins + 1]
  uint32_t* chunk_start;  // [nbins + 1]
  uint32_t* chunk_bin;    // [max_chunks] bin of each chunk
  void* sorted;           // [max_records] records grouped by bin: each entry's offset in its
                          // bin as uint16_t (the bin is implied by the slot) ...
  uint32_t* sorted_vals;  // ... and its values here: (g0, g1) in FP32 as uint2, or
                          // g0 | g1 << 16 in BF16 as uint32_t ([max_records], inside the
                          // space reserved for sorted)
};

struct BinPlan {
  uint32_t entries;
  int nbins, nunits, levels, stride, max_chunks;
  uint32_t chunk;  // corner additions per reduce workgroup: kChunk, or fewer for tables of few bins
  int64_t max_records;
  BinLevels bl;
};
// Records per reduce workgroup for FP32 or BF16 (paired) records, and whether
// bins of more records than that take chunks of half the size (bins.h).
uint32_t bin_chunk(const BinPlan& p, bool bf16_values);
bool bin_split(const BinPlan& p);

// The column scan (one workgroup of 256 threads per bin) and the bin starts
// (one workgroup) of a table-gradient sort whose records the encoding kernel
// has counted, run as extra workgroups of launches that do not depend on
// them: the forward MLP takes the column scan, the compositing the bin
// starts.  nbins = 0: none.
struct BinPrep {
  RecordBuffers rb;
  int nunits, nbins;
  uint32_t chunk;
  bool split;
};

BinPlan bin_plan(const LevelInfo& lv, uint32_t entries, int64_t max_samples);
// grad_table += the table gradient of the samples of src, from the dL/de
// that the backward kernel left in rb.de; with overwrite, grad_table = that
// gradient (every entry is written, so the caller need not clear it first).
// overflow (may be null): set to 1.0f when a gradient value the call writes
// is not finite (the loss-scale overflow flag).
// counted: rb.hist already holds the record counts (from the encoding).
// ws (may be null): the weight-gradient sum (and the loss sum) of the same
// step, done by extra workgroups of the column-scan launch (it depends only
// on the backward's partials, and the launch is short of work).
struct WeightSum {
  int shape;
  const float* partial;
  int nblocks;
  WOffsets wo;
  float* grads;
  float* overflow;
  LossSum ls;  // ls.loss null: no loss sum
};
// prescanned: the column scan and the bin starts have run already (as the
// extra workgroups of the forward and compositing launches that BinPrep
// describes), so the scatter is the placement, with the weight and loss sums
// of ws as extra workgroups, and the reduction.
hipError_t bin_scatter(const BinPlan& p, const RecordBuffers& rb, const SampleSrc& src, const LevelInfo& lv,
                       bool bf16_values, bool overwrite, float* grad_table, float* overflow, hipStream_t st,
                       bool counted = false, const WeightSum* ws = nullptr, bool prescanned = false);

// field.hip
size_t field_prep_floats(int shape);
size_t field_nweights(int shape);
hipError_t field_prep(int shape, const float* params, const WOffsets& wo, float* out, hipStream_t st);
hipError_t field_forward(int shape, const FieldArgs& a, const SampleSrc& src, int max_samples,
                         float* sigma, float* rgb, hipStream_t st, const BinPrep* bp = nullptr);
constexpr int kFieldBwdWaves = 4;             // waves per workgroup of the FP32 backward
// Writes dL/de of every sample to rec.de and the weight gradients of each
// workgroup to partial[nblocks][weights]; field_dw_reduce then adds them
// into grads and bin_scatter the table gradient.
hipError_t field_backward(int shape, const FieldArgs& a, const SampleSrc& src, int nblocks,
                          const float* dsigma, const float* drgb, const RecordBuffers& rec,
                          float* partial, const WOffsets& wo, float* grads, hipStream_t st);

// loss[0..2] from the per-ray shares alone (one workgroup, fixed order).
hipError_t loss_sum(const LossSum& ls, hipStream_t st);
// ls (may be null): the step's loss is summed by the same launch.
hipError_t field_dw_reduce(int shape, const float* partial, int nblocks, const WOffsets& wo, float* grads,
                           float* overflow, const LossSum* ls, hipStream_t st);
// The encoding of every sample of src into src.ecache (FP32 table).  With
// hist (at most kEncodeLevelBins bins a level; nullable), also the
// table-gradient record counts per bin and unit, written to every
// hist[bin][unit] of bl (no clearing needed): bin_scatter can then skip its
// counting pass.  bl.nunits must be the units of max_samples.
hipError_t field_encode(int shape, const FieldArgs& a, const SampleSrc& src, int max_samples, uint32_t* hist,
                        const BinLevels& bl, hipStream_t st);

struct RenderParams {
  float t_near, dt, stop_T;
  int n_samples;  // at most kRenderMaxSamples
};
constexpr int kRenderMaxSamples = NSL_RENDER_MAX_SAMPLES;
// Fused ray-major rendering of tiles (tiles == nullptr: tile t covers pixels
// [64t, 64t+64) of request 0).
hipError_t render_tiles(int shape, const LevelInfo& lv, const Aabb& box, const nsl_render_request* reqs,
                        int n_req, const nsl_render_tile* tiles, int n_tiles, const RenderParams& rp,
                        hipStream_t st);
size_t field_fwd_floats(int shape);

// field_mixed.hip: FP16 table, BF16 MLP on MFMA, FP32 accumulation.  The
// shadow buffer holds the BF16 operands and the FP16 table copy.
size_t mixed_shadow_bytes(int shape, int64_t table_floats);
// zero_grads (may be null): a gradient vector of total floats whose entries
// from table_floats rounded down to a multiple of 8 onwards (the MLP weights
// and padding) are cleared in the same pass as the FP16 table copy; the table
// part is left to bin_scatter's overwrite.  clear_flag (may be null) is set
// to 0 by the same launch (the loss-scale overflow flag at the start of a
// step).
hipError_t mixed_prepare(int shape, const float* params, const WOffsets& wo, int64_t table_floats, void* shadow,
                         float* zero_grads, int64_t total, float* clear_flag, hipStream_t st);
hipError_t mixed_forward(int shape, const LevelInfo& lv, const void* shadow, const SampleSrc& src, int max_samples,
                         float* sigma, float* rgb, hipStream_t st, const BinPrep* bp = nullptr);
// The encoding of every sample of src into src.ecache (FP16 table, BF16 out);
// hist as for field_encode.
hipError_t mixed_encode(int shape, const LevelInfo& lv, const void* shadow, const SampleSrc& src, int max_samples,
                        uint32_t* hist, const BinLevels& bl, hipStream_t st);
hipError_t mixed_backward(int shape, const LevelInfo& lv, const void* shadow, const SampleSrc& src, int nblocks,
                          const float* dsigma, const float* drgb, const RecordBuffers& rec, float* partial,
                          const WOffsets& wo, float* grads, hipStream_t st);

// march.hip
struct KeyframeStore {
  const float* rgb;        // [K,H,W,3]
  const float* depth;      // [K,H,W]
  const float* var;        // [K,H,W]
  const float* pose;       // [K,12]
  const float* intr;       // [K,4]
  const uint32_t* occ;     // bitfield
  int H, W, K, grid_res;
};

struct MarchParams {
  int sampler;
  float t_near, t_far, dt;
  int n_uniform, max_per_ray, max_samples;
  Aabb box;
};

// Per-candidate ray records and targets written by the ray kernel.
struct RayBuffers {
  float4* rays;        // [2*n]: (o, s), (d, 0)
  float4* target;      // [n]: (r, g, b, D_ray)
  float* prec;         // [n]: 1/Sigma_ray or 0
  uint32_t* counts;    // [n]
  uint32_t* offsets;   // [n+1]
  uint32_t* block_sums;
  uint32_t* stats;     // [4]: R, S, kept, masked
  float* loss;         // [3]
};

hipError_t march_rays(const KeyframeStore& kf, const MarchParams& mp, const uint32_t* ids, int n,
                      const RayBuffers& rb, hipStream_t st);
hipError_t march_emit(const KeyframeStore& kf, const MarchParams& mp, const uint32_t* ids, int n,
                      const RayBuffers& rb, float* t_out, uint32_t* ray_out, hipStream_t st);
// The offsets and batch cut of counts the ray setup has written.
hipError_t march_scan(const MarchParams& mp, int n, const RayBuffers& rb, hipStream_t st);
size_t march_block_count(int n);
// mixed_prepare and the ray setup and sample counts of march_rays in one
// launch (field_mixed.hip); march_scan then completes march_rays.
hipError_t mixed_prepare_count(int shape, const float* params, const WOffsets& wo, int64_t table_floats,
                               void* shadow, float* zero_grads, int64_t total, float* clear_flag,
                               const KeyframeStore& kf, const MarchParams& mp, const uint32_t* ids, int n,
                               const RayBuffers& rb, hipStream_t st);

// composite.hip
struct CompositeIO {
  const float* sigma;
  const float* rgb;
  const float* t;
  const uint32_t* off;     // ray r owns [off[r], off[r+1])  (train step: candidate offsets)
  const uint32_t* counts;  // optional: kept iff off[r+1] <= max_samples and counts[r] > 0
  int max_samples;
  int R;
  float delta;
  float stop_T;
  float* out6;             // [R,6] ray units (or null)
};

struct LossIO {
  const float4* target;    // (r, g, b, D_ray)
  const float* prec;
  const float4* rays;      // for s (z units)
  const uint32_t* stats;   // R at stats[0]
  float lambda_d;
  float loss_scale;
  const float* scale_dev;  // if set, the loss scale is read from scale_dev[0]
  float* loss;             // [3] written: L, L_rgb, L_D
  float* parts;            // [R,2] per-ray L_rgb and L_D shares (workspace)
  float* ray_out;          // [R,6] z units or null
};

hipError_t composite_forward(const CompositeIO& io, hipStream_t st);
hipError_t composite_backward(const CompositeIO& io, const float* g_rgb, const float* g_depth,
                              const float* g_var, const float* g_opacity, float* g_sigma, float* g_rgb_s,
                              hipStream_t st);
// Writes the per-ray loss shares to lo.parts; their sum into lo.loss is
// left to a LossSum (the step's last reduction launch).
hipError_t composite_loss_backward(const CompositeIO& io, const LossIO& lo, float* g_sigma,
                                   float* g_rgb_s, hipStream_t st, const BinPrep* bp = nullptr);

// Per-ray loss shares (parts [R][2], nullable) and adjoint seeds (g_out
// [R][6], nullable) of rays rendered outside the step; n_masked (nullable)
// += rays whose depth measurement is unusable.
hipError_t loss_terms(const float* out6, int R, const float* rgb_target, const float* depth_z, const float* var_z,
                      const float* ray_scale, float lambda_d, const float* g_loss, float* parts, float* g_out,
                      uint32_t* n_masked, hipStream_t st);

// noalloc.hip: the static device scratch of nsl_render_noalloc (its size,
// and its address on the current device, looked up once per device).
size_t noalloc_scratch_bytes();
hipError_t noalloc_scratch(void** out);

// peaks.hip: machine-peak probes (not part of the step)
hipError_t peak_copy(const void* src, void* dst, size_t bytes, hipStream_t st);
hipError_t peak_gather(const uint32_t* table, int log2_entries, uint32_t* out, int n_threads, int loads,
                       hipStream_t st);
hipError_t peak_mfma(int bf16, float* out, int n_workgroups, int iters, hipStream_t st);

// cov.hip
size_t cov_partial_blocks(int p);
hipError_t depth_covariance(int c, int p, const double* C, const double* Et, const double* P,
                            const double* inv_depth, double* sigma_T, double* sigma_d, float* depth_var,
                            int* status, double* partial, hipStream_t st);

// misc.hip
// scale_state (nullable): gradient scale 1/scale_state[0], skip if scale_state[3] != 0.
hipError_t adam_update(float* p, float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, int step, float grad_scale, const float* scale_state,
                       hipStream_t st);
// Dynamic loss scaling: clear the overflow flag, flag non-finite gradients,
// then halve (overflow) or count clean steps and double after 2000.
hipError_t scale_begin(float* state, hipStream_t st);
hipError_t scale_end(float* state, hipStream_t st);
// p[0, n) = 0 and, in the same launch, q[0, m) = 0 (q nullable); both
// 16-byte aligned.
hipError_t fill_zero(float* p, int64_t n, hipStream_t st);
// Writes one request record to device memory (taken by value at launch),
// with its pose [12] and intrinsics [4] read from device memory.
hipError_t store_request(const nsl_render_request* r, const float* pose, const float* intr,
                         nsl_render_request* dst, hipStream_t st);

}  // namespace nsl
