/*
 * nsl.h -- C ABI of the NeRF-SLAM mapping step on AMD Instinct MI355X (gfx950).
 *
 * The paper (Rosinol, Leonard, Carlone, "NeRF-SLAM") trains a hash-grid
 * radiance field from the output of dense monocular SLAM: keyframe images,
 * poses, dense depth maps and their marginal covariances (Sec. 3.1, Eq. 2,
 * and Sec. 3.3: the tracking thread sends them on every new keyframe).  The
 * mapping thread minimises  L_M = L_rgb + lambda_D * L_D  over the field
 * parameters (Sec. 3.2, Eq. 3, lambda_D = 1.0) using all keyframes received,
 * with the depth loss weighted by the depth covariance (Eq. 4), rendered
 * depth as the expected termination distance (Eq. 5), transmittance (Eq. 6)
 * and the photometric loss (Eq. 7).  This library is that training step, one
 * call per iteration, plus forward rendering (Sec. 3.3, last paragraph).
 *
 * Conventions (every call):
 *  - Every function returns an int status: NSL_OK (0) or a negative NSL_E_*.
 *    On error nsl_last_error() returns a thread-local message.  No C++
 *    exception crosses the ABI.
 *  - All device memory is owned by the caller and passed as plain device
 *    pointers; the library never allocates device memory.  Calls that need
 *    scratch space take a caller workspace whose size a *_workspace_bytes
 *    query returns (NSL_E_WORKSPACE if too small); nsl_render_noalloc uses
 *    a static device array of the library instead.  Host-side handles
 *    (nsl_field, nsl_mapper) are small host allocations.
 *  - Calls are asynchronous on the given stream; results are valid after the
 *    stream is synchronised.  Pointers must stay valid until then.
 *  - Parameter vectors (params, grads, Adam moments, the params of render
 *    requests) and mixed-precision shadows are 16-byte aligned: the kernels
 *    read them with 16-byte loads.  Calls that receive them reject other
 *    addresses with NSL_E_INVALID (render requests are device records and
 *    are not checked).
 *  - Camera model: pinhole, OpenCV axes (x right, y down, z forward);
 *    pose = camera-to-world [R | t], 3x4 row-major float; intrinsics
 *    (fx, fy, cx, cy); pixel (u, v) has its centre at (u+1/2, v+1/2).
 *    Depths and variances at the boundary are z-depth D_z and its variance
 *    Sigma_D in m^2 (the paper's Sigma_D, Eq. 4); internally distances are
 *    measured along the unit ray direction.
 *  - Pixel ids address keyframe slot k, row v, column u as k*H*W + v*W + u.
 *  - Unusable depth measurements (non-finite D_z, non-finite or non-positive
 *    Sigma_D) are masked (weight 0), not errors; their count is reported.
 */
#ifndef NSL_H_
#define NSL_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NSL_OK 0
#define NSL_E_INVALID -1     /* null pointer, bad shape, bad or unsupported config */
#define NSL_E_WORKSPACE -2   /* workspace smaller than the size query returned */
#define NSL_E_HIP -3         /* a HIP runtime call failed; message has the code */
#define NSL_E_BUDGET -4      /* request exceeds the configured memory budget */
#define NSL_E_CAPACITY -5    /* keyframe store full */

#define NSL_F32 0
#define NSL_F16 1
#define NSL_BF16 2

#define NSL_PRECISION_FP32 0   /* FP32 tables, FP32 MLP on FP32 MFMA */
#define NSL_PRECISION_MIXED 1  /* FP16 tables, BF16 MLP on MFMA, FP32 accumulation */

#define NSL_SAMPLER_UNIFORM 0
#define NSL_SAMPLER_OCCUPANCY 1

#define NSL_MAX_LEVELS 16
#define NSL_MAX_LAYERS 8

/* Last error message of the calling thread ("" if none). */
const char* nsl_last_error(void);

/* ABI version (major*100 + minor). */
int nsl_version(void);

/* ------------------------------------------------------------------------
 * Field: multiresolution hash grid + density net + colour net.
 *
 * The paper builds its map on Instant-NGP and defers the network inputs to
 * it (Sec. 3.2 after Eq. 5; Sec. 3.4).  Level l has resolution
 * N_l = floor(base_res * b^l) (b = per_level_scale, or, if that is <= 0,
 * b = exp((ln max_res - ln base_res)/(levels-1)); with max_res > 0 the top
 * level is max_res).  A level with (N_l+1)^3 <= 2^log2_table entries is
 * dense (index x + (N+1)(y + (N+1)z)), otherwise hashed
 * ((x ^ 2654435761 y ^ 805459861 z) mod 2^log2_table).  Trilinear weights
 * use p = xn*N_l, i0 = min(floor(p), N_l-1).  Density: h = ReLU(e W1),
 * o = h W2 (geo_dim = 16 wide), sigma = exp(o_0).  Colour: c =
 * sigmoid(MLP([o_0..o_15, SH(d)])) with ReLU hidden layers, real
 * orthonormal SH of sh_bands bands.  Layers are bias-free.
 *
 * Supported shapes (compiled kernels): feat_per_level 2, geo_dim 16 and
 *   levels 4,  density_hidden 32, colour_hidden {32},     sh_bands 3, or
 *   levels 16, density_hidden 64, colour_hidden {64, 64}, sh_bands 4.
 * Anything else returns NSL_E_INVALID from nsl_field_create, as does a
 * table of more than 2^25 entries (all levels together).
 * ------------------------------------------------------------------------ */
typedef struct nsl_field_config {
  int32_t levels;
  int32_t feat_per_level;
  int32_t log2_table;
  int32_t base_res;
  float per_level_scale; /* <= 0: derived from max_res */
  int32_t max_res;       /* 0: none */
  int32_t density_hidden;
  int32_t geo_dim;
  int32_t sh_bands;
  int32_t n_colour_hidden;
  int32_t colour_hidden[4];
  float aabb_min[3];
  float aabb_max[3];
} nsl_field_config;

/* Parameter vector layout: FP32, the tables first (level-major, then entry,
 * then feature), then every weight matrix [fan_in, fan_out] row-major in
 * network order (W1, W2, colour layers...), each block starting at a
 * multiple of 64 floats. */
typedef struct nsl_param_layout {
  int32_t levels;
  int32_t res[NSL_MAX_LEVELS];
  int32_t dense[NSL_MAX_LEVELS];
  int64_t level_entries[NSL_MAX_LEVELS];
  int64_t level_offset[NSL_MAX_LEVELS]; /* in entries */
  int64_t table_floats;
  int32_t n_layers;
  int64_t w_offset[NSL_MAX_LAYERS]; /* in floats */
  int32_t w_in[NSL_MAX_LAYERS];
  int32_t w_out[NSL_MAX_LAYERS];
  int64_t total_floats;
} nsl_param_layout;

typedef struct nsl_field nsl_field;

/* Fill *out from cfg (host-only arithmetic). */
int nsl_field_layout(const nsl_field_config* cfg, nsl_param_layout* out);
int nsl_field_create(const nsl_field_config* cfg, nsl_field** out);
void nsl_field_destroy(nsl_field* f);

/* ------------------------------------------------------------------------
 * Mapper: keyframe store and occupancy grid (Sec. 3.3: the mapping thread
 * optimises all keyframes received; tracking re-sends the keyframes of its
 * window, whose poses and depths it keeps re-estimating).
 *
 * Storage is a caller-owned device buffer of nsl_mapper_storage_bytes().
 * ------------------------------------------------------------------------ */
typedef struct nsl_mapper nsl_mapper;

size_t nsl_mapper_storage_bytes(int max_keyframes, int H, int W, int grid_res);
int nsl_mapper_create(int max_keyframes, int H, int W, int grid_res, void* storage,
                      size_t storage_bytes, nsl_mapper** out);
void nsl_mapper_destroy(nsl_mapper* m);
/* Number of keyframe slots in use. */
int nsl_mapper_count(const nsl_mapper* m);

/* Insert or update n keyframes.  ids: host array of caller ids; an id seen
 * before overwrites its slot, a new id takes the next free slot (slots in
 * order of first arrival; NSL_E_CAPACITY when full, nothing copied).
 *   rgb       [n,H,W,3] float in [0,1]
 *   pose      [n,3,4]   camera-to-world
 *   intr      [n,4]     fx, fy, cx, cy
 *   depth     [n,H,W]   z-depth D_z
 *   depth_var [n,H,W]   Sigma_D (m^2)
 * src_on_host: 1 if the arrays are host memory, 0 if device memory. */
int nsl_keyframes_upsert(nsl_mapper* m, int n, const int32_t* ids, const float* rgb,
                         const float* pose, const float* intr, const float* depth,
                         const float* depth_var, int src_on_host, hipStream_t stream);
/* Slot of caller id, or -1. */
int nsl_keyframe_slot(const nsl_mapper* m, int32_t id);

/* Occupancy bitfield over the field's AABB: res^3 bits (res given at
 * creation), cell (x,y,z) -> bit x + res*(y + res*z), uint32 words, least
 * significant bit first. */
int nsl_occupancy_set(nsl_mapper* m, const uint32_t* bits, int src_on_host,
                      hipStream_t stream);

/* ------------------------------------------------------------------------
 * Training step.
 *
 * Rays: pixel_ids[n_candidates] (device) in keyframe slots.  Samples:
 *  - NSL_SAMPLER_UNIFORM:   t_i = t_near + (i+1/2)*dt, i < n_uniform;
 *  - NSL_SAMPLER_OCCUPANCY: lattice t_k = (k+1/2)*dt from the ray origin,
 *    kept iff t_near <= t_k <= t_far, the point is inside the closed AABB
 *    and its occupancy bit is set; at most max_per_ray per ray.
 * Every sample has bin width delta = dt (Eq. 5 takes delta_i = d_{i+1}-d_i;
 * with midpoint bins this is dt for every interior pair, and empty space
 * skipped by the grid has sigma = 0).  Candidates are kept in order while
 * their inclusive sample prefix is <= max_samples; kept candidates with at
 * least one sample are the R rays of the batch.  max_samples * 8 * levels
 * must stay below 2^32 (the workspace query returns 0 otherwise).
 *
 * Loss (Eq. 3, 4, 7), mean over the R rays:
 *   L_rgb = mean_r sum_ch (I*_r - I_r)^2
 *   L_D   = mean_r (d*_r - D_r)^2 / Sigma_D,r   (ray units; invariant to z/ray)
 *   L     = L_rgb + lambda_d * L_D
 * Rendering (Eq. 5, 6): w_i = T_i (1 - exp(-sigma_i delta)), I* = sum w_i c_i,
 * d* = sum w_i t_i; also V* = sum w_i (t_i - d*)^2 and A = sum w_i; no
 * background colour, no normalisation by A.
 *
 * Gradients are ACCUMULATED (+=) into grads, scaled by the loss scale, unless
 * zero_grads = 1 (grads are cleared first).  With do_adam = 1 the step then
 * applies bias-corrected Adam at step adam_step (>= 1) to every parameter
 * with gradient grads / loss scale and clears grads afterwards.
 *
 * keep_encoding: the backward needs the encoding e of every sample.  With 0
 * it gathers the table again (no per-sample activations are kept between the
 * forward and the backward; the MLP is always recomputed).  With 1 the
 * forward stores e in the workspace (2*levels values per sample, FP32, or
 * BF16 in mixed precision, exactly as the MLP consumes it) and the backward
 * reads it: the same results, about 128 (64) bytes per sample of traffic
 * instead of a second gather, whose random reads move whole cache lines.
 *
 * precision: NSL_PRECISION_FP32, or NSL_PRECISION_MIXED: the step converts
 * the FP32 master parameters to an FP16 table copy and BF16 MLP operands,
 * evaluates and differentiates the field with BF16 MFMA and FP32
 * accumulation, and accumulates every gradient in FP32; transmittance, the
 * depth-variance reduction and the Sigma_D-weighted loss stay FP32.
 * scale_state (device float[4], may be NULL): dynamic loss scaling.  The
 * scale is read from scale_state[0] (loss_scale is then ignored); a
 * non-finite value among the gradients the step writes (every MLP weight
 * gradient and the table entries its samples touch, checked as they are
 * written) sets scale_state[3] = 1, Adam skips the update (gradients are
 * cleared), the scale is halved and scale_state[2] counts the skip; otherwise
 * scale_state[1] counts clean steps and the scale doubles after 2000 of them.
 * adam_step counts every step the caller runs, skipped ones included; the
 * bias correction uses the number of updates made, adam_step - scale_state[2]
 * (at least 1), read on the device.
 * Gradients carried over from earlier steps (zero_grads = 0 without Adam)
 * were checked by the step that wrote them.
 *
 * loss_out (device, 3 floats): L, L_rgb, L_D.  stats_out (device, may be
 * NULL).  ray_out (device, may be NULL): [n_candidates, 6] per candidate:
 * r, g, b, depth_z = d* / s, var_z = V* / s^2, opacity A (zeros for candidates
 * that are not rays of the batch).
 * ------------------------------------------------------------------------ */
typedef struct nsl_step_config {
  int32_t sampler;
  float t_near, t_far, dt;
  int32_t n_uniform;
  int32_t max_per_ray;
  int32_t max_samples;
  float lambda_d;
  int32_t zero_grads;
  int32_t do_adam;
  float lr, beta1, beta2, eps;
  int32_t adam_step;
  float loss_scale;
  int32_t precision;     /* NSL_PRECISION_FP32 or NSL_PRECISION_MIXED */
  float* scale_state;    /* device float[4] or NULL (static loss_scale) */
  int32_t keep_encoding; /* 0: the backward recomputes the encoding from the table; 1: the
                            forward keeps it in the workspace for the backward */
} nsl_step_config;

typedef struct nsl_step_stats {
  uint32_t n_rays;        /* R */
  uint32_t n_samples;     /* S */
  uint32_t n_kept;        /* kept candidates (including zero-sample ones) */
  uint32_t n_masked;      /* rays whose depth measurement was unusable */
} nsl_step_stats;

size_t nsl_step_workspace_bytes(const nsl_field* f, const nsl_step_config* cfg,
                                int n_candidates);
int nsl_train_step(nsl_mapper* m, const nsl_field* f, float* params, float* grads,
                   float* adam_m, float* adam_v, const nsl_step_config* cfg,
                   const uint32_t* pixel_ids, int n_candidates, void* workspace,
                   size_t workspace_bytes, float* loss_out, nsl_step_stats* stats_out,
                   float* ray_out, hipStream_t stream);

/* Phase timing.  While enabled, every nsl_train_step records a HIP event on
 * its stream before each phase and after the last one, waits for the last
 * event (so profiled steps synchronise the host), and accumulates the
 * elapsed milliseconds per phase:
 *   0 gradient clearing (the MLP weights and padding; the table part is
 *   overwritten by the reduction of phase 6) and weight-operand preparation,
 *   1 rays + march +
 *   batch cut, 2 encoding of every sample (keep_encoding = 1 only),
 *   3 field forward (MLP; with keep_encoding = 0 also the table gather),
 *   4 compositing + loss + its adjoint, 5 field backward kernel (MLP
 *   recompute and adjoint, weight gradients per workgroup, dL/de),
 *   6 table gradient (bin count, scans, placement, reduction), with the
 *   weight-gradient reduction and the sum of the loss done by the same
 *   launches, 7 (empty: kept so that the phase numbers stay), 8 Adam (and
 *   the loss-scale update).
 * nsl_profile_read copies the sums (ms[NSL_PHASES]) and the number of
 * profiled steps; enabling again resets them. */
#define NSL_PHASES 9
int nsl_profile_enable(int on);
int nsl_profile_read(double* ms, int* n_steps);

/* ------------------------------------------------------------------------
 * Kernel-level entry points: the same kernels as the step, one phase each.
 * ------------------------------------------------------------------------ */

/* Rays and samples of the step for the given candidates (the sampler of
 * nsl_train_step).  Outputs (device): counts[n_candidates] samples per
 * candidate before the cut, offsets[n_candidates+1] exclusive prefix,
 * t[max_samples] and ray[max_samples] (candidate index of each sample) for
 * the kept candidates, stats (device).  Workspace: nsl_step_workspace_bytes. */
int nsl_march(nsl_mapper* m, const nsl_field* f, const nsl_step_config* cfg,
              const uint32_t* pixel_ids, int n_candidates, void* workspace,
              size_t workspace_bytes, uint32_t* counts, uint32_t* offsets, float* t,
              uint32_t* ray, nsl_step_stats* stats_out, hipStream_t stream);

/* Field at S normalised positions xn [S,3] in [0,1]^3 with unit view
 * directions dirs [S,3]: sigma [S], rgb [S,3].  Workspace:
 * nsl_field_workspace_bytes(f, S) (the weights laid out for the MFMA
 * operands, the per-block weight gradients and the table-gradient records of
 * the backward; one size serves both precisions and any count up to S).
 * Returns 0 when S * 8 * levels reaches 2^32. */
size_t nsl_field_workspace_bytes(const nsl_field* f, int S);
int nsl_field_fwd(const nsl_field* f, const float* params, const float* xn, const float* dirs,
                  int S, float* sigma, float* rgb, void* workspace, size_t workspace_bytes,
                  hipStream_t stream);

/* Adjoint of nsl_field_fwd: accumulates (+=) dL/dparams into grads given
 * dsigma [S] and drgb [S,3].  The table part (the trilinear weights times
 * dL/de, summed over samples and corners) is written as records, grouped by
 * table bin and reduced in LDS (summation order unspecified); the weight
 * part is reduced in a fixed order. */
int nsl_field_bwd(const nsl_field* f, const float* params, const float* xn, const float* dirs,
                  int S, const float* dsigma, const float* drgb, float* grads, void* workspace,
                  size_t workspace_bytes, hipStream_t stream);

/* Mixed precision at the kernel level: nsl_field_prepare_mixed converts the
 * FP32 parameters into a shadow buffer (BF16 MLP operands and an FP16 copy
 * of the tables, nsl_mixed_shadow_bytes); nsl_field_fwd_mixed and
 * nsl_field_bwd_mixed evaluate and differentiate the field from it (FP32
 * accumulation; gradients with respect to the FP32 parameters, accumulated
 * into grads).  Workspace of the backward: nsl_field_workspace_bytes. */
size_t nsl_mixed_shadow_bytes(const nsl_field* f);
int nsl_field_prepare_mixed(const nsl_field* f, const float* params, void* shadow, hipStream_t stream);
int nsl_field_fwd_mixed(const nsl_field* f, const void* shadow, const float* xn, const float* dirs, int S,
                        float* sigma, float* rgb, hipStream_t stream);
int nsl_field_bwd_mixed(const nsl_field* f, const void* shadow, const float* xn, const float* dirs, int S,
                        const float* dsigma, const float* drgb, float* grads, void* workspace,
                        size_t workspace_bytes, hipStream_t stream);

/* Compositing of R rays whose samples are contiguous: ray r owns samples
 * [ray_off[r], ray_off[r+1]).  out[R,6] = (r, g, b, d*, V*, A) in ray
 * units (Eq. 5, 6).  With stop_T > 0 a ray stops before the first sample
 * with T_i < stop_T (early termination; 0 disables). */
int nsl_composite_fwd(const float* sigma, const float* rgb, const float* t,
                      const uint32_t* ray_off, int R, float delta, float stop_T, float* out,
                      hipStream_t stream);

/* Adjoint of nsl_composite_fwd (stop_T = 0) for seeds g_rgb [R,3],
 * g_depth [R], g_var [R], g_opacity [R] (any of them may be NULL = 0):
 * g_sigma [S], g_rgb_s [S,3] (overwritten). */
int nsl_composite_bwd(const float* sigma, const float* rgb, const float* t,
                      const uint32_t* ray_off, int R, float delta, const float* g_rgb,
                      const float* g_depth, const float* g_var, const float* g_opacity,
                      float* g_sigma, float* g_rgb_s, hipStream_t stream);

/* ------------------------------------------------------------------------
 * The mapping loss on its own (Sec. 3.2, Eq. 3, 4 and 7), for rays rendered
 * by nsl_composite_fwd (the autograd path); the step computes the same
 * per-ray terms inside its compositing kernel.
 *
 * out6 [R,6]: r, g, b, d*, V*, A in ray units, as nsl_composite_fwd writes
 * them; rgb_target [R,3]; depth_z [R] (z-depth D); depth_var_z [R] (Sigma_D,
 * a variance in m^2); ray_scale [R] = s = |d~| (ray length per unit of z).
 * The depth target along the ray is D s with precision 1/(Sigma_D s^2); a
 * non-finite D or Sigma_D, or Sigma_D <= 0, gives precision 0 (masked).
 *   L_rgb = (1/R) sum_r |I*_r - I_r|^2,  L_D = (1/R) sum_r pi_r (d*_r - D_r s_r)^2,
 *   L = L_rgb + lambda_d L_D.
 * nsl_loss_fwd writes loss_out [3] = (L, L_rgb, L_D) (device), summed in a
 * fixed order (deterministic), and the number of masked rays into n_masked
 * (device uint32, may be NULL).  ws: nsl_loss_workspace_bytes(R) bytes.
 * nsl_loss_bwd writes the seeds of the adjoint, g_out6 [R,6] = dJ/d out6,
 * for upstream gradients g_loss (device [3]: dJ/dL, dJ/dL_rgb, dJ/dL_D;
 * NULL means (1, 0, 0)); the V* and A columns get 0.  All pointers are
 * device memory; R >= 1.  Both calls are asynchronous on the stream.
 * ------------------------------------------------------------------------ */
size_t nsl_loss_workspace_bytes(int R);
int nsl_loss_fwd(const float* out6, int R, const float* rgb_target, const float* depth_z,
                 const float* depth_var_z, const float* ray_scale, float lambda_d, float* loss_out,
                 uint32_t* n_masked, void* workspace, size_t workspace_bytes, hipStream_t stream);
int nsl_loss_bwd(const float* out6, int R, const float* rgb_target, const float* depth_z,
                 const float* depth_var_z, const float* ray_scale, float lambda_d, const float* g_loss,
                 float* g_out6, hipStream_t stream);

/* ------------------------------------------------------------------------
 * The hash-grid encoding and its adjoint on their own (Sec. 3.2 after Eq. 5:
 * the map's inputs are the multiresolution hash-grid features of the prior
 * work), with the kernels the step runs when it keeps the encoding.
 *
 * xn [S,3]: normalised positions (clamped to [0,1]).  e_out is level-major,
 * [levels][S]: nsl_encode_fwd writes FP32 feature pairs (float2) from the
 * FP32 table of params; nsl_encode_fwd_mixed writes each pair as two BF16
 * values packed in 32 bits (first feature in the low half), from the FP16
 * table copy of a shadow made by nsl_field_prepare_mixed, exactly as the
 * mixed-precision MLP consumes them.
 *
 * nsl_encode_bwd scatters dL/de into the table part of grads: de is
 * level-major [levels][S] float2 (FP32); each (sample, level, corner)
 * contributes w_c * dL/de, formed in FP32 (precision NSL_PRECISION_FP32) or
 * rounded to BF16 (NSL_PRECISION_MIXED, the mixed step's records), and every
 * sum is FP32.  overwrite = 0 adds to grads; overwrite = 1 sets the table
 * part to the gradient (untouched entries become 0).  The MLP part of grads
 * is not touched.  grads and de must be 16-byte aligned; ws:
 * nsl_encode_bwd_workspace_bytes(f, S) bytes.  S * 8 * levels < 2^32.
 * ------------------------------------------------------------------------ */
int nsl_encode_fwd(const nsl_field* f, const float* params, const float* xn, int S, float* e_out,
                   hipStream_t stream);
int nsl_encode_fwd_mixed(const nsl_field* f, const void* shadow, const float* xn, int S, uint32_t* e_out,
                         hipStream_t stream);
size_t nsl_encode_bwd_workspace_bytes(const nsl_field* f, int S);
int nsl_encode_bwd(const nsl_field* f, const float* xn, int S, const float* de, int precision, int overwrite,
                   float* grads, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * The field's MLP on its own (Sec. 3.2 after Eq. 7: the density sigma and
 * colour c of a sample come from one evaluation of the density and colour
 * networks), on a given encoding, with the kernels the step runs when it
 * keeps the encoding (FP32).
 *
 * enc: level-major [levels][S] FP32 feature pairs (float2), as
 * nsl_encode_fwd writes them; dirs [S,3]: unit view directions.
 * nsl_mlp_fwd writes sigma [S] and rgb [S,3].  nsl_mlp_bwd, given dsigma [S]
 * and drgb [S,3], accumulates (+=) the weight gradients into the MLP part of
 * grads (the table part is not touched) and writes dL/de to d_enc, laid out
 * like enc (the input of nsl_encode_bwd).  Workspace:
 * nsl_field_workspace_bytes(f, S).  params, grads, enc and d_enc must be
 * 16-byte aligned.
 * ------------------------------------------------------------------------ */
int nsl_mlp_fwd(const nsl_field* f, const float* params, const float* enc, const float* dirs, int S,
                float* sigma, float* rgb, void* workspace, size_t workspace_bytes, hipStream_t stream);
int nsl_mlp_bwd(const nsl_field* f, const float* params, const float* enc, const float* dirs, int S,
                const float* dsigma, const float* drgb, float* grads, float* d_enc, void* workspace,
                size_t workspace_bytes, hipStream_t stream);

/* Bias-corrected Adam over n parameters, gradient = grads * grad_scale;
 * clears grads. */
int nsl_adam(float* params, float* grads, float* m, float* v, int64_t n, float lr, float beta1,
             float beta2, float eps, int step, float grad_scale, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Depth covariances from the tracking Hessian (Sec. 3.1, Eq. 1 and 2): the
 * producer of the Sigma_D that weights the depth loss (Eq. 4).
 *
 * The dense-BA system of a keyframe window is [[C, E], [E^T, P]] with P
 * diagonal (one inverse depth per pixel).  In FP64:
 *   H_T = C - E P^{-1} E^T = L L^T,  Sigma_T = (L L^T)^{-1},
 *   Sigma_d,j = 1/P_j + e_j^T Sigma_T e_j / P_j^2   (diagonal of Eq. 2),
 *   depth_var_j = Sigma_d,j / d_j^4                 (variance of D = 1/d,
 *                                                    first order).
 * Arguments (device): C [c,c] row-major (c = 6 per keyframe, c <= 60);
 * Et [p,c] = E^T row-major (pixel j's coupling e_j contiguous); P [p] > 0;
 * inv_depth [p]; outputs sigma_T [c,c], sigma_d [p] (may be NULL),
 * depth_var [p] float (may be NULL, ready for nsl_keyframes_upsert);
 * status [1] int: 0, or 1 if H_T is not positive definite (sigma_T is then
 * NaN).  Workspace: nsl_covariance_workspace_bytes.
 * ------------------------------------------------------------------------ */
size_t nsl_covariance_workspace_bytes(int c, int p);
int nsl_depth_covariance(int c, int p, const double* C, const double* Et, const double* P,
                         const double* inv_depth, double* sigma_T, double* sigma_d, float* depth_var,
                         int* status, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Rendering (Sec. 3.3: the mapping thread also renders for interactive
 * visualisation).  Uniform samples t_i = t_near + (i+1/2)*dt,
 * i < n_samples <= NSL_RENDER_MAX_SAMPLES; a ray stops before its first sample with
 * T_i < stop_T (0 disables), which also ends its work.  One wave renders
 * one ray; per pixel: rgb, depth_z, var_z (z units) and opacity.
 * ------------------------------------------------------------------------ */
typedef struct nsl_render_config {
  float t_near, dt;
  int32_t n_samples;
  float stop_T;
} nsl_render_config;

#define NSL_RENDER_TILE 64  /* pixels per render tile (one workgroup) */
#define NSL_RENDER_MAX_SAMPLES 1024  /* samples per ray at most */

/* Parameter snapshot operands: the weights of `params` laid out for the
 * MFMA kernels.  A snapshot (params copy + prepared operands) stays valid
 * while training updates the live parameters. */
size_t nsl_field_prepared_bytes(const nsl_field* f);
int nsl_field_prepare(const nsl_field* f, const float* params, void* prepared, hipStream_t stream);

/* One render request as the kernels read it (device memory). */
typedef struct nsl_render_request {
  const float* params;    /* snapshot parameter vector (device) */
  const void* prepared;   /* its nsl_field_prepare output (device) */
  float pose[12];         /* camera-to-world, row-major */
  float intr[4];          /* fx, fy, cx, cy */
  int32_t H, W;
  float* rgb;             /* [H*W,3] */
  float* depth_z;         /* [H*W] */
  float* var_z;           /* [H*W] */
  float* opacity;         /* [H*W] or NULL */
} nsl_render_request;

/* Pixels [first_pixel, first_pixel + n_pixels) of request `request`,
 * n_pixels <= NSL_RENDER_TILE. */
typedef struct nsl_render_tile {
  int32_t request;
  int32_t first_pixel;
  int32_t n_pixels;
} nsl_render_tile;

/* Render n_tiles tiles of n_req requests in one launch (continuous batching:
 * tiles of different requests and snapshots share the launch; each tile
 * uses its own request's snapshot).  requests and tiles are device arrays;
 * tiles naming a request >= n_req or pixels outside the image are skipped.
 * Results per pixel do not depend on which other tiles share the launch. */
int nsl_render_batch(const nsl_field* f, const nsl_render_request* requests, int n_req,
                     const nsl_render_tile* tiles, int n_tiles, const nsl_render_config* cfg,
                     hipStream_t stream);

/* Single image with the live parameters (prepares them in the workspace). */
size_t nsl_render_workspace_bytes(const nsl_field* f, int H, int W,
                                  const nsl_render_config* cfg);
int nsl_render(const nsl_field* f, const float* params, const float* pose, const float* intr,
               int H, int W, const nsl_render_config* cfg, float* rgb, float* depth_z,
               float* var_z, float* opacity, void* workspace, size_t workspace_bytes,
               hipStream_t stream);

/* nsl_render without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The scratch it needs (the prepared
 * MFMA operands and one request record: nsl_render_workspace_bytes, at most
 * 77 056 bytes for the supported field shapes) lives in a static device
 * array of the library, one per GPU, held until the process ends; a field
 * whose scratch would exceed it is rejected with NSL_E_WORKSPACE.  The
 * caller still passes the outputs.  No device memory is allocated, and
 * nothing in the scratch needs to start at zero.  Calls that overlap on one
 * GPU (on different streams, or from different threads) share that array
 * and race: serialise them. */
int nsl_render_noalloc(const nsl_field* f, const float* params, const float* pose, const float* intr,
                       int H, int W, const nsl_render_config* cfg, float* rgb, float* depth_z,
                       float* var_z, float* opacity, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* NSL_H_ */
