// C ABI of the mapping step: validation, layouts, workspace carving and the
// launch sequence.  All device memory comes from the caller.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/nsl.h"
#include "../../include/nsl_peaks.h"
#include "kernels.h"

using namespace nsl;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(NSL_E_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define HIP_TRY(expr, what)                       \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Parameter vectors and shadows are read with 16-byte loads.
bool misaligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) != 0; }

// Sequential carving of a caller buffer into 256-byte aligned pieces.
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* p) : base(static_cast<char*>(p)) {}
  template <class T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += align256(count * sizeof(T));
    return p;
  }
};

constexpr int kBwdBlocks = 256;  // persistent backward grid (one block per CU)

// Buffers of the table-gradient reduction of at most max_samples samples.
RecordBuffers carve_records(Carver& cv, const BinPlan& p) {
  RecordBuffers r{};
  r.de = cv.take<float2>((size_t)p.levels * p.stride);
  r.stride = p.stride;
  r.hist = cv.take<uint32_t>((size_t)p.nbins * p.nunits);
  r.off = cv.take<uint32_t>((size_t)p.nbins * p.nunits);
  r.bin_total = cv.take<uint32_t>((size_t)p.nbins);
  r.bin_start = cv.take<uint32_t>((size_t)p.nbins + 1);
  r.chunk_start = cv.take<uint32_t>((size_t)p.nbins + 1);
  r.chunk_bin = cv.take<uint32_t>((size_t)p.max_chunks);
  // in-bin offsets (2 bytes a record), then values (8 bytes: room for FP32 or BF16 pairs)
  const size_t key_bytes = align256((size_t)p.max_records * 2);
  r.sorted = cv.take<char>(key_bytes + (size_t)p.max_records * 8);
  r.sorted_vals = reinterpret_cast<uint32_t*>(static_cast<char*>(r.sorted) + key_bytes);
  return r;
}

// Records are addressed with 32-bit positions.
bool records_fit(int levels, int64_t max_samples) { return max_samples * 8 * levels < ((int64_t)1 << 32) - 4096; }

struct Profiler {
  bool on = false;
  hipEvent_t ev[NSL_PHASES + 1] = {};
  double ms[NSL_PHASES] = {};
  int steps = 0;
};
Profiler g_prof;

}  // namespace

struct nsl_field {
  nsl_field_config cfg;
  nsl_param_layout lay;
  int shape;
  LevelInfo lv;
  Aabb box;
  WOffsets wo;
};

struct nsl_mapper {
  int max_kf, H, W, grid_res;
  char* storage;
  size_t bytes;
  float *rgb, *depth, *var, *pose, *intr;
  uint32_t* occ;
  std::unordered_map<int32_t, int> slots;
  int used;
};

extern "C" {

const char* nsl_last_error(void) { return g_err.c_str(); }

int nsl_version(void) { return 100; }

int nsl_field_layout(const nsl_field_config* c, nsl_param_layout* out) {
  if (!c || !out) return fail(NSL_E_INVALID, "null argument");
  if (c->levels < 1 || c->levels > NSL_MAX_LEVELS) return fail(NSL_E_INVALID, "levels must be in [1, %d]", NSL_MAX_LEVELS);
  if (c->feat_per_level != 2) return fail(NSL_E_INVALID, "feat_per_level must be 2");
  if (c->log2_table < 4 || c->log2_table > 24) return fail(NSL_E_INVALID, "log2_table must be in [4, 24]");
  if (c->base_res < 1) return fail(NSL_E_INVALID, "base_res must be >= 1");
  if (c->per_level_scale <= 0.0f && (c->max_res <= 0 || c->levels < 2))
    return fail(NSL_E_INVALID, "per_level_scale <= 0 needs max_res > 0 and levels >= 2");
  if (c->n_colour_hidden < 1 || c->n_colour_hidden > 4) return fail(NSL_E_INVALID, "n_colour_hidden must be in [1, 4]");
  if (c->sh_bands < 1 || c->sh_bands > 4) return fail(NSL_E_INVALID, "sh_bands must be in [1, 4]");
  for (int i = 0; i < 3; ++i)
    if (!(c->aabb_max[i] > c->aabb_min[i])) return fail(NSL_E_INVALID, "empty AABB");
  std::memset(out, 0, sizeof *out);
  const int L = c->levels;
  const double b = c->per_level_scale > 0.0f
                       ? (double)c->per_level_scale
                       : std::exp((std::log((double)c->max_res) - std::log((double)c->base_res)) / (L - 1));
  const int64_t T = (int64_t)1 << c->log2_table;
  int64_t off = 0;
  out->levels = L;
  for (int l = 0; l < L; ++l) {
    int n = (int)std::floor((double)c->base_res * std::pow(b, (double)l));
    if (l == L - 1 && c->max_res > 0) n = c->max_res;
    if (n < 1 || n > (1 << 20)) return fail(NSL_E_INVALID, "level %d resolution %d out of range", l, n);
    const int64_t full = (int64_t)(n + 1) * (n + 1) * (n + 1);
    out->res[l] = n;
    out->dense[l] = full <= T;
    out->level_entries[l] = full <= T ? full : T;
    out->level_offset[l] = off;
    off += out->level_entries[l];
  }
  out->table_floats = off * c->feat_per_level;
  auto al = [](int64_t x) { return (x + 63) / 64 * 64; };
  int64_t w = al(out->table_floats);
  std::vector<std::pair<int, int>> dims;
  dims.push_back({2 * L, c->density_hidden});
  dims.push_back({c->density_hidden, c->geo_dim});
  int prev = c->geo_dim + c->sh_bands * c->sh_bands;
  for (int i = 0; i < c->n_colour_hidden; ++i) {
    dims.push_back({prev, c->colour_hidden[i]});
    prev = c->colour_hidden[i];
  }
  dims.push_back({prev, 3});
  out->n_layers = (int)dims.size();
  for (size_t j = 0; j < dims.size(); ++j) {
    out->w_offset[j] = w;
    out->w_in[j] = dims[j].first;
    out->w_out[j] = dims[j].second;
    w = al(w + (int64_t)dims[j].first * dims[j].second);
  }
  out->total_floats = w;
  if (off > kMaxTableEntries) return fail(NSL_E_INVALID, "table too large (more than 2^25 entries)");
  return NSL_OK;
}

int nsl_field_create(const nsl_field_config* c, nsl_field** out) {
  if (!out) return fail(NSL_E_INVALID, "null out");
  *out = nullptr;
  nsl_param_layout lay;
  int rc = nsl_field_layout(c, &lay);
  if (rc) return rc;
  int shape = -1;
  if (c->geo_dim == 16) {
    if (c->levels == 4 && c->density_hidden == 32 && c->n_colour_hidden == 1 && c->colour_hidden[0] == 32 &&
        c->sh_bands == 3)
      shape = kShapeTiny;
    if (c->levels == 16 && c->density_hidden == 64 && c->n_colour_hidden == 2 && c->colour_hidden[0] == 64 &&
        c->colour_hidden[1] == 64 && c->sh_bands == 4)
      shape = kShapeFull;
  }
  if (shape < 0) return fail(NSL_E_INVALID, "unsupported network shape (see nsl.h for the compiled shapes)");
  nsl_field* f = new (std::nothrow) nsl_field;
  if (!f) return fail(NSL_E_INVALID, "out of host memory");
  f->cfg = *c;
  f->lay = lay;
  f->shape = shape;
  std::memset(&f->lv, 0, sizeof f->lv);
  f->lv.levels = c->levels;
  f->lv.table_mask = (uint32_t)((1u << c->log2_table) - 1u);
  for (int l = 0; l < c->levels; ++l) {
    f->lv.res[l] = lay.res[l];
    f->lv.offset[l] = (uint32_t)lay.level_offset[l];
    if (lay.dense[l]) f->lv.dense_bits |= 1u << l;
  }
  for (int i = 0; i < 3; ++i) {
    f->box.lo[i] = c->aabb_min[i];
    f->box.hi[i] = c->aabb_max[i];
    f->box.inv[i] = (float)(1.0 / ((double)c->aabb_max[i] - (double)c->aabb_min[i]));
  }
  for (int j = 0; j < 8; ++j) f->wo.off[j] = j < lay.n_layers ? (int)lay.w_offset[j] : 0;
  *out = f;
  return NSL_OK;
}

void nsl_field_destroy(nsl_field* f) { delete f; }

// ---------------------------------------------------------------------------
// Mapper
// ---------------------------------------------------------------------------

static size_t mapper_carve(nsl_mapper* m, int K, int H, int W, int G, void* base) {
  Carver cv(base);
  const size_t px = (size_t)K * H * W;
  float* rgb = cv.take<float>(px * 3);
  float* depth = cv.take<float>(px);
  float* var = cv.take<float>(px);
  float* pose = cv.take<float>((size_t)K * 12);
  float* intr = cv.take<float>((size_t)K * 4);
  uint32_t* occ = cv.take<uint32_t>(((size_t)G * G * G + 31) / 32);
  if (m) {
    m->rgb = rgb; m->depth = depth; m->var = var; m->pose = pose; m->intr = intr; m->occ = occ;
  }
  return cv.used;
}

size_t nsl_mapper_storage_bytes(int K, int H, int W, int G) {
  if (K < 1 || H < 1 || W < 1 || G < 1) return 0;
  return mapper_carve(nullptr, K, H, W, G, nullptr);
}

int nsl_mapper_create(int K, int H, int W, int G, void* storage, size_t bytes, nsl_mapper** out) {
  if (!out) return fail(NSL_E_INVALID, "null out");
  *out = nullptr;
  if (K < 1 || H < 1 || W < 1 || G < 1) return fail(NSL_E_INVALID, "bad mapper shape");
  if ((int64_t)K * H * W > 0xFFFFFFFFll) return fail(NSL_E_INVALID, "pixel ids exceed 32 bits");
  if (!storage) return fail(NSL_E_INVALID, "null storage");
  if ((reinterpret_cast<uintptr_t>(storage) & 255) != 0) return fail(NSL_E_INVALID, "storage must be 256-byte aligned");
  if (bytes < nsl_mapper_storage_bytes(K, H, W, G)) return fail(NSL_E_WORKSPACE, "mapper storage too small");
  nsl_mapper* m = new (std::nothrow) nsl_mapper;
  if (!m) return fail(NSL_E_INVALID, "out of host memory");
  m->max_kf = K; m->H = H; m->W = W; m->grid_res = G;
  m->storage = static_cast<char*>(storage);
  m->bytes = bytes;
  m->used = 0;
  mapper_carve(m, K, H, W, G, storage);
  *out = m;
  return NSL_OK;
}

void nsl_mapper_destroy(nsl_mapper* m) { delete m; }

int nsl_mapper_count(const nsl_mapper* m) { return m ? m->used : 0; }

int nsl_keyframe_slot(const nsl_mapper* m, int32_t id) {
  if (!m) return -1;
  auto it = m->slots.find(id);
  return it == m->slots.end() ? -1 : it->second;
}

int nsl_keyframes_upsert(nsl_mapper* m, int n, const int32_t* ids, const float* rgb, const float* pose,
                         const float* intr, const float* depth, const float* depth_var, int src_on_host,
                         hipStream_t st) {
  if (!m || !ids || !rgb || !pose || !intr || !depth || !depth_var) return fail(NSL_E_INVALID, "null argument");
  if (n < 0) return fail(NSL_E_INVALID, "negative count");
  int fresh = 0;
  for (int i = 0; i < n; ++i) {
    bool dup = false;
    for (int j = 0; j < i; ++j) dup |= ids[j] == ids[i];
    if (dup) return fail(NSL_E_INVALID, "duplicate id %d in one call", ids[i]);
    if (m->slots.find(ids[i]) == m->slots.end()) ++fresh;
  }
  if (m->used + fresh > m->max_kf) return fail(NSL_E_CAPACITY, "keyframe store full (%d slots)", m->max_kf);
  const hipMemcpyKind kind = src_on_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  const size_t px = (size_t)m->H * m->W;
  for (int i = 0; i < n; ++i) {
    auto it = m->slots.find(ids[i]);
    int slot;
    if (it == m->slots.end()) {
      slot = m->used++;
      m->slots[ids[i]] = slot;
    } else {
      slot = it->second;
    }
    HIP_TRY(hipMemcpyAsync(m->rgb + slot * px * 3, rgb + i * px * 3, px * 3 * sizeof(float), kind, st), "copy rgb");
    HIP_TRY(hipMemcpyAsync(m->depth + slot * px, depth + i * px, px * sizeof(float), kind, st), "copy depth");
    HIP_TRY(hipMemcpyAsync(m->var + slot * px, depth_var + i * px, px * sizeof(float), kind, st), "copy var");
    HIP_TRY(hipMemcpyAsync(m->pose + slot * 12, pose + i * 12, 12 * sizeof(float), kind, st), "copy pose");
    HIP_TRY(hipMemcpyAsync(m->intr + slot * 4, intr + i * 4, 4 * sizeof(float), kind, st), "copy intr");
  }
  return NSL_OK;
}

int nsl_occupancy_set(nsl_mapper* m, const uint32_t* bits, int src_on_host, hipStream_t st) {
  if (!m || !bits) return fail(NSL_E_INVALID, "null argument");
  const size_t words = ((size_t)m->grid_res * m->grid_res * m->grid_res + 31) / 32;
  HIP_TRY(hipMemcpyAsync(m->occ, bits, words * 4, src_on_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st),
          "copy occupancy");
  return NSL_OK;
}

// ---------------------------------------------------------------------------
// Step
// ---------------------------------------------------------------------------

namespace {

struct StepBuffers {
  RayBuffers rb;
  float* wprep;
  void* shadow;  // mixed precision: BF16 operands + FP16 tables
  float* t;
  uint32_t* ray;
  float* sigma;
  float* rgb;
  float* dsigma;
  float* drgb;
  float* partial;
  float* loss_parts;
  void* ecache;
  RecordBuffers rec;
  BinPlan plan;
};

BinPlan plan_of(const nsl_field* f, int64_t max_samples) {
  return bin_plan(f->lv, (uint32_t)(f->lay.table_floats / 2), max_samples);
}

size_t step_carve(const nsl_field* f, int n, int max_samples, bool mixed, bool keep_e, void* base, StepBuffers* b) {
  Carver cv(base);
  StepBuffers s{};
  s.rb.rays = cv.take<float4>(2 * (size_t)n);
  s.rb.target = cv.take<float4>((size_t)n);
  s.rb.prec = cv.take<float>((size_t)n);
  s.rb.counts = cv.take<uint32_t>((size_t)n);
  s.rb.offsets = cv.take<uint32_t>((size_t)n + 1);
  s.rb.stats = cv.take<uint32_t>(4);
  s.rb.block_sums = nullptr;
  s.wprep = cv.take<float>(field_prep_floats(f->shape));
  s.t = cv.take<float>((size_t)max_samples);
  s.ray = cv.take<uint32_t>((size_t)max_samples);
  s.sigma = cv.take<float>((size_t)max_samples);
  s.rgb = cv.take<float>(3 * (size_t)max_samples);
  s.dsigma = cv.take<float>((size_t)max_samples);
  s.drgb = cv.take<float>(3 * (size_t)max_samples);
  s.partial = cv.take<float>((size_t)kBwdBlocks * field_nweights(f->shape));
  s.loss_parts = cv.take<float>(2 * (size_t)n);
  // kept encoding: [levels][max_samples] FP32 or packed BF16 pairs
  const size_t e_pairs = (size_t)max_samples * f->cfg.levels;
  s.ecache = keep_e ? (mixed ? (void*)cv.take<uint32_t>(e_pairs) : (void*)cv.take<float2>(e_pairs)) : nullptr;
  s.shadow = mixed ? cv.take<char>(mixed_shadow_bytes(f->shape, f->lay.table_floats)) : nullptr;
  s.plan = plan_of(f, max_samples);
  s.rec = carve_records(cv, s.plan);
  if (b) *b = s;
  return cv.used;
}

int check_step_cfg(const nsl_step_config* c, const nsl_field* f) {
  if (!c) return fail(NSL_E_INVALID, "null step config");
  if (c->sampler != NSL_SAMPLER_UNIFORM && c->sampler != NSL_SAMPLER_OCCUPANCY) return fail(NSL_E_INVALID, "bad sampler");
  if (!(c->dt > 0.0f) || !(c->t_far >= c->t_near) || !(c->t_near >= 0.0f)) return fail(NSL_E_INVALID, "bad t range or dt");
  if (c->max_samples < 1 || c->max_samples > (1 << 26)) return fail(NSL_E_INVALID, "max_samples must be in [1, 2^26]");
  if (f && !records_fit(f->cfg.levels, c->max_samples))
    return fail(NSL_E_INVALID, "max_samples * 8 * levels must stay below 2^32");
  if (c->sampler == NSL_SAMPLER_UNIFORM && (c->n_uniform < 1 || c->n_uniform > 4096))
    return fail(NSL_E_INVALID, "n_uniform must be in [1, 4096]");
  if (c->sampler == NSL_SAMPLER_OCCUPANCY && (c->max_per_ray < 1 || c->max_per_ray > 4096))
    return fail(NSL_E_INVALID, "max_per_ray must be in [1, 4096]");
  if (c->sampler == NSL_SAMPLER_OCCUPANCY && (double)c->t_far / c->dt > 1e7) return fail(NSL_E_INVALID, "lattice too long");
  if (c->do_adam && c->adam_step < 1) return fail(NSL_E_INVALID, "adam_step must be >= 1");
  if (!(c->loss_scale > 0.0f)) return fail(NSL_E_INVALID, "loss_scale must be > 0");
  if (c->precision != NSL_PRECISION_FP32 && c->precision != NSL_PRECISION_MIXED) return fail(NSL_E_INVALID, "bad precision");
  if (c->keep_encoding != 0 && c->keep_encoding != 1) return fail(NSL_E_INVALID, "keep_encoding must be 0 or 1");
  return NSL_OK;
}

KeyframeStore store_of(const nsl_mapper* m) {
  KeyframeStore k;
  k.rgb = m->rgb; k.depth = m->depth; k.var = m->var; k.pose = m->pose; k.intr = m->intr; k.occ = m->occ;
  k.H = m->H; k.W = m->W; k.K = m->used; k.grid_res = m->grid_res;
  return k;
}

MarchParams march_of(const nsl_field* f, const nsl_step_config* c) {
  MarchParams p;
  p.sampler = c->sampler;
  p.t_near = c->t_near; p.t_far = c->t_far; p.dt = c->dt;
  p.n_uniform = c->n_uniform;
  p.max_per_ray = c->sampler == NSL_SAMPLER_UNIFORM ? c->n_uniform : c->max_per_ray;
  p.max_samples = c->max_samples;
  p.box = f->box;
  return p;
}

int check_ids_range(const nsl_mapper* m, int n) {
  if (n < 0) return fail(NSL_E_INVALID, "negative candidate count");
  if (m->used < 1) return fail(NSL_E_INVALID, "no keyframes in the store");
  return NSL_OK;
}

}  // namespace

size_t nsl_step_workspace_bytes(const nsl_field* f, const nsl_step_config* c, int n) {
  if (!f || !c || n < 0 || c->max_samples < 1 || !records_fit(f->cfg.levels, c->max_samples)) return 0;
  return step_carve(f, n, c->max_samples, c->precision == NSL_PRECISION_MIXED, c->keep_encoding != 0, nullptr,
                    nullptr);
}

static int run_march(nsl_mapper* m, const nsl_field* f, const nsl_step_config* c, const uint32_t* ids, int n,
                     StepBuffers& b, hipStream_t st) {
  const KeyframeStore kf = store_of(m);
  const MarchParams mp = march_of(f, c);
  HIP_TRY(march_rays(kf, mp, ids, n, b.rb, st), "march count");
  HIP_TRY(march_emit(kf, mp, ids, n, b.rb, b.t, b.ray, st), "march emit");
  return NSL_OK;
}

int nsl_train_step(nsl_mapper* m, const nsl_field* f, float* params, float* grads, float* adam_m, float* adam_v,
                   const nsl_step_config* c, const uint32_t* ids, int n, void* ws, size_t ws_bytes,
                   float* loss_out, nsl_step_stats* stats_out, float* ray_out, hipStream_t st) {
  if (!m || !f || !params || !grads || !ids || !ws || !loss_out) return fail(NSL_E_INVALID, "null argument");
  int rc = check_step_cfg(c, f);
  if (rc) return rc;
  if ((rc = check_ids_range(m, n))) return rc;
  if (c->do_adam && (!adam_m || !adam_v)) return fail(NSL_E_INVALID, "adam needs m and v");
  if (misaligned(params) || misaligned(grads) || (c->do_adam && (misaligned(adam_m) || misaligned(adam_v))))
    return fail(NSL_E_INVALID, "params, grads and Adam moments must be 16-byte aligned");
  if (c->sampler == NSL_SAMPLER_OCCUPANCY && m->grid_res < 1) return fail(NSL_E_INVALID, "no occupancy grid");
  if (ws_bytes < nsl_step_workspace_bytes(f, c, n)) return fail(NSL_E_WORKSPACE, "step workspace too small");
  StepBuffers b;
  const bool mixed = c->precision == NSL_PRECISION_MIXED;
  step_carve(f, n, c->max_samples, mixed, c->keep_encoding != 0, ws, &b);
  b.rec.de_bf16 = mixed;  // the mixed backward stores dL/de as BF16 pairs
  if (stats_out) b.rb.stats = reinterpret_cast<uint32_t*>(stats_out);
  b.rb.loss = loss_out;
  const int64_t total = f->lay.total_floats;
  const bool prof = g_prof.on;
  auto mark = [&](int i) -> hipError_t { return prof ? hipEventRecord(g_prof.ev[i], st) : hipSuccess; };
  HIP_TRY(mark(0), "profile event");
  // with the encoding kept, the encoding kernel also counts the
  // table-gradient records per bin and unit
  const bool counted = c->keep_encoding != 0 && b.plan.bl.max_level_bins <= kEncodeLevelBins;
  // the mixed step prepares (FP16 table copy, gradient clearing,
  // overflow-flag reset, BF16 operands) and counts the candidates' samples in
  // one launch; profiled steps keep them apart to time the two phases
  const bool fused_count = mixed && !prof;
  if (fused_count) {
    HIP_TRY(mixed_prepare_count(f->shape, params, f->wo, f->lay.table_floats, b.shadow,
                                c->zero_grads ? grads : nullptr, total, c->scale_state ? c->scale_state + 3 : nullptr,
                                store_of(m), march_of(f, c), ids, n, b.rb, st),
            "prep mixed and ray setup");
  } else if (mixed) {
    HIP_TRY(mixed_prepare(f->shape, params, f->wo, f->lay.table_floats, b.shadow, c->zero_grads ? grads : nullptr,
                          total, c->scale_state ? c->scale_state + 3 : nullptr, st),
            "prep mixed");
  } else {
    if (c->scale_state) HIP_TRY(scale_begin(c->scale_state, st), "loss scale");
    // the table part is overwritten by the table-gradient reduction
    const int64_t z0 = f->lay.table_floats & ~(int64_t)3;
    if (c->zero_grads) HIP_TRY(fill_zero(grads + z0, total - z0, st), "zero grads");
    HIP_TRY(field_prep(f->shape, params, f->wo, b.wprep, st), "prep weights");
  }
  HIP_TRY(mark(1), "profile event");
  if (fused_count) {
    const MarchParams mp = march_of(f, c);
    HIP_TRY(march_scan(mp, n, b.rb, st), "march scan");
    HIP_TRY(march_emit(store_of(m), mp, ids, n, b.rb, b.t, b.ray, st), "march emit");
  } else if ((rc = run_march(m, f, c, ids, n, b, st))) {
    return rc;
  }
  HIP_TRY(mark(2), "profile event");

  FieldArgs fa{params, b.wprep, f->lv};
  SampleSrc src{};
  src.t = b.t; src.ray = b.ray; src.rays = b.rb.rays; src.box = f->box; src.n_dev = b.rb.stats + 1; src.n = 0;
  src.ecache = b.ecache;
  src.ecache_stride = c->max_samples;
  if (src.ecache) {
    uint32_t* hist = counted ? b.rec.hist : nullptr;
    if (mixed)
      HIP_TRY(mixed_encode(f->shape, f->lv, b.shadow, src, c->max_samples, hist, b.plan.bl, st), "encoding");
    else
      HIP_TRY(field_encode(f->shape, fa, src, c->max_samples, hist, b.plan.bl, st), "encoding");
  }
  HIP_TRY(mark(3), "profile event");
  // with the records counted, the table-gradient column scan and bin starts
  // ride along the forward and the compositing launches
  BinPrep bp{};
  if (counted) {
    bp.rb = b.rec;
    bp.nunits = b.plan.nunits;
    bp.nbins = b.plan.nbins;
    bp.chunk = bin_chunk(b.plan, mixed);
    bp.split = bin_split(b.plan);
  }
  const BinPrep* prescan = counted && b.plan.nbins > 0 && b.plan.nunits > 0 ? &bp : nullptr;
  if (mixed)
    HIP_TRY(mixed_forward(f->shape, f->lv, b.shadow, src, c->max_samples, b.sigma, b.rgb, st, prescan),
            "field forward");
  else
    HIP_TRY(field_forward(f->shape, fa, src, c->max_samples, b.sigma, b.rgb, st, prescan), "field forward");
  HIP_TRY(mark(4), "profile event");

  CompositeIO io{};
  io.sigma = b.sigma; io.rgb = b.rgb; io.t = b.t; io.off = b.rb.offsets; io.counts = b.rb.counts;
  io.max_samples = c->max_samples; io.R = n; io.delta = c->dt; io.stop_T = 0.0f; io.out6 = nullptr;
  LossIO lo{};
  lo.target = b.rb.target; lo.prec = b.rb.prec; lo.rays = b.rb.rays; lo.stats = b.rb.stats;
  lo.lambda_d = c->lambda_d; lo.loss_scale = c->loss_scale; lo.scale_dev = c->scale_state;
  lo.loss = loss_out; lo.parts = b.loss_parts; lo.ray_out = ray_out;
  HIP_TRY(composite_loss_backward(io, lo, b.dsigma, b.drgb, st, prescan), "composite");
  HIP_TRY(mark(5), "profile event");

  if (mixed)
    HIP_TRY(mixed_backward(f->shape, f->lv, b.shadow, src, kBwdBlocks, b.dsigma, b.drgb, b.rec, b.partial, f->wo,
                           grads, st),
            "field backward");
  else
    HIP_TRY(field_backward(f->shape, fa, src, kBwdBlocks, b.dsigma, b.drgb, b.rec, b.partial, f->wo, grads, st),
            "field backward");
  HIP_TRY(mark(6), "profile event");
  float* overflow = c->scale_state ? c->scale_state + 3 : nullptr;  // set by the two gradient writers
  // the weight-gradient and loss sums ride along the scatter's placement (or,
  // when it scans the counts itself, its column scan)
  const WeightSum wsum{f->shape, b.partial, kBwdBlocks, f->wo, grads, overflow,
                     LossSum{b.loss_parts, n, c->lambda_d, loss_out}};
  HIP_TRY(bin_scatter(b.plan, b.rec, src, f->lv, mixed, c->zero_grads != 0, grads, overflow, st, counted, &wsum,
                      prescan != nullptr),
          "table, weight and loss gradients");
  HIP_TRY(mark(7), "profile event");
  HIP_TRY(mark(8), "profile event");
  if (c->do_adam)
    HIP_TRY(adam_update(params, grads, adam_m, adam_v, total, c->lr, c->beta1, c->beta2, c->eps, c->adam_step,
                        1.0f / c->loss_scale, c->scale_state, st),
            "adam");
  if (c->scale_state) HIP_TRY(scale_end(c->scale_state, st), "loss scale");
  HIP_TRY(mark(9), "profile event");
  if (prof) {
    HIP_TRY(hipEventSynchronize(g_prof.ev[NSL_PHASES]), "profile sync");
    for (int i = 0; i < NSL_PHASES; ++i) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, g_prof.ev[i], g_prof.ev[i + 1]), "profile elapsed");
      g_prof.ms[i] += ms;
    }
    ++g_prof.steps;
  }
  return NSL_OK;
}

int nsl_march(nsl_mapper* m, const nsl_field* f, const nsl_step_config* c, const uint32_t* ids, int n, void* ws,
              size_t ws_bytes, uint32_t* counts, uint32_t* offsets, float* t, uint32_t* ray,
              nsl_step_stats* stats_out, hipStream_t st) {
  if (!m || !f || !ids || !ws || !counts || !offsets || !t || !ray) return fail(NSL_E_INVALID, "null argument");
  int rc = check_step_cfg(c, f);
  if (rc) return rc;
  if ((rc = check_ids_range(m, n))) return rc;
  if (ws_bytes < nsl_step_workspace_bytes(f, c, n)) return fail(NSL_E_WORKSPACE, "march workspace too small");
  StepBuffers b;
  step_carve(f, n, c->max_samples, c->precision == NSL_PRECISION_MIXED, c->keep_encoding != 0, ws, &b);
  b.rb.counts = counts;
  b.rb.offsets = offsets;
  b.t = t;
  b.ray = ray;
  if (stats_out) b.rb.stats = reinterpret_cast<uint32_t*>(stats_out);
  b.rb.loss = nullptr;
  return run_march(m, f, c, ids, n, b, st);
}

int nsl_profile_enable(int on) {
  if (on && !g_prof.on) {
    for (auto& e : g_prof.ev) HIP_TRY(hipEventCreate(&e), "create profile event");
  }
  if (!on && g_prof.on) {
    for (auto& e : g_prof.ev) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
  }
  g_prof.on = on != 0;
  for (double& x : g_prof.ms) x = 0.0;
  g_prof.steps = 0;
  return NSL_OK;
}

int nsl_profile_read(double* ms, int* n_steps) {
  if (!ms || !n_steps) return fail(NSL_E_INVALID, "null argument");
  for (int i = 0; i < NSL_PHASES; ++i) ms[i] = g_prof.ms[i];
  *n_steps = g_prof.steps;
  return NSL_OK;
}

// Field-level workspace: MFMA operands, per-block weight-gradient partials and
// the table-gradient buffers of S samples (the same for either precision).
struct FieldWs {
  float* wprep;
  float* partial;
  RecordBuffers rec;
  BinPlan plan;
};

static size_t field_carve(const nsl_field* f, int S, void* base, FieldWs* w) {
  Carver cv(base);
  FieldWs x{};
  x.wprep = cv.take<float>(field_prep_floats(f->shape));
  x.partial = cv.take<float>((size_t)kBwdBlocks * field_nweights(f->shape));
  x.plan = plan_of(f, S);
  x.rec = carve_records(cv, x.plan);
  if (w) *w = x;
  return cv.used;
}

size_t nsl_field_workspace_bytes(const nsl_field* f, int S) {
  if (!f || S < 0 || !records_fit(f->cfg.levels, S)) return 0;
  return field_carve(f, S, nullptr, nullptr);
}

static int field_common(const nsl_field* f, const float* params, const float* xn, const float* dirs, int S,
                        void* ws, size_t ws_bytes, bool mixed, FieldWs& w, SampleSrc& src) {
  if (!f || !xn || !dirs || !ws) return fail(NSL_E_INVALID, "null argument");
  if (!mixed && !params) return fail(NSL_E_INVALID, "null params");
  if (S < 0) return fail(NSL_E_INVALID, "negative sample count");
  if (!records_fit(f->cfg.levels, S)) return fail(NSL_E_INVALID, "S * 8 * levels must stay below 2^32");
  if (ws_bytes < nsl_field_workspace_bytes(f, S)) return fail(NSL_E_WORKSPACE, "field workspace too small");
  field_carve(f, S, ws, &w);
  src = SampleSrc{};
  src.xn = xn; src.dir = dirs; src.box = f->box; src.n = S; src.n_dev = nullptr;
  return NSL_OK;
}

int nsl_field_fwd(const nsl_field* f, const float* params, const float* xn, const float* dirs, int S, float* sigma,
                  float* rgb, void* ws, size_t ws_bytes, hipStream_t st) {
  if (!sigma || !rgb) return fail(NSL_E_INVALID, "null output");
  if (misaligned(params)) return fail(NSL_E_INVALID, "params must be 16-byte aligned");
  FieldWs w;
  SampleSrc src;
  int rc = field_common(f, params, xn, dirs, S, ws, ws_bytes, false, w, src);
  if (rc) return rc;
  HIP_TRY(field_prep(f->shape, params, f->wo, w.wprep, st), "prep weights");
  FieldArgs fa{params, w.wprep, f->lv};
  HIP_TRY(field_forward(f->shape, fa, src, S, sigma, rgb, st), "field forward");
  return NSL_OK;
}

int nsl_field_bwd(const nsl_field* f, const float* params, const float* xn, const float* dirs, int S,
                  const float* dsigma, const float* drgb, float* grads, void* ws, size_t ws_bytes, hipStream_t st) {
  if (!dsigma || !drgb || !grads) return fail(NSL_E_INVALID, "null argument");
  if (misaligned(params) || misaligned(grads)) return fail(NSL_E_INVALID, "params and grads must be 16-byte aligned");
  FieldWs w;
  SampleSrc src;
  int rc = field_common(f, params, xn, dirs, S, ws, ws_bytes, false, w, src);
  if (rc) return rc;
  HIP_TRY(field_prep(f->shape, params, f->wo, w.wprep, st), "prep weights");
  FieldArgs fa{params, w.wprep, f->lv};
  HIP_TRY(field_backward(f->shape, fa, src, kBwdBlocks, dsigma, drgb, w.rec, w.partial, f->wo, grads, st),
          "field backward");
  HIP_TRY(field_dw_reduce(f->shape, w.partial, kBwdBlocks, f->wo, grads, nullptr, nullptr, st), "weight gradient");
  HIP_TRY(bin_scatter(w.plan, w.rec, src, f->lv, false, false, grads, nullptr, st), "table gradient");
  return NSL_OK;
}

size_t nsl_mixed_shadow_bytes(const nsl_field* f) {
  return f ? mixed_shadow_bytes(f->shape, f->lay.table_floats) : 0;
}

int nsl_field_prepare_mixed(const nsl_field* f, const float* params, void* shadow, hipStream_t st) {
  if (!f || !params || !shadow) return fail(NSL_E_INVALID, "null argument");
  if (misaligned(params) || misaligned(shadow)) return fail(NSL_E_INVALID, "params and shadow must be 16-byte aligned");
  HIP_TRY(mixed_prepare(f->shape, params, f->wo, f->lay.table_floats, shadow, nullptr, 0, nullptr, st),
          "prepare mixed");
  return NSL_OK;
}

int nsl_field_fwd_mixed(const nsl_field* f, const void* shadow, const float* xn, const float* dirs, int S,
                        float* sigma, float* rgb, hipStream_t st) {
  if (!f || !shadow || !xn || !dirs || !sigma || !rgb) return fail(NSL_E_INVALID, "null argument");
  if (misaligned(shadow)) return fail(NSL_E_INVALID, "shadow must be 16-byte aligned");
  if (S < 0) return fail(NSL_E_INVALID, "negative sample count");
  SampleSrc src{};
  src.xn = xn; src.dir = dirs; src.box = f->box; src.n = S;
  HIP_TRY(mixed_forward(f->shape, f->lv, shadow, src, S, sigma, rgb, st), "field forward (mixed)");
  return NSL_OK;
}

int nsl_field_bwd_mixed(const nsl_field* f, const void* shadow, const float* xn, const float* dirs, int S,
                        const float* dsigma, const float* drgb, float* grads, void* ws, size_t ws_bytes,
                        hipStream_t st) {
  if (!f || !shadow || !dsigma || !drgb || !grads) return fail(NSL_E_INVALID, "null argument");
  if (misaligned(shadow) || misaligned(grads)) return fail(NSL_E_INVALID, "shadow and grads must be 16-byte aligned");
  FieldWs w;
  SampleSrc src;
  int rc = field_common(f, nullptr, xn, dirs, S, ws, ws_bytes, true, w, src);
  if (rc) return rc;
  w.rec.de_bf16 = true;  // the mixed backward stores dL/de as BF16 pairs
  HIP_TRY(mixed_backward(f->shape, f->lv, shadow, src, kBwdBlocks, dsigma, drgb, w.rec, w.partial, f->wo, grads, st),
          "field backward (mixed)");
  HIP_TRY(field_dw_reduce(f->shape, w.partial, kBwdBlocks, f->wo, grads, nullptr, nullptr, st), "weight gradient");
  HIP_TRY(bin_scatter(w.plan, w.rec, src, f->lv, true, false, grads, nullptr, st), "table gradient");
  return NSL_OK;
}

int nsl_composite_fwd(const float* sigma, const float* rgb, const float* t, const uint32_t* off, int R, float delta,
                      float stop_T, float* out, hipStream_t st) {
  if (!sigma || !rgb || !t || !off || !out) return fail(NSL_E_INVALID, "null argument");
  if (R < 0) return fail(NSL_E_INVALID, "negative ray count");
  if (!(delta > 0.0f) || !(stop_T >= 0.0f)) return fail(NSL_E_INVALID, "bad delta or stop_T");
  CompositeIO io{};
  io.sigma = sigma; io.rgb = rgb; io.t = t; io.off = off; io.counts = nullptr; io.R = R; io.delta = delta;
  io.stop_T = stop_T; io.out6 = out;
  HIP_TRY(composite_forward(io, st), "composite forward");
  return NSL_OK;
}

int nsl_composite_bwd(const float* sigma, const float* rgb, const float* t, const uint32_t* off, int R, float delta,
                      const float* g_rgb, const float* g_depth, const float* g_var, const float* g_opacity,
                      float* g_sigma, float* g_rgb_s, hipStream_t st) {
  if (!sigma || !rgb || !t || !off || !g_sigma || !g_rgb_s) return fail(NSL_E_INVALID, "null argument");
  if (R < 0) return fail(NSL_E_INVALID, "negative ray count");
  if (!(delta > 0.0f)) return fail(NSL_E_INVALID, "bad delta");
  CompositeIO io{};
  io.sigma = sigma; io.rgb = rgb; io.t = t; io.off = off; io.counts = nullptr; io.R = R; io.delta = delta;
  io.stop_T = 0.0f;
  HIP_TRY(composite_backward(io, g_rgb, g_depth, g_var, g_opacity, g_sigma, g_rgb_s, st), "composite backward");
  return NSL_OK;
}

size_t nsl_loss_workspace_bytes(int R) { return R < 0 ? 0 : align256(2 * sizeof(float) * (size_t)R); }

static int check_loss_args(const float* out6, int R, const float* rgb_target, const float* depth_z,
                           const float* depth_var_z, const float* ray_scale) {
  if (!out6 || !rgb_target || !depth_z || !depth_var_z || !ray_scale) return fail(NSL_E_INVALID, "null argument");
  if (R < 1) return fail(NSL_E_INVALID, "the loss needs at least one ray");
  return NSL_OK;
}

int nsl_loss_fwd(const float* out6, int R, const float* rgb_target, const float* depth_z, const float* depth_var_z,
                 const float* ray_scale, float lambda_d, float* loss_out, uint32_t* n_masked, void* ws,
                 size_t ws_bytes, hipStream_t st) {
  int rc = check_loss_args(out6, R, rgb_target, depth_z, depth_var_z, ray_scale);
  if (rc) return rc;
  if (!loss_out || !ws) return fail(NSL_E_INVALID, "null argument");
  if (ws_bytes < nsl_loss_workspace_bytes(R)) return fail(NSL_E_WORKSPACE, "loss workspace too small");
  float* parts = static_cast<float*>(ws);
  if (n_masked) HIP_TRY(hipMemsetAsync(n_masked, 0, sizeof(uint32_t), st), "clear mask count");
  HIP_TRY(loss_terms(out6, R, rgb_target, depth_z, depth_var_z, ray_scale, lambda_d, nullptr, parts, nullptr,
                     n_masked, st),
          "loss terms");
  const LossSum ls{parts, R, lambda_d, loss_out};
  HIP_TRY(loss_sum(ls, st), "loss sum");
  return NSL_OK;
}

int nsl_loss_bwd(const float* out6, int R, const float* rgb_target, const float* depth_z, const float* depth_var_z,
                 const float* ray_scale, float lambda_d, const float* g_loss, float* g_out6, hipStream_t st) {
  int rc = check_loss_args(out6, R, rgb_target, depth_z, depth_var_z, ray_scale);
  if (rc) return rc;
  if (!g_out6) return fail(NSL_E_INVALID, "null argument");
  HIP_TRY(loss_terms(out6, R, rgb_target, depth_z, depth_var_z, ray_scale, lambda_d, g_loss, nullptr, g_out6,
                     nullptr, st),
          "loss seeds");
  return NSL_OK;
}

// ---------------------------------------------------------------------------
// Encoding and its adjoint on their own
// ---------------------------------------------------------------------------

static int check_encode_args(const nsl_field* f, const float* xn, int S) {
  if (!f || !xn) return fail(NSL_E_INVALID, "null argument");
  if (S < 0) return fail(NSL_E_INVALID, "negative sample count");
  if (!records_fit(f->cfg.levels, S)) return fail(NSL_E_INVALID, "S * 8 * levels must stay below 2^32");
  return NSL_OK;
}

int nsl_encode_fwd(const nsl_field* f, const float* params, const float* xn, int S, float* e_out, hipStream_t st) {
  int rc = check_encode_args(f, xn, S);
  if (rc) return rc;
  if (!params || !e_out) return fail(NSL_E_INVALID, "null argument");
  SampleSrc src{};
  src.xn = xn; src.box = f->box; src.n = S; src.ecache = e_out; src.ecache_stride = S;
  FieldArgs fa{params, nullptr, f->lv};
  HIP_TRY(field_encode(f->shape, fa, src, S, nullptr, BinLevels{}, st), "encoding");
  return NSL_OK;
}

int nsl_encode_fwd_mixed(const nsl_field* f, const void* shadow, const float* xn, int S, uint32_t* e_out,
                         hipStream_t st) {
  int rc = check_encode_args(f, xn, S);
  if (rc) return rc;
  if (!shadow || !e_out) return fail(NSL_E_INVALID, "null argument");
  if (misaligned(shadow)) return fail(NSL_E_INVALID, "shadow must be 16-byte aligned");
  SampleSrc src{};
  src.xn = xn; src.box = f->box; src.n = S; src.ecache = e_out; src.ecache_stride = S;
  HIP_TRY(mixed_encode(f->shape, f->lv, shadow, src, S, nullptr, BinLevels{}, st), "encoding (mixed)");
  return NSL_OK;
}

static size_t encode_bwd_carve(const nsl_field* f, int S, void* base, BinPlan* plan, RecordBuffers* rec) {
  Carver cv(base);
  const BinPlan p = plan_of(f, S);
  RecordBuffers r = carve_records(cv, p);
  if (plan) *plan = p;
  if (rec) *rec = r;
  return cv.used;
}

size_t nsl_encode_bwd_workspace_bytes(const nsl_field* f, int S) {
  if (!f || S < 0 || !records_fit(f->cfg.levels, S)) return 0;
  return encode_bwd_carve(f, S, nullptr, nullptr, nullptr);
}

int nsl_encode_bwd(const nsl_field* f, const float* xn, int S, const float* de, int precision, int overwrite,
                   float* grads, void* ws, size_t ws_bytes, hipStream_t st) {
  int rc = check_encode_args(f, xn, S);
  if (rc) return rc;
  if (!de || !grads || !ws) return fail(NSL_E_INVALID, "null argument");
  if (precision != NSL_PRECISION_FP32 && precision != NSL_PRECISION_MIXED) return fail(NSL_E_INVALID, "bad precision");
  if (misaligned(grads) || misaligned(de)) return fail(NSL_E_INVALID, "grads and de must be 16-byte aligned");
  if (ws_bytes < nsl_encode_bwd_workspace_bytes(f, S)) return fail(NSL_E_WORKSPACE, "encode workspace too small");
  BinPlan plan;
  RecordBuffers rec;
  encode_bwd_carve(f, S, ws, &plan, &rec);
  rec.de = const_cast<float2*>(reinterpret_cast<const float2*>(de));  // read only
  rec.stride = S;
  SampleSrc src{};
  src.xn = xn; src.box = f->box; src.n = S;
  if (S == 0) {  // nothing to scatter; an overwrite still leaves the table gradient at zero
    if (overwrite) HIP_TRY(fill_zero(grads, f->lay.table_floats, st), "clear table gradient");
    return NSL_OK;
  }
  HIP_TRY(bin_scatter(plan, rec, src, f->lv, precision == NSL_PRECISION_MIXED, overwrite != 0, grads, nullptr, st),
          "table gradient");
  return NSL_OK;
}

// The MLP alone on a given level-major FP32 encoding (the kept-encoding path
// of the field kernels).
static int mlp_common(const nsl_field* f, const float* params, const float* enc, const float* dirs, int S, void* ws,
                      size_t ws_bytes, FieldWs& w, SampleSrc& src) {
  if (!f || !params || !enc || !dirs || !ws) return fail(NSL_E_INVALID, "null argument");
  if (S < 0) return fail(NSL_E_INVALID, "negative sample count");
  if (!records_fit(f->cfg.levels, S)) return fail(NSL_E_INVALID, "S * 8 * levels must stay below 2^32");
  if (misaligned(params) || misaligned(enc)) return fail(NSL_E_INVALID, "params and enc must be 16-byte aligned");
  if (ws_bytes < nsl_field_workspace_bytes(f, S)) return fail(NSL_E_WORKSPACE, "field workspace too small");
  field_carve(f, S, ws, &w);
  src = SampleSrc{};
  src.dir = dirs; src.box = f->box; src.n = S; src.n_dev = nullptr;
  src.ecache = const_cast<float*>(enc);  // read only
  src.ecache_stride = S;
  return NSL_OK;
}

int nsl_mlp_fwd(const nsl_field* f, const float* params, const float* enc, const float* dirs, int S, float* sigma,
                float* rgb, void* ws, size_t ws_bytes, hipStream_t st) {
  if (!sigma || !rgb) return fail(NSL_E_INVALID, "null output");
  FieldWs w;
  SampleSrc src;
  int rc = mlp_common(f, params, enc, dirs, S, ws, ws_bytes, w, src);
  if (rc) return rc;
  HIP_TRY(field_prep(f->shape, params, f->wo, w.wprep, st), "prep weights");
  FieldArgs fa{params, w.wprep, f->lv};
  HIP_TRY(field_forward(f->shape, fa, src, S, sigma, rgb, st), "mlp forward");
  return NSL_OK;
}

int nsl_mlp_bwd(const nsl_field* f, const float* params, const float* enc, const float* dirs, int S,
                const float* dsigma, const float* drgb, float* grads, float* d_enc, void* ws, size_t ws_bytes,
                hipStream_t st) {
  if (!dsigma || !drgb || !grads || !d_enc) return fail(NSL_E_INVALID, "null argument");
  if (misaligned(grads) || misaligned(d_enc)) return fail(NSL_E_INVALID, "grads and d_enc must be 16-byte aligned");
  FieldWs w;
  SampleSrc src;
  int rc = mlp_common(f, params, enc, dirs, S, ws, ws_bytes, w, src);
  if (rc) return rc;
  HIP_TRY(field_prep(f->shape, params, f->wo, w.wprep, st), "prep weights");
  FieldArgs fa{params, w.wprep, f->lv};
  RecordBuffers rec = w.rec;
  rec.de = reinterpret_cast<float2*>(d_enc);
  rec.stride = S;
  rec.de_bf16 = false;
  HIP_TRY(field_backward(f->shape, fa, src, kBwdBlocks, dsigma, drgb, rec, w.partial, f->wo, grads, st),
          "mlp backward");
  HIP_TRY(field_dw_reduce(f->shape, w.partial, kBwdBlocks, f->wo, grads, nullptr, nullptr, st), "weight gradient");
  return NSL_OK;
}

// ---------------------------------------------------------------------------
// Machine-peak probes
// ---------------------------------------------------------------------------

int nsl_peak_copy(const void* src, void* dst, size_t bytes, hipStream_t st) {
  if (!src || !dst) return fail(NSL_E_INVALID, "null argument");
  if (bytes % 16 || misaligned(src) || misaligned(dst)) return fail(NSL_E_INVALID, "16-byte aligned copies only");
  HIP_TRY(peak_copy(src, dst, bytes, st), "peak copy");
  return NSL_OK;
}

int nsl_peak_gather(const uint32_t* table, int log2_entries, uint32_t* out, int n_threads, int loads,
                    hipStream_t st) {
  if (!table || !out) return fail(NSL_E_INVALID, "null argument");
  if (log2_entries < 4 || log2_entries > 30 || n_threads < 0 || n_threads % 256 || loads < 16 || loads % 16)
    return fail(NSL_E_INVALID, "bad gather shape");
  HIP_TRY(peak_gather(table, log2_entries, out, n_threads, loads, st), "peak gather");
  return NSL_OK;
}

int nsl_peak_mfma(int bf16, float* out, int n_workgroups, int iters, hipStream_t st) {
  if (!out) return fail(NSL_E_INVALID, "null argument");
  if (n_workgroups < 0 || iters < 1) return fail(NSL_E_INVALID, "bad mfma loop shape");
  HIP_TRY(peak_mfma(bf16 != 0, out, n_workgroups, iters, st), "peak mfma");
  return NSL_OK;
}

int nsl_adam(float* p, float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps, int step,
             float grad_scale, hipStream_t st) {
  if (!p || !g || !m || !v) return fail(NSL_E_INVALID, "null argument");
  if (misaligned(p) || misaligned(g) || misaligned(m) || misaligned(v))
    return fail(NSL_E_INVALID, "params, grads and moments must be 16-byte aligned");
  if (n < 0 || step < 1) return fail(NSL_E_INVALID, "bad count or step");
  HIP_TRY(adam_update(p, g, m, v, n, lr, b1, b2, eps, step, grad_scale, nullptr, st), "adam");
  return NSL_OK;
}

// ---------------------------------------------------------------------------
// Render
// ---------------------------------------------------------------------------

static int check_render_cfg(const nsl_render_config* c) {
  if (!c) return fail(NSL_E_INVALID, "null render config");
  if (c->n_samples < 1 || c->n_samples > kRenderMaxSamples)
    return fail(NSL_E_INVALID, "n_samples must be in [1, %d]", kRenderMaxSamples);
  if (!(c->dt > 0.0f) || !(c->stop_T >= 0.0f) || !(c->t_near >= 0.0f)) return fail(NSL_E_INVALID, "bad render config");
  return NSL_OK;
}

static RenderParams render_params(const nsl_render_config* c) {
  RenderParams rp;
  rp.t_near = c->t_near;
  rp.dt = c->dt;
  rp.stop_T = c->stop_T;
  rp.n_samples = c->n_samples;
  return rp;
}

size_t nsl_field_prepared_bytes(const nsl_field* f) {
  return f ? align256(field_prep_floats(f->shape) * sizeof(float)) : 0;
}

int nsl_field_prepare(const nsl_field* f, const float* params, void* prepared, hipStream_t st) {
  if (!f || !params || !prepared) return fail(NSL_E_INVALID, "null argument");
  if (misaligned(params)) return fail(NSL_E_INVALID, "params must be 16-byte aligned");
  HIP_TRY(field_prep(f->shape, params, f->wo, static_cast<float*>(prepared), st), "prepare");
  return NSL_OK;
}

int nsl_render_batch(const nsl_field* f, const nsl_render_request* reqs, int n_req, const nsl_render_tile* tiles,
                     int n_tiles, const nsl_render_config* c, hipStream_t st) {
  if (!f || !reqs || !tiles) return fail(NSL_E_INVALID, "null argument");
  if (n_req < 0 || n_tiles < 0) return fail(NSL_E_INVALID, "negative count");
  int rc = check_render_cfg(c);
  if (rc) return rc;
  HIP_TRY(render_tiles(f->shape, f->lv, f->box, reqs, n_req, tiles, n_tiles, render_params(c), st), "render");
  return NSL_OK;
}

size_t nsl_render_workspace_bytes(const nsl_field* f, int H, int W, const nsl_render_config* c) {
  if (!f || !c || H < 1 || W < 1) return 0;
  return nsl_field_prepared_bytes(f) + align256(sizeof(nsl_render_request));
}

static int check_render_args(const nsl_field* f, const float* params, const float* pose, const float* intr, int H,
                             int W, const nsl_render_config* c, const float* rgb, const float* depth,
                             const float* var) {
  if (!f || !params || !pose || !intr || !c || !rgb || !depth || !var) return fail(NSL_E_INVALID, "null argument");
  if (H < 1 || W < 1 || (int64_t)H * W > (1 << 30)) return fail(NSL_E_INVALID, "bad image size");
  return check_render_cfg(c);
}

// One image into rgb/depth/var/opacity: the parameters' MFMA operands and the
// request record are written to ws (nsl_render_workspace_bytes).
static int render_image(const nsl_field* f, const float* params, const float* pose, const float* intr, int H, int W,
                        const nsl_render_config* c, float* rgb, float* depth, float* var, float* opacity, void* ws,
                        hipStream_t st) {
  char* base = static_cast<char*>(ws);
  void* prepared = base;
  nsl_render_request* dev_req = reinterpret_cast<nsl_render_request*>(base + nsl_field_prepared_bytes(f));
  int rc = nsl_field_prepare(f, params, prepared, st);
  if (rc) return rc;
  nsl_render_request r;
  r.params = params;
  r.prepared = prepared;
  std::memset(r.pose, 0, sizeof r.pose);
  std::memset(r.intr, 0, sizeof r.intr);
  r.H = H;
  r.W = W;
  r.rgb = rgb;
  r.depth_z = depth;
  r.var_z = var;
  r.opacity = opacity;
  HIP_TRY(store_request(&r, pose, intr, dev_req, st), "store request");
  const int n_tiles = (H * W + NSL_RENDER_TILE - 1) / NSL_RENDER_TILE;
  HIP_TRY(render_tiles(f->shape, f->lv, f->box, dev_req, 1, nullptr, n_tiles, render_params(c), st), "render");
  return NSL_OK;
}

int nsl_render(const nsl_field* f, const float* params, const float* pose, const float* intr, int H, int W,
               const nsl_render_config* c, float* rgb, float* depth, float* var, float* opacity, void* ws,
               size_t ws_bytes, hipStream_t st) {
  int rc = check_render_args(f, params, pose, intr, H, W, c, rgb, depth, var);
  if (rc) return rc;
  if (!ws) return fail(NSL_E_INVALID, "null argument");
  if (ws_bytes < nsl_render_workspace_bytes(f, H, W, c)) return fail(NSL_E_WORKSPACE, "render workspace too small");
  return render_image(f, params, pose, intr, H, W, c, rgb, depth, var, opacity, ws, st);
}

int nsl_render_noalloc(const nsl_field* f, const float* params, const float* pose, const float* intr, int H, int W,
                       const nsl_render_config* c, float* rgb, float* depth, float* var, float* opacity,
                       hipStream_t st) {
  int rc = check_render_args(f, params, pose, intr, H, W, c, rgb, depth, var);
  if (rc) return rc;
  const size_t need = nsl_render_workspace_bytes(f, H, W, c);
  if (need > noalloc_scratch_bytes())
    return fail(NSL_E_WORKSPACE, "render needs %zu bytes of scratch, the static scratch holds %zu", need,
                noalloc_scratch_bytes());
  void* ws = nullptr;
  HIP_TRY(noalloc_scratch(&ws), "static scratch address");
  return render_image(f, params, pose, intr, H, W, c, rgb, depth, var, opacity, ws, st);
}

// ---------------------------------------------------------------------------
// Covariances
// ---------------------------------------------------------------------------

size_t nsl_covariance_workspace_bytes(int c, int p) {
  if (c < 1 || p < 0) return 0;
  return align256(cov_partial_blocks(p) * (size_t)c * c * sizeof(double));
}

int nsl_depth_covariance(int c, int p, const double* C, const double* Et, const double* P, const double* inv_depth,
                         double* sigma_T, double* sigma_d, float* depth_var, int* status, void* ws,
                         size_t ws_bytes, hipStream_t st) {
  if (!C || !Et || !P || !sigma_T || !status || !ws) return fail(NSL_E_INVALID, "null argument");
  if (c < 1 || c > 60) return fail(NSL_E_INVALID, "c must be in [1, 60]");
  if (p < 0) return fail(NSL_E_INVALID, "negative pixel count");
  if (depth_var && !inv_depth) return fail(NSL_E_INVALID, "depth_var needs inv_depth");
  if (ws_bytes < nsl_covariance_workspace_bytes(c, p)) return fail(NSL_E_WORKSPACE, "covariance workspace too small");
  HIP_TRY(depth_covariance(c, p, C, Et, P, inv_depth, sigma_T, sigma_d, depth_var, status, static_cast<double*>(ws), st),
          "covariance");
  return NSL_OK;
}

}  // extern "C"
