"""ctypes binding of libnsl.so (include/nsl.h): argument marshalling only.

Every function here forwards torch device pointers and the current HIP
stream to the library; all computation runs in the library's gfx950
kernels.  If the library is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnsl.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2210_13641_amd.build`")
_lib = C.CDLL(LIB_PATH)

OK = 0
E_INVALID, E_WORKSPACE, E_HIP, E_BUDGET, E_CAPACITY = -1, -2, -3, -4, -5
SAMPLER_UNIFORM, SAMPLER_OCCUPANCY = 0, 1
PRECISION_FP32, PRECISION_MIXED = 0, 1
MAX_LEVELS, MAX_LAYERS = 16, 8


class FieldConfig(C.Structure):
    _fields_ = [("levels", C.c_int32), ("feat_per_level", C.c_int32), ("log2_table", C.c_int32),
                ("base_res", C.c_int32), ("per_level_scale", C.c_float), ("max_res", C.c_int32),
                ("density_hidden", C.c_int32), ("geo_dim", C.c_int32), ("sh_bands", C.c_int32),
                ("n_colour_hidden", C.c_int32), ("colour_hidden", C.c_int32 * 4),
                ("aabb_min", C.c_float * 3), ("aabb_max", C.c_float * 3)]


class ParamLayout(C.Structure):
    _fields_ = [("levels", C.c_int32), ("res", C.c_int32 * MAX_LEVELS), ("dense", C.c_int32 * MAX_LEVELS),
                ("level_entries", C.c_int64 * MAX_LEVELS), ("level_offset", C.c_int64 * MAX_LEVELS),
                ("table_floats", C.c_int64), ("n_layers", C.c_int32), ("w_offset", C.c_int64 * MAX_LAYERS),
                ("w_in", C.c_int32 * MAX_LAYERS), ("w_out", C.c_int32 * MAX_LAYERS),
                ("total_floats", C.c_int64)]


class StepConfig(C.Structure):
    _fields_ = [("sampler", C.c_int32), ("t_near", C.c_float), ("t_far", C.c_float), ("dt", C.c_float),
                ("n_uniform", C.c_int32), ("max_per_ray", C.c_int32), ("max_samples", C.c_int32),
                ("lambda_d", C.c_float), ("zero_grads", C.c_int32), ("do_adam", C.c_int32),
                ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("adam_step", C.c_int32), ("loss_scale", C.c_float), ("precision", C.c_int32),
                ("scale_state", C.c_void_p), ("keep_encoding", C.c_int32)]


class RenderConfig(C.Structure):
    _fields_ = [("t_near", C.c_float), ("dt", C.c_float), ("n_samples", C.c_int32), ("stop_T", C.c_float)]


class RenderRequest(C.Structure):
    """Mirror of nsl_render_request (the kernels read an array of these)."""
    _fields_ = [("params", C.c_void_p), ("prepared", C.c_void_p), ("pose", C.c_float * 12),
                ("intr", C.c_float * 4), ("H", C.c_int32), ("W", C.c_int32), ("rgb", C.c_void_p),
                ("depth_z", C.c_void_p), ("var_z", C.c_void_p), ("opacity", C.c_void_p)]


class RenderTile(C.Structure):
    _fields_ = [("request", C.c_int32), ("first_pixel", C.c_int32), ("n_pixels", C.c_int32)]


RENDER_TILE = 64


_vp, _i, _sz, _f = C.c_void_p, C.c_int, C.c_size_t, C.c_float


def _sig(name, res, args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = args
    return fn


_sig("nsl_last_error", C.c_char_p, [])
_sig("nsl_version", _i, [])
_sig("nsl_field_layout", _i, [C.POINTER(FieldConfig), C.POINTER(ParamLayout)])
_sig("nsl_field_create", _i, [C.POINTER(FieldConfig), C.POINTER(_vp)])
_sig("nsl_field_destroy", None, [_vp])
_sig("nsl_mapper_storage_bytes", _sz, [_i, _i, _i, _i])
_sig("nsl_mapper_create", _i, [_i, _i, _i, _i, _vp, _sz, C.POINTER(_vp)])
_sig("nsl_mapper_destroy", None, [_vp])
_sig("nsl_mapper_count", _i, [_vp])
_sig("nsl_keyframes_upsert", _i, [_vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _i, _vp])
_sig("nsl_keyframe_slot", _i, [_vp, C.c_int32])
_sig("nsl_occupancy_set", _i, [_vp, _vp, _i, _vp])
_sig("nsl_step_workspace_bytes", _sz, [_vp, C.POINTER(StepConfig), _i])
_sig("nsl_train_step", _i, [_vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(StepConfig), _vp, _i, _vp, _sz, _vp,
                            _vp, _vp, _vp])
_sig("nsl_march", _i, [_vp, _vp, C.POINTER(StepConfig), _vp, _i, _vp, _sz, _vp, _vp, _vp, _vp, _vp, _vp])
_sig("nsl_field_workspace_bytes", _sz, [_vp, _i])
_sig("nsl_field_fwd", _i, [_vp, _vp, _vp, _vp, _i, _vp, _vp, _vp, _sz, _vp])
_sig("nsl_field_bwd", _i, [_vp, _vp, _vp, _vp, _i, _vp, _vp, _vp, _vp, _sz, _vp])
_sig("nsl_mlp_fwd", _i, [_vp, _vp, _vp, _vp, _i, _vp, _vp, _vp, _sz, _vp])
_sig("nsl_mlp_bwd", _i, [_vp, _vp, _vp, _vp, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp])
_sig("nsl_composite_fwd", _i, [_vp, _vp, _vp, _vp, _i, _f, _f, _vp, _vp])
_sig("nsl_composite_bwd", _i, [_vp, _vp, _vp, _vp, _i, _f, _vp, _vp, _vp, _vp, _vp, _vp, _vp])
_sig("nsl_adam", _i, [_vp, _vp, _vp, _vp, C.c_int64, _f, _f, _f, _f, _i, _f, _vp])
_sig("nsl_render_workspace_bytes", _sz, [_vp, _i, _i, C.POINTER(RenderConfig)])
_sig("nsl_field_prepared_bytes", _sz, [_vp])
_sig("nsl_field_prepare", _i, [_vp, _vp, _vp, _vp])
_sig("nsl_render_batch", _i, [_vp, _vp, _i, _vp, _i, C.POINTER(RenderConfig), _vp])
_sig("nsl_render", _i, [_vp, _vp, _vp, _vp, _i, _i, C.POINTER(RenderConfig), _vp, _vp, _vp, _vp, _vp, _sz, _vp])
_sig("nsl_render_noalloc", _i, [_vp, _vp, _vp, _vp, _i, _i, C.POINTER(RenderConfig), _vp, _vp, _vp, _vp, _vp])

_sig("nsl_mixed_shadow_bytes", _sz, [_vp])
_sig("nsl_field_prepare_mixed", _i, [_vp, _vp, _vp, _vp])
_sig("nsl_field_fwd_mixed", _i, [_vp, _vp, _vp, _vp, _i, _vp, _vp, _vp])
_sig("nsl_field_bwd_mixed", _i, [_vp, _vp, _vp, _vp, _i, _vp, _vp, _vp, _vp, _sz, _vp])
_sig("nsl_loss_workspace_bytes", _sz, [_i])
_sig("nsl_loss_fwd", _i, [_vp, _i, _vp, _vp, _vp, _vp, _f, _vp, _vp, _vp, _sz, _vp])
_sig("nsl_loss_bwd", _i, [_vp, _i, _vp, _vp, _vp, _vp, _f, _vp, _vp, _vp])
_sig("nsl_encode_fwd", _i, [_vp, _vp, _vp, _i, _vp, _vp])
_sig("nsl_encode_fwd_mixed", _i, [_vp, _vp, _vp, _i, _vp, _vp])
_sig("nsl_encode_bwd_workspace_bytes", _sz, [_vp, _i])
_sig("nsl_encode_bwd", _i, [_vp, _vp, _i, _vp, _i, _i, _vp, _vp, _sz, _vp])
_sig("nsl_peak_copy", _i, [_vp, _vp, _sz, _vp])
_sig("nsl_peak_gather", _i, [_vp, _i, _vp, _i, _i, _vp])
_sig("nsl_peak_mfma", _i, [_i, _vp, _i, _i, _vp])
_sig("nsl_covariance_workspace_bytes", _sz, [_i, _i])
_sig("nsl_depth_covariance", _i, [_i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp])
_sig("nsl_profile_enable", _i, [_i])
_sig("nsl_profile_read", _i, [C.POINTER(C.c_double), C.POINTER(_i)])

EXPORTED = [n for n in dir(_lib) if n.startswith("nsl_")]


class NslError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nsl error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise NslError(rc, _lib.nsl_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype):
    if t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return _ptr(t)


PHASES = ("prep", "march", "encode", "field_fwd", "composite_loss", "field_bwd", "table_grad", "weight_grad",
          "adam")


def profile_enable(on=True):
    _check(_lib.nsl_profile_enable(int(on)))


def profile_read():
    ms = (C.c_double * len(PHASES))()
    n = C.c_int()
    _check(_lib.nsl_profile_read(ms, C.byref(n)))
    return dict(zip(PHASES, list(ms))), n.value


def version():
    return _lib.nsl_version()


# ---------------------------------------------------------------------------
# Field
# ---------------------------------------------------------------------------

def field_config(spec) -> FieldConfig:
    """nsl_field_config from a workloads.FieldSpec-like object."""
    c = FieldConfig()
    c.levels, c.feat_per_level, c.log2_table, c.base_res = spec.levels, spec.feat_per_level, spec.log2_table, spec.base_res
    c.per_level_scale = spec.per_level_scale if spec.per_level_scale is not None else 0.0
    c.max_res = spec.max_res or 0
    c.density_hidden, c.geo_dim, c.sh_bands = spec.density_hidden, spec.geo_dim, spec.sh_bands
    c.n_colour_hidden = len(spec.colour_hidden)
    for i, h in enumerate(spec.colour_hidden):
        c.colour_hidden[i] = h
    for i in range(3):
        c.aabb_min[i], c.aabb_max[i] = spec.aabb_min[i], spec.aabb_max[i]
    return c


def field_layout(spec) -> dict:
    cfg = field_config(spec)
    lay = ParamLayout()
    _check(_lib.nsl_field_layout(C.byref(cfg), C.byref(lay)))
    L, nl = lay.levels, lay.n_layers
    return dict(res=list(lay.res[:L]), dense=[bool(x) for x in lay.dense[:L]],
                level_entries=list(lay.level_entries[:L]), level_offset=list(lay.level_offset[:L]),
                table_floats=lay.table_floats, w_offsets=list(lay.w_offset[:nl]),
                w_shapes=list(zip(lay.w_in[:nl], lay.w_out[:nl])), total=lay.total_floats)


class Field:
    def __init__(self, spec):
        self.spec = spec
        self.cfg = field_config(spec)
        h = C.c_void_p()
        _check(_lib.nsl_field_create(C.byref(self.cfg), C.byref(h)))
        self.handle = h
        self.layout = field_layout(spec)

    def __del__(self):
        if getattr(self, "handle", None):
            _lib.nsl_field_destroy(self.handle)
            self.handle = None

    def workspace_bytes(self, S):
        """Workspace of fwd/bwd (either precision) for up to S samples."""
        return _lib.nsl_field_workspace_bytes(self.handle, S)

    def fwd(self, params, xn, dirs, ws):
        S = xn.shape[0]
        sigma = torch.empty(S, device=xn.device, dtype=torch.float32)
        rgb = torch.empty(S, 3, device=xn.device, dtype=torch.float32)
        _check(_lib.nsl_field_fwd(self.handle, _dev(params, torch.float32), _dev(xn, torch.float32),
                                  _dev(dirs, torch.float32), S, _ptr(sigma), _ptr(rgb), _ptr(ws),
                                  ws.numel(), _stream()))
        return sigma, rgb

    def shadow_bytes(self):
        return _lib.nsl_mixed_shadow_bytes(self.handle)

    def prepare_mixed(self, params, shadow=None):
        shadow = torch.empty(self.shadow_bytes(), dtype=torch.uint8, device=params.device) if shadow is None else shadow
        _check(_lib.nsl_field_prepare_mixed(self.handle, _dev(params, torch.float32), _ptr(shadow), _stream()))
        return shadow

    def fwd_mixed(self, shadow, xn, dirs):
        S = xn.shape[0]
        sigma = torch.empty(S, device=xn.device, dtype=torch.float32)
        rgb = torch.empty(S, 3, device=xn.device, dtype=torch.float32)
        _check(_lib.nsl_field_fwd_mixed(self.handle, _ptr(shadow), _dev(xn, torch.float32), _dev(dirs, torch.float32),
                                        S, _ptr(sigma), _ptr(rgb), _stream()))
        return sigma, rgb

    def bwd_mixed(self, shadow, xn, dirs, dsigma, drgb, grads, ws):
        S = xn.shape[0]
        _check(_lib.nsl_field_bwd_mixed(self.handle, _ptr(shadow), _dev(xn, torch.float32), _dev(dirs, torch.float32),
                                        S, _dev(dsigma, torch.float32), _dev(drgb, torch.float32),
                                        _dev(grads, torch.float32), _ptr(ws), ws.numel(), _stream()))

    def bwd(self, params, xn, dirs, dsigma, drgb, grads, ws):
        S = xn.shape[0]
        _check(_lib.nsl_field_bwd(self.handle, _dev(params, torch.float32), _dev(xn, torch.float32),
                                  _dev(dirs, torch.float32), S, _dev(dsigma, torch.float32),
                                  _dev(drgb, torch.float32), _dev(grads, torch.float32), _ptr(ws),
                                  ws.numel(), _stream()))


# ---------------------------------------------------------------------------
# Mapper
# ---------------------------------------------------------------------------

def mapper_storage_bytes(max_kf, H, W, grid_res):
    return _lib.nsl_mapper_storage_bytes(max_kf, H, W, grid_res)


class Mapper:
    def __init__(self, max_kf, H, W, grid_res=1, device="cuda"):
        self.H, self.W, self.grid_res = H, W, grid_res
        nbytes = mapper_storage_bytes(max_kf, H, W, grid_res)
        self.storage = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        _check(_lib.nsl_mapper_create(max_kf, H, W, grid_res, _ptr(self.storage), nbytes, C.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None):
            _lib.nsl_mapper_destroy(self.handle)
            self.handle = None

    def count(self):
        return _lib.nsl_mapper_count(self.handle)

    def slot(self, kf_id):
        return _lib.nsl_keyframe_slot(self.handle, kf_id)

    def upsert(self, ids, rgb, pose, intr, depth, depth_var):
        """ids: sequence of ints; arrays are device tensors (float32)."""
        ids_c = (C.c_int32 * len(ids))(*ids)
        _check(_lib.nsl_keyframes_upsert(self.handle, len(ids), ids_c, _dev(rgb, torch.float32),
                                         _dev(pose, torch.float32), _dev(intr, torch.float32),
                                         _dev(depth, torch.float32), _dev(depth_var, torch.float32), 0,
                                         _stream()))

    def set_occupancy(self, bits):
        _check(_lib.nsl_occupancy_set(self.handle, _dev(bits, torch.int32), 0, _stream()))


# ---------------------------------------------------------------------------
# Step
# ---------------------------------------------------------------------------

def step_config(sampler_spec, lambda_d=1.0, zero_grads=True, do_adam=False, lr=1e-2, betas=(0.9, 0.99),
                eps=1e-15, adam_step=1, loss_scale=1.0, precision=PRECISION_FP32, scale_state=None,
                keep_encoding=False) -> StepConfig:
    c = StepConfig()
    c.sampler = SAMPLER_UNIFORM if sampler_spec.mode == "uniform" else SAMPLER_OCCUPANCY
    c.t_near, c.t_far, c.dt = sampler_spec.t_near, sampler_spec.t_far, sampler_spec.dt
    c.n_uniform, c.max_per_ray, c.max_samples = sampler_spec.n_uniform, sampler_spec.max_per_ray, sampler_spec.max_samples
    c.lambda_d, c.zero_grads, c.do_adam = lambda_d, int(zero_grads), int(do_adam)
    c.lr, c.beta1, c.beta2, c.eps = lr, betas[0], betas[1], eps
    c.adam_step, c.loss_scale = adam_step, loss_scale
    c.precision = precision
    c.scale_state = scale_state.data_ptr() if scale_state is not None else None
    c.keep_encoding = int(keep_encoding)
    return c


def step_workspace_bytes(field: Field, cfg: StepConfig, n_candidates: int) -> int:
    return _lib.nsl_step_workspace_bytes(field.handle, C.byref(cfg), n_candidates)


def train_step(mapper: Mapper, field: Field, params, grads, adam_m, adam_v, cfg: StepConfig, pixel_ids,
               ws, loss_out, stats_out=None, ray_out=None):
    _check(_lib.nsl_train_step(mapper.handle, field.handle, _dev(params, torch.float32), _dev(grads, torch.float32),
                               _ptr(adam_m), _ptr(adam_v), C.byref(cfg), _dev(pixel_ids, torch.int32),
                               pixel_ids.numel(), _ptr(ws), ws.numel(), _dev(loss_out, torch.float32),
                               _ptr(stats_out), _ptr(ray_out), _stream()))


def march(mapper: Mapper, field: Field, cfg: StepConfig, pixel_ids, ws, counts, offsets, t, ray, stats_out=None):
    _check(_lib.nsl_march(mapper.handle, field.handle, C.byref(cfg), _dev(pixel_ids, torch.int32),
                          pixel_ids.numel(), _ptr(ws), ws.numel(), _dev(counts, torch.int32),
                          _dev(offsets, torch.int32), _dev(t, torch.float32), _dev(ray, torch.int32),
                          _ptr(stats_out), _stream()))


def composite_fwd(sigma, rgb, t, ray_off, delta, stop_T=0.0):
    R = ray_off.numel() - 1
    out = torch.empty(R, 6, device=sigma.device, dtype=torch.float32)
    _check(_lib.nsl_composite_fwd(_dev(sigma, torch.float32), _dev(rgb, torch.float32), _dev(t, torch.float32),
                                  _dev(ray_off, torch.int32), R, delta, stop_T, _ptr(out), _stream()))
    return out


def composite_bwd(sigma, rgb, t, ray_off, delta, g_rgb=None, g_depth=None, g_var=None, g_opacity=None):
    R = ray_off.numel() - 1
    g_sigma = torch.zeros_like(sigma)
    g_rgb_s = torch.zeros_like(rgb)
    _check(_lib.nsl_composite_bwd(_dev(sigma, torch.float32), _dev(rgb, torch.float32), _dev(t, torch.float32),
                                  _dev(ray_off, torch.int32), R, delta, _ptr(g_rgb), _ptr(g_depth), _ptr(g_var),
                                  _ptr(g_opacity), _ptr(g_sigma), _ptr(g_rgb_s), _stream()))
    return g_sigma, g_rgb_s


def adam(params, grads, m, v, lr, beta1, beta2, eps, step, grad_scale=1.0):
    _check(_lib.nsl_adam(_dev(params, torch.float32), _dev(grads, torch.float32), _dev(m, torch.float32),
                         _dev(v, torch.float32), params.numel(), lr, beta1, beta2, eps, step, grad_scale,
                         _stream()))


def loss_fwd(out6, rgb_target, depth_z, depth_var_z, ray_scale, lambda_d=1.0, ws=None, n_masked=None):
    """(L, L_rgb, L_D) as a device [3] tensor."""
    R = out6.shape[0]
    dev = out6.device
    ws = torch.empty(_lib.nsl_loss_workspace_bytes(R), dtype=torch.uint8, device=dev) if ws is None else ws
    loss = torch.empty(3, dtype=torch.float32, device=dev)
    _check(_lib.nsl_loss_fwd(_dev(out6, torch.float32), R, _dev(rgb_target, torch.float32),
                             _dev(depth_z, torch.float32), _dev(depth_var_z, torch.float32),
                             _dev(ray_scale, torch.float32), lambda_d, _ptr(loss), _ptr(n_masked), _ptr(ws),
                             ws.numel(), _stream()))
    return loss


def loss_bwd(out6, rgb_target, depth_z, depth_var_z, ray_scale, lambda_d=1.0, g_loss=None):
    """dJ/d out6 [R,6] for upstream gradients g_loss [3] of (L, L_rgb, L_D)."""
    g = torch.empty_like(out6)
    _check(_lib.nsl_loss_bwd(_dev(out6, torch.float32), out6.shape[0], _dev(rgb_target, torch.float32),
                             _dev(depth_z, torch.float32), _dev(depth_var_z, torch.float32),
                             _dev(ray_scale, torch.float32), lambda_d,
                             _dev(g_loss, torch.float32) if g_loss is not None else None, _ptr(g), _stream()))
    return g


def encode_fwd(field: "Field", params, xn):
    """Level-major encoding [levels, S, 2] (FP32 table)."""
    S = xn.shape[0]
    e = torch.empty(field.spec.levels, S, 2, dtype=torch.float32, device=xn.device)
    _check(_lib.nsl_encode_fwd(field.handle, _dev(params, torch.float32), _dev(xn, torch.float32), S, _ptr(e),
                               _stream()))
    return e


def mlp_fwd(field: "Field", params, enc, dirs, ws):
    """sigma [S] and rgb [S,3] of the MLP on a level-major encoding [levels, S, 2]."""
    S = dirs.shape[0]
    sigma = torch.empty(S, device=dirs.device, dtype=torch.float32)
    rgb = torch.empty(S, 3, device=dirs.device, dtype=torch.float32)
    _check(_lib.nsl_mlp_fwd(field.handle, _dev(params, torch.float32), _dev(enc, torch.float32),
                            _dev(dirs, torch.float32), S, _ptr(sigma), _ptr(rgb), _ptr(ws), ws.numel(), _stream()))
    return sigma, rgb


def mlp_bwd(field: "Field", params, enc, dirs, dsigma, drgb, grads, ws):
    """Weight part of grads += the MLP's adjoint; returns dL/de [levels, S, 2]."""
    S = dirs.shape[0]
    d_enc = torch.empty(field.spec.levels, S, 2, dtype=torch.float32, device=dirs.device)
    _check(_lib.nsl_mlp_bwd(field.handle, _dev(params, torch.float32), _dev(enc, torch.float32),
                            _dev(dirs, torch.float32), S, _dev(dsigma, torch.float32), _dev(drgb, torch.float32),
                            _dev(grads, torch.float32), _ptr(d_enc), _ptr(ws), ws.numel(), _stream()))
    return d_enc


def encode_fwd_mixed(field: "Field", shadow, xn):
    """Level-major encoding [levels, S] of BF16 pairs packed in int32 (FP16 table copy)."""
    S = xn.shape[0]
    e = torch.empty(field.spec.levels, S, dtype=torch.int32, device=xn.device)
    _check(_lib.nsl_encode_fwd_mixed(field.handle, _ptr(shadow), _dev(xn, torch.float32), S, _ptr(e), _stream()))
    return e


def encode_bwd(field: "Field", xn, de, grads, precision=PRECISION_FP32, overwrite=False, ws=None):
    """Table part of grads += (or =) the scatter of dL/de [levels, S, 2]."""
    S = xn.shape[0]
    if ws is None:
        ws = torch.empty(_lib.nsl_encode_bwd_workspace_bytes(field.handle, S), dtype=torch.uint8,
                         device=xn.device)
    _check(_lib.nsl_encode_bwd(field.handle, _dev(xn, torch.float32), S, _dev(de, torch.float32), precision,
                               int(overwrite), _dev(grads, torch.float32), _ptr(ws), ws.numel(), _stream()))


def peak_copy(src, dst):
    _check(_lib.nsl_peak_copy(_ptr(src), _ptr(dst), src.numel() * src.element_size(), _stream()))


def peak_gather(table, log2_entries, out, loads):
    _check(_lib.nsl_peak_gather(_ptr(table), log2_entries, _ptr(out), out.numel(), loads, _stream()))


def peak_mfma(bf16, out, iters):
    _check(_lib.nsl_peak_mfma(int(bf16), _ptr(out), out.numel() // 256, iters, _stream()))


def render_config(t_near, dt, n_samples, stop_T=0.0) -> RenderConfig:
    c = RenderConfig()
    c.t_near, c.dt, c.n_samples, c.stop_T = t_near, dt, n_samples, stop_T
    return c


def render_workspace_bytes(field: Field, H, W, cfg: RenderConfig):
    return _lib.nsl_render_workspace_bytes(field.handle, H, W, C.byref(cfg))


def render(field: Field, params, pose, intr, H, W, cfg: RenderConfig, ws, rgb=None, depth=None, var=None,
           opacity=None):
    dev = params.device
    rgb = torch.empty(H * W, 3, device=dev) if rgb is None else rgb
    depth = torch.empty(H * W, device=dev) if depth is None else depth
    var = torch.empty(H * W, device=dev) if var is None else var
    _check(_lib.nsl_render(field.handle, _dev(params, torch.float32), _dev(pose, torch.float32),
                           _dev(intr, torch.float32), H, W, C.byref(cfg), _ptr(rgb), _ptr(depth), _ptr(var),
                           _ptr(opacity), _ptr(ws), ws.numel(), _stream()))
    return rgb, depth, var, opacity


def render_noalloc(field: Field, params, pose, intr, H, W, cfg: RenderConfig, rgb, depth, var, opacity=None):
    """nsl_render_noalloc: the library's static scratch instead of a
    workspace; every output is the caller's."""
    _check(_lib.nsl_render_noalloc(field.handle, _dev(params, torch.float32), _dev(pose, torch.float32),
                                   _dev(intr, torch.float32), H, W, C.byref(cfg), _ptr(rgb), _ptr(depth), _ptr(var),
                                   _ptr(opacity), _stream()))
    return rgb, depth, var, opacity


def prepared_bytes(field: Field) -> int:
    return _lib.nsl_field_prepared_bytes(field.handle)


def prepare(field: Field, params, out=None):
    """MFMA operands of a parameter snapshot (device uint8 buffer)."""
    out = torch.empty(prepared_bytes(field), dtype=torch.uint8, device=params.device) if out is None else out
    _check(_lib.nsl_field_prepare(field.handle, _dev(params, torch.float32), _ptr(out), _stream()))
    return out


def render_request(params, prepared, pose, intr, H, W, rgb, depth, var, opacity=None) -> RenderRequest:
    """Host record of one request; pose/intr are host sequences."""
    r = RenderRequest()
    r.params, r.prepared = params.data_ptr(), prepared.data_ptr()
    for i, x in enumerate(list(pose)):
        r.pose[i] = float(x)
    for i, x in enumerate(list(intr)):
        r.intr[i] = float(x)
    r.H, r.W = H, W
    r.rgb, r.depth_z, r.var_z = rgb.data_ptr(), depth.data_ptr(), var.data_ptr()
    r.opacity = opacity.data_ptr() if opacity is not None else None
    return r


def records_to_device(records, ctype, device):
    """Pack ctypes records into a device byte tensor."""
    n = len(records)
    buf = (ctype * max(n, 1))(*records)
    return bytes_to_device(bytes(buf), device)


def bytes_to_device(data, device):
    """Copy host bytes to a new device byte tensor through pinned memory,
    asynchronously on the current stream (the pinned block is recycled only
    after the copy has completed)."""
    raw = torch.frombuffer(bytearray(data), dtype=torch.uint8).pin_memory()
    return raw.to(device, non_blocking=True)


def render_batch(field: Field, requests_dev, n_req, tiles_dev, n_tiles, cfg: RenderConfig):
    _check(_lib.nsl_render_batch(field.handle, _ptr(requests_dev), n_req, _ptr(tiles_dev), n_tiles, C.byref(cfg),
                                 _stream()))


def depth_covariance(C, Et, P, inv_depth=None, want_sigma_d=True):
    """Sigma_T [c,c], Sigma_d [p] (FP64) and depth variances [p] (float32)
    from a window's Hessian blocks (device float64 tensors)."""
    c, p = C.shape[0], Et.shape[0]
    dev = C.device
    ws = torch.empty(_lib.nsl_covariance_workspace_bytes(c, p), dtype=torch.uint8, device=dev)
    sT = torch.empty(c, c, dtype=torch.float64, device=dev)
    sd = torch.empty(p, dtype=torch.float64, device=dev) if want_sigma_d else None
    dv = torch.empty(p, dtype=torch.float32, device=dev) if inv_depth is not None else None
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    _check(_lib.nsl_depth_covariance(c, p, _dev(C, torch.float64), _dev(Et, torch.float64), _dev(P, torch.float64),
                                     _ptr(inv_depth), _ptr(sT), _ptr(sd), _ptr(dv), _ptr(st), _ptr(ws), ws.numel(),
                                     _stream()))
    return sT, sd, dv, st
