"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/nsl.h declares, computes the same parameter layout as
the oracle, and reports invalid calls with status codes before touching the
device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import field as ofield

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
HEADER = os.path.join(INCLUDE, "nsl.h")


def declared_functions():
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if h.endswith(".h"):
            text = re.sub(r"/\*.*?\*/", "", open(os.path.join(INCLUDE, h)).read(), flags=re.S)
            names |= set(re.findall(r"\b(nsl_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported(nsl):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(nsl._lib, n), n


@pytest.mark.parametrize("spec", [W.C1_FIELD, W.C2_FIELD], ids=["tiny", "full"])
def test_layout_matches_oracle(nsl, spec):
    got = nsl.field_layout(spec)
    res, dense, sizes, offs = ofield.level_layout(spec)
    lay = ofield.param_layout(spec)
    assert got["res"] == res
    assert got["dense"] == dense
    assert got["level_entries"] == sizes
    assert got["level_offset"] == offs.tolist()
    assert got["table_floats"] == lay["table_floats"]
    assert got["w_offsets"] == lay["w_offsets"]
    assert got["w_shapes"] == spec.mlp_dims()
    assert got["total"] == lay["total"]


def test_unsupported_shape_is_rejected(nsl):
    import dataclasses
    bad = dataclasses.replace(W.C1_FIELD, density_hidden=48)
    with pytest.raises(nsl.NslError) as e:
        nsl.Field(bad)
    assert e.value.code == nsl.E_INVALID and "unsupported" in str(e.value)
    with pytest.raises(nsl.NslError):
        nsl.Field(dataclasses.replace(W.C1_FIELD, aabb_max=(-3.0, 2.0, 2.0)))


def test_host_side_errors(nsl):
    lib = nsl._lib
    f = nsl.Field(W.C1_FIELD)
    fake = C.c_void_p(1 << 20)          # never dereferenced: validation fails first
    need = lib.nsl_field_workspace_bytes(f.handle, 16)
    assert need > 0 and lib.nsl_field_workspace_bytes(f.handle, 1 << 20) > need
    assert lib.nsl_field_workspace_bytes(f.handle, 1 << 27) == 0      # records beyond 32-bit positions
    rc = lib.nsl_field_fwd(f.handle, fake, fake, fake, 16, fake, fake, fake, need - 1, None)
    assert rc == nsl.E_WORKSPACE and b"workspace" in lib.nsl_last_error()
    rc = lib.nsl_field_fwd(f.handle, None, fake, fake, 16, fake, fake, fake, need, None)
    assert rc == nsl.E_INVALID
    h = C.c_void_p()
    assert lib.nsl_mapper_create(2, 8, 8, 4, None, 0, C.byref(h)) == nsl.E_INVALID
    nb = lib.nsl_mapper_storage_bytes(2, 8, 8, 4)
    assert lib.nsl_mapper_create(2, 8, 8, 4, fake, nb - 1, C.byref(h)) == nsl.E_WORKSPACE
    assert lib.nsl_mapper_create(2, 8, 8, 4, C.c_void_p((1 << 20) + 4), nb, C.byref(h)) == nsl.E_INVALID
    assert lib.nsl_mapper_create(2, 8, 8, 4, fake, nb, C.byref(h)) == nsl.OK
    m = h
    assert lib.nsl_mapper_count(m) == 0 and lib.nsl_keyframe_slot(m, 7) == -1
    cfg = nsl.step_config(W.C1_SAMPLER)
    # no keyframes yet
    rc = lib.nsl_train_step(m, f.handle, fake, fake, None, None, C.byref(cfg), fake, 4, fake, 1 << 30, fake,
                            None, None, None)
    assert rc == nsl.E_INVALID and b"keyframes" in lib.nsl_last_error()
    bad = nsl.step_config(W.C1_SAMPLER)
    bad.dt = 0.0
    rc = lib.nsl_train_step(m, f.handle, fake, fake, None, None, C.byref(bad), fake, 4, fake, 1 << 30, fake,
                            None, None, None)
    assert rc == nsl.E_INVALID and b"dt" in lib.nsl_last_error()
    # duplicate ids in one upsert, and over-capacity
    ids = (C.c_int32 * 2)(3, 3)
    assert lib.nsl_keyframes_upsert(m, 2, ids, fake, fake, fake, fake, fake, 0, None) == nsl.E_INVALID
    ids3 = (C.c_int32 * 3)(1, 2, 3)
    assert lib.nsl_keyframes_upsert(m, 3, ids3, fake, fake, fake, fake, fake, 0, None) == nsl.E_CAPACITY
    assert lib.nsl_mapper_count(m) == 0
    lib.nsl_mapper_destroy(m)
    assert lib.nsl_composite_fwd(None, fake, fake, fake, 1, 0.1, 0.0, fake, None) == nsl.E_INVALID
    assert lib.nsl_adam(fake, fake, fake, fake, 10, 1e-2, 0.9, 0.99, 1e-15, 0, 1.0, None) == nsl.E_INVALID
    # parameter vectors and shadows are read with 16-byte loads
    odd = C.c_void_p((1 << 20) + 8)
    assert lib.nsl_adam(odd, fake, fake, fake, 10, 1e-2, 0.9, 0.99, 1e-15, 1, 1.0, None) == nsl.E_INVALID
    assert b"16-byte" in lib.nsl_last_error()
    rc = lib.nsl_field_fwd(f.handle, odd, fake, fake, 16, fake, fake, fake, need, None)
    assert rc == nsl.E_INVALID and b"16-byte" in lib.nsl_last_error()
    assert lib.nsl_field_prepare_mixed(f.handle, fake, odd, None) == nsl.E_INVALID
    # the loss and the encoding on their own
    nl = lib.nsl_loss_workspace_bytes(5)
    assert nl >= 40 and lib.nsl_loss_workspace_bytes(-1) == 0
    rc = lib.nsl_loss_fwd(fake, 5, fake, fake, fake, fake, 1.0, fake, None, fake, nl - 1, None)
    assert rc == nsl.E_WORKSPACE
    assert lib.nsl_loss_fwd(fake, 0, fake, fake, fake, fake, 1.0, fake, None, fake, nl, None) == nsl.E_INVALID
    assert lib.nsl_loss_bwd(fake, 5, fake, None, fake, fake, 1.0, None, fake, None) == nsl.E_INVALID
    assert lib.nsl_encode_fwd(f.handle, fake, fake, -1, fake, None) == nsl.E_INVALID
    assert lib.nsl_encode_fwd_mixed(f.handle, odd, fake, 4, fake, None) == nsl.E_INVALID
    ne = lib.nsl_encode_bwd_workspace_bytes(f.handle, 64)
    assert ne > lib.nsl_encode_bwd_workspace_bytes(f.handle, 16) > 0
    assert lib.nsl_encode_bwd(f.handle, fake, 64, fake, 0, 0, fake, fake, ne - 1, None) == nsl.E_WORKSPACE
    assert lib.nsl_encode_bwd(f.handle, fake, 64, fake, 7, 0, fake, fake, ne, None) == nsl.E_INVALID
    assert lib.nsl_encode_bwd(f.handle, fake, 64, fake, 0, 0, odd, fake, ne, None) == nsl.E_INVALID
    # machine-peak probes validate their shapes
    assert lib.nsl_peak_copy(fake, fake, 24, None) == nsl.E_INVALID
    assert lib.nsl_peak_gather(fake, 20, fake, 100, 16, None) == nsl.E_INVALID
    assert lib.nsl_peak_gather(fake, 20, fake, 256, 15, None) == nsl.E_INVALID
    assert lib.nsl_peak_mfma(1, None, 4, 10, None) == nsl.E_INVALID


def test_workspace_queries_scale(nsl):
    f = nsl.Field(W.C2_FIELD)
    cfg = nsl.step_config(W.C2_SAMPLER)
    a = nsl.step_workspace_bytes(f, cfg, 1000)
    b = nsl.step_workspace_bytes(f, cfg, 2000)
    assert b > a > 0
    # per-sample buffers dominate: t, ray, sigma, rgb, dsigma, drgb = 40 B/sample
    assert a > 40 * W.C2_SAMPLER.max_samples


def test_records_match_c_layout(nsl, tmp_path):
    """The binding's ctypes mirrors of the render records and the step
    configuration have the C sizes and offsets (checked with the host C
    compiler)."""
    import ctypes as C
    import subprocess
    src = tmp_path / "lay.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "nsl.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(nsl_render_request), '
                   'offsetof(nsl_render_request, rgb), offsetof(nsl_render_request, H), sizeof(nsl_render_tile), '
                   'sizeof(nsl_step_config), offsetof(nsl_step_config, precision), '
                   'offsetof(nsl_step_config, scale_state), offsetof(nsl_step_config, keep_encoding));return 0;}\n')
    exe = tmp_path / "lay"
    inc = os.path.join(os.path.dirname(HEADER))
    r = subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", inc, "-I", "/opt/rocm/include", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("host C compiler cannot build against the HIP headers: " + r.stderr[-200:])
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert got == [C.sizeof(nsl.RenderRequest), nsl.RenderRequest.rgb.offset, nsl.RenderRequest.H.offset,
                   C.sizeof(nsl.RenderTile), C.sizeof(nsl.StepConfig), nsl.StepConfig.precision.offset,
                   nsl.StepConfig.scale_state.offset, nsl.StepConfig.keep_encoding.offset]
