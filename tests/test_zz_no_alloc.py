"""nsl_render_noalloc (the library's static scratch instead of a caller
workspace) against nsl_render (the same kernels with a workspace), through
the C ABI: bit-identical images on two calls in a row, the second on a
smaller image and the other field shape."""
import numpy as np
import pytest

import workloads as W
from parity import params_for, report

pytestmark = pytest.mark.gpu


def _t(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _render_both(nsl, torch, dev, spec, H, Wd, seed):
    f = nsl.Field(spec)
    flat, _, _ = params_for(spec, f.layout, seed=seed, table_range=1.0)
    P = _t(torch, dev, flat)
    pose = _t(torch, dev, W.look_at_pose((1.5, 0.3, 0.2)).astype(np.float32).reshape(12))
    intr = _t(torch, dev, np.array([0.9375 * Wd, 0.9375 * Wd, Wd / 2.0, H / 2.0], np.float32))
    rcfg = nsl.render_config(0.5, 2.0 / 32, 32, 1e-4)
    n = H * Wd
    ws = torch.empty(nsl.render_workspace_bytes(f, H, Wd, rcfg), dtype=torch.uint8, device=dev)
    ref = [torch.full((n, 3), -1.0, device=dev)] + [torch.full((n,), -1.0, device=dev) for _ in range(3)]
    nsl.render(f, P, pose, intr, H, Wd, rcfg, ws, *ref)
    got = [torch.full((n, 3), -2.0, device=dev)] + [torch.full((n,), -2.0, device=dev) for _ in range(3)]
    nsl.render_noalloc(f, P, pose, intr, H, Wd, rcfg, *got)
    torch.cuda.synchronize()
    return ref, got


def test_render_noalloc_equals_render(nsl, gpu):
    import torch
    dev = gpu
    for spec, (H, Wd), seed in ((W.C2_FIELD, (120, 160), 1), (W.C1_FIELD, (30, 40), 2),
                                (W.C2_FIELD, (48, 64), 3)):
        ref, got = _render_both(nsl, torch, dev, spec, H, Wd, seed)
        for a, b in zip(ref, got):
            assert torch.equal(a, b), (spec.levels, H, Wd)
        assert float(ref[3].max()) > 0.0                  # something was rendered
        report(f"render_noalloc: {spec.levels} levels, {Wd}x{H}: equal to nsl_render")
