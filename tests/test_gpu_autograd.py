"""Differentiation workload: the recompute adjoint behind torch.autograd and
through nsl_train_step, against the FP64 oracle's gradient on 4096 rays and
against FP64 central finite differences of the oracle loss on 64 rays."""
import numpy as np
import pytest

import workloads as W
from oracle import field as ofield
from oracle import rays as orays
from oracle import step as ostep
from parity import check_mag, params_for, report, split_grads, upload_keyframes

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _t(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _cam64():
    pose = np.zeros((1, 3, 4))
    pose[0, :, :3] = np.eye(3)
    pose[0, :, 3] = (0.0, 0.0, -2.0)
    return W.sphere_keyframes(0, pose, 64, 64, 64.0, W.C1_SAMPLER.t_far)


def test_autograd_matches_oracle_on_4096_rays(nsl, gpu):
    import torch
    from paper_2210_13641_amd import autograd as ag
    dev = gpu
    report("autograd: 4096 rays (64x64 camera), recompute adjoint vs oracle gradient")
    spec, sampler = W.C1_FIELD, W.C1_SAMPLER
    kf = _cam64()
    ids = np.arange(64 * 64, dtype=np.uint32)
    f = nsl.Field(spec)
    flat, t64, w64 = params_for(spec, f.layout, seed=4, table_range=0.2)
    o = ostep.train_step(spec, sampler, kf, t64, w64, ids)
    # inputs of the differentiable path: FP32 sample positions and directions
    o32, d32, s32 = orays.rays_fp32(kf.pose, kf.intr, ids, 64, 64)
    ts = [orays.uniform_t(sampler)] * len(ids)
    t_all, ray_of, xn = ostep.sample_positions(spec, o32, d32, ts, o["sel"])
    P = _t(torch, dev, flat).requires_grad_(True)
    ws = torch.empty(f.workspace_bytes(len(xn)), dtype=torch.uint8, device=dev)
    off = _t(torch, dev, o["offsets"].astype(np.int32))
    out = ag.render_samples(f, P, _t(torch, dev, xn), _t(torch, dev, d32[o["sel"]][ray_of]),
                            _t(torch, dev, t_all), off, sampler.dt, ws)
    k, v, u = orays.split_pixel_ids(ids, 64, 64)
    s64 = orays.rays_fp64(kf.pose, kf.intr, ids, 64, 64)[2]
    L, Lr, Ld = ag.mapping_loss(out, _t(torch, dev, s64.astype(np.float32)), _t(torch, dev, kf.rgb[k, v, u]),
                                _t(torch, dev, kf.depth[k, v, u]), _t(torch, dev, kf.depth_var[k, v, u]))
    L.backward()
    assert float(L.detach()) == pytest.approx(o["loss"], rel=2e-5)
    outc = out.detach().cpu().numpy()
    check_mag("rgb", outc[:, :3], o["rgb"], o["rgb_mag"], TOL)
    check_mag("depth", outc[:, 3], o["depth_ray"], o["depth_z_mag"] * o["scale"], TOL)
    g = P.grad.cpu().numpy()
    gtab, gws = split_grads(g, f.layout, spec)
    check_mag("grad table", gtab, o["grad_table"], o["grad_table_mag"], 2 * TOL)
    for j in range(len(gws)):
        check_mag(f"grad W{j}", gws[j], o["grad_w"][j], o["grad_w_mag"][j], 2 * TOL)


def test_step_gradient_vs_finite_differences(nsl, gpu):
    """GPU gradient of nsl_train_step on 64 random rays against FP64 central
    differences of the oracle loss: h = 1e-3 for the network weights; table
    entries (values ~1e-1) use h = 1e-5 so the perturbation stays inside one
    linear piece of every ReLU."""
    import torch
    dev = gpu
    spec, sampler = W.C1_FIELD, W.C1_SAMPLER
    kf = W.c1_keyframes()
    ids = W.random_rays_subset(64, 1024, seed=21)
    f = nsl.Field(spec)
    flat, t64, w64 = params_for(spec, f.layout, seed=6, table_range=0.1)
    m = upload_keyframes(nsl, torch, kf, dev)
    cfg = nsl.step_config(sampler)
    wsb = torch.empty(nsl.step_workspace_bytes(f, cfg, len(ids)), dtype=torch.uint8, device=dev)
    P = _t(torch, dev, flat)
    G = torch.zeros_like(P)
    loss = torch.zeros(3, device=dev)
    nsl.train_step(m, f, P, G, None, None, cfg, _t(torch, dev, ids.view(np.int32)), wsb, loss)
    gtab, gws = split_grads(G.cpu().numpy(), f.layout, spec)

    def L(tab, wl):
        return ostep.train_step(spec, sampler, kf, tab, wl, ids, band=0.0)["loss"]

    rng = np.random.default_rng(0)
    checked = 0
    for j, Wj in enumerate(w64):
        for _ in range(8):
            a, b = rng.integers(0, Wj.shape[0]), rng.integers(0, Wj.shape[1])
            h = 1e-3
            wp = [w.copy() for w in w64]
            wm = [w.copy() for w in w64]
            wp[j][a, b] += h
            wm[j][a, b] -= h
            fd = (L(t64, wp) - L(t64, wm)) / (2 * h)
            scale = np.abs(gws[j]).max()
            assert gws[j][a, b] == pytest.approx(fd, rel=1e-3, abs=1e-4 * scale), (j, a, b)
            checked += 1
    touched = np.nonzero(gtab)[0]
    for q in rng.choice(touched, size=24, replace=False):
        h = 1e-5
        tp, tm = t64.copy(), t64.copy()
        tp[q] += h
        tm[q] -= h
        fd = (L(tp, w64) - L(tm, w64)) / (2 * h)
        assert gtab[q] == pytest.approx(fd, rel=1e-3, abs=1e-4 * np.abs(gtab).max()), q
        checked += 1
    assert checked == 8 * len(w64) + 24
