"""GPU parity: every phase of the HIP path, called through the C ABI, against
the FP64 oracle on the same seeded inputs.  FP32 tolerance 1e-5 relative to
the oracle's magnitude of each element (value for rendered sums, abs-sum of
contributions for gradients); integer and sample-set outputs bit-exact."""
import dataclasses
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import field as ofield
from oracle import rays as orays
from oracle import render as orender
from oracle import step as ostep
from parity import c2_inputs, check_mag, params_for, report, split_grads, upload_keyframes

pytestmark = pytest.mark.gpu
TOL = 1e-5
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


@pytest.fixture(scope="module")
def torch_dev(nsl, gpu):
    import torch
    return torch, gpu


def _t(torch, dev, a, dtype=None):
    x = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        x = x.to(dtype)
    return x.to(dev)


# ----------------------------------------------------------------------------
# Compositing
# ----------------------------------------------------------------------------

def _random_rays(seed, lengths):
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int32)
    S = int(off[-1])
    sig = (rng.exponential(2.0, S) * (rng.uniform(size=S) < 0.8)).astype(np.float32)
    col = rng.uniform(size=(S, 3)).astype(np.float32)
    t = np.concatenate([np.sort(rng.uniform(0.5, 3.0, n)) for n in lengths]).astype(np.float32) if S else np.zeros(0, np.float32)
    return off, sig, col, t


LENGTHS = [0, 1, 2, 3, 17, 63, 64, 65, 127, 128, 129, 200, 256, 0, 5, 31, 32, 33]


def test_composite_forward_and_adjoint(nsl, torch_dev):
    torch, dev = torch_dev
    report("composite: ragged rays 0..256 samples")
    off, sig, col, t = _random_rays(0, LENGTHS)
    delta = 0.03
    out = nsl.composite_fwd(_t(torch, dev, sig), _t(torch, dev, col), _t(torch, dev, t),
                            _t(torch, dev, off), delta).cpu().numpy()
    rng = np.random.default_rng(1)
    R = len(LENGTHS)
    gC = rng.normal(size=(R, 3)).astype(np.float32)
    gD = rng.normal(size=R).astype(np.float32)
    gV = rng.normal(size=R).astype(np.float32)
    gs, gc = nsl.composite_bwd(_t(torch, dev, sig), _t(torch, dev, col), _t(torch, dev, t), _t(torch, dev, off),
                               delta, _t(torch, dev, gC), _t(torch, dev, gD), _t(torch, dev, gV))
    gs, gc = gs.cpu().numpy(), gc.cpu().numpy()
    for r in range(R):
        a, b = off[r], off[r + 1]
        dl = np.full(b - a, delta)
        fw = orender.composite_ray(sig[a:b], col[a:b], t[a:b], dl)
        # exact FP32 inputs: the magnitudes carry the kernel's rounding only
        fm = orender.composite_magnitudes(fw, t[a:b], dl, np.zeros(b - a), col[a:b], np.zeros((b - a, 3)), TOL)
        want = np.concatenate([fw["C"], [fw["D"], fw["V"], fw["A"]]])
        mag = np.concatenate([fm["C"], [fm["D"], fm["V"], fm["A"]]]) + 1e-30
        check_mag(f"ray {r} (n={b - a}) outputs", out[r], want, mag, TOL, floor=0.0)
        if b == a:
            continue
        ds, dc, dsm, dcm = orender.composite_ray_bwd(fw, col[a:b], t[a:b], dl, gC[r], float(gD[r]),
                                                     float(gV[r]), mag=fm)
        check_mag(f"ray {r} dsigma", gs[a:b], ds, dsm, TOL)
        check_mag(f"ray {r} dcolour", gc[a:b], dc, dcm, TOL)


def test_composite_slab_closed_form(nsl, torch_dev):
    """Tiny workload's centre pixel through the density-50 sphere: d*, V*, A
    against the decimal closed form."""
    torch, dev = torch_dev
    kf = W.c1_keyframes()
    o32, d32, _ = orays.rays_fp32(kf.pose, kf.intr, np.array([16 * 32 + 16]), 32, 32)
    t = orays.uniform_t(W.C1_SAMPLER)
    x = orays.positions_f32(o32[[0] * 32], d32[[0] * 32], t).astype(np.float64)
    sig = np.where(np.linalg.norm(x, axis=-1) < 0.5, 50.0, 0.0).astype(np.float32)
    out = nsl.composite_fwd(_t(torch, dev, sig), _t(torch, dev, np.zeros((32, 3), np.float32)),
                            _t(torch, dev, t), _t(torch, dev, np.array([0, 32], np.int32)), 0.0625).cpu().numpy()
    g = GOLD["slab"]
    assert out[0, 3] == pytest.approx(float(g["depth"]), rel=1e-6)
    assert out[0, 4] == pytest.approx(float(g["var"]), rel=1e-4)
    assert out[0, 5] == pytest.approx(1.0, abs=1e-6)


def test_composite_early_termination(nsl, torch_dev):
    torch, dev = torch_dev
    off, sig, col, t = _random_rays(3, [40, 100, 7, 256])
    sig = sig * 4
    stop = 1e-2
    out = nsl.composite_fwd(_t(torch, dev, sig), _t(torch, dev, col), _t(torch, dev, t), _t(torch, dev, off),
                            0.05, stop).cpu().numpy()
    for r in range(4):
        a, b = off[r], off[r + 1]
        dl = np.full(b - a, 0.05)
        fw = orender.composite_ray(sig[a:b], col[a:b], t[a:b], dl, stop_T=stop)
        T = fw["T"]
        if np.any(np.abs(T[:b - a] / stop - 1) < 1e-4):
            continue   # stop undecided in float32 -- not this seed's rays
        fm = orender.composite_magnitudes(fw, t[a:b], dl, np.zeros(b - a), col[a:b], np.zeros((b - a, 3)), 1e-5)
        want = np.concatenate([fw["C"], [fw["D"], fw["V"], fw["A"]]])
        mag = np.concatenate([fm["C"], [fm["D"], fm["V"], fm["A"]]])
        check_mag(f"stop ray {r}", out[r], want, mag, 1e-5, floor=0.0)


# ----------------------------------------------------------------------------
# Field (encode + MLP) forward and adjoint
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("spec,table_range", [(W.C1_FIELD, 1e-4), (W.C1_FIELD, 0.5), (W.C2_FIELD, 1e-4),
                                              (W.C2_FIELD, 0.5)], ids=["tiny", "tiny-big", "full", "full-big"])
def test_field_forward_and_adjoint(nsl, torch_dev, spec, table_range):
    torch, dev = torch_dev
    S = 1037                                   # several 16-sample tiles and a ragged tail
    report(f"field: levels={spec.levels} S={S} table_range={table_range}")
    f = nsl.Field(spec)
    lay = f.layout
    flat, t64, w64 = params_for(spec, lay, seed=2, table_range=table_range)
    rng = np.random.default_rng(4)
    xn = rng.uniform(size=(S, 3)).astype(np.float32)
    xn[:8] = np.array([[0, 0, 0], [1, 1, 1], [1, 0, 0.5], [0.5, 0.5, 0.5], [0.25, 0.75, 1],
                       [1, 1, 0], [0, 1, 1], [0.125, 0.375, 0.625]], np.float32)   # faces, vertices
    d = rng.normal(size=(S, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    ws = torch.empty(f.workspace_bytes(S), dtype=torch.uint8, device=dev)
    P = _t(torch, dev, flat)
    sig, rgb = f.fwd(P, _t(torch, dev, xn), _t(torch, dev, d), ws)
    torch.cuda.synchronize()
    e, em, corners = ofield.encode_fwd(spec, t64, xn)
    cache = ofield.mlp_fwd(spec, w64, e, em, ofield.sh_basis(d.astype(np.float64), spec.sh_bands))
    check_mag("sigma", sig.cpu().numpy(), cache["sigma"], cache["sigma_mag"], TOL)
    check_mag("colour", rgb.cpu().numpy(), cache["colour"], cache["colour_mag"], TOL)
    # adjoint for random seeds
    dsig = rng.normal(size=S).astype(np.float32)
    drgb = rng.normal(size=(S, 3)).astype(np.float32)
    grads = torch.zeros(lay["total"], dtype=torch.float32, device=dev)
    f.bwd(P, _t(torch, dev, xn), _t(torch, dev, d), _t(torch, dev, dsig), _t(torch, dev, drgb), grads, ws)
    g = grads.cpu().numpy()
    dWs, dWm, de, dem = ofield.mlp_bwd(spec, w64, cache, dsig.astype(np.float64), np.abs(dsig).astype(np.float64),
                                       drgb.astype(np.float64), np.abs(drgb).astype(np.float64))
    gt, gtm = ofield.encode_bwd(spec, corners, de, dem, lay["table_floats"])
    gtab, gws = split_grads(g, lay, spec)
    check_mag("grad table", gtab, gt, gtm, TOL)
    for j, (a, b, m) in enumerate(zip(gws, dWs, dWm)):
        check_mag(f"grad W{j}", a, b, m, TOL)
    # untouched padding of the parameter vector stays zero
    pad = np.ones(lay["total"], bool)
    pad[:lay["table_floats"]] = False
    for o, (a, b) in zip(lay["w_offsets"], spec.mlp_dims()):
        pad[o:o + a * b] = False
    assert np.all(g[pad] == 0)


def test_field_gradient_accumulates(nsl, torch_dev):
    """Two backward calls add up (grads are accumulated, not overwritten)."""
    torch, dev = torch_dev
    spec = W.C1_FIELD
    f = nsl.Field(spec)
    flat, _, _ = params_for(spec, f.layout, seed=3, table_range=0.3)
    rng = np.random.default_rng(5)
    S = 300
    xn = _t(torch, dev, rng.uniform(size=(S, 3)).astype(np.float32))
    d = rng.normal(size=(S, 3))
    d = _t(torch, dev, (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32))
    ds = _t(torch, dev, rng.normal(size=S).astype(np.float32))
    dc = _t(torch, dev, rng.normal(size=(S, 3)).astype(np.float32))
    ws = torch.empty(f.workspace_bytes(S), dtype=torch.uint8, device=dev)
    P = _t(torch, dev, flat)
    g1 = torch.zeros(f.layout["total"], device=dev)
    f.bwd(P, xn, d, ds, dc, g1, ws)
    g2 = g1.clone()
    f.bwd(P, xn, d, ds, dc, g2, ws)
    assert torch.allclose(g2, 2 * g1, rtol=1e-5, atol=1e-7)


# ----------------------------------------------------------------------------
# Rays and marcher: bit-exact sample sets
# ----------------------------------------------------------------------------

def _march_gpu(nsl, torch, dev, mapper, f, cfg, ids):
    n = len(ids)
    ws = torch.empty(nsl.step_workspace_bytes(f, cfg, n), dtype=torch.uint8, device=dev)
    counts = torch.zeros(n, dtype=torch.int32, device=dev)
    offs = torch.zeros(n + 1, dtype=torch.int32, device=dev)
    t = torch.zeros(cfg.max_samples, dtype=torch.float32, device=dev)
    ray = torch.zeros(cfg.max_samples, dtype=torch.int32, device=dev)
    stats = torch.zeros(4, dtype=torch.int32, device=dev)
    nsl.march(mapper, f, cfg, _t(torch, dev, ids.view(np.int32)), ws, counts, offs, t, ray, stats)
    torch.cuda.synchronize()
    return counts.cpu().numpy(), offs.cpu().numpy(), t.cpu().numpy(), ray.cpu().numpy(), stats.cpu().numpy()


def test_march_occupancy_bit_exact(nsl, torch_dev):
    torch, dev = torch_dev
    scene, occ, kf = c2_inputs()
    report("march: paper-scale occupancy grid, 4096 candidates")
    f = nsl.Field(W.C2_FIELD)
    m = upload_keyframes(nsl, torch, kf, dev, grid_res=128, occ=occ)
    ids = W.c2_candidates(4096)
    cfg = nsl.step_config(W.C2_SAMPLER)
    counts, offs, t, ray, stats = _march_gpu(nsl, torch, dev, m, f, cfg, ids)
    o32, d32, _ = orays.rays_fp32(kf.pose, kf.intr, ids, 480, 640)
    oc, ots = orays.march(W.C2_FIELD, W.C2_SAMPLER, o32, d32, occ)
    assert np.array_equal(counts, oc)
    assert np.array_equal(offs, np.concatenate([[0], np.cumsum(oc)]))
    kept, rmask = orays.batch_cut(oc, W.C2_SAMPLER.max_samples)
    S = int(np.cumsum(oc)[kept].max()) if kept.any() else 0
    assert stats.tolist()[:3] == [int(rmask.sum()), S, int(kept.sum())]
    assert S > 200000 and not kept.all()        # the cut applies at this size
    sel = np.nonzero(rmask)[0]
    want_t = np.concatenate([ots[r] for r in sel])
    want_r = np.concatenate([np.full(len(ots[r]), r) for r in sel])
    assert np.array_equal(t[:S], want_t)        # bit-exact positions on the lattice
    assert np.array_equal(ray[:S], want_r)
    assert oc.max() == 256 and (oc == 0).any()


@pytest.mark.parametrize("reps", [1, 40], ids=["1026", "40962"])
def test_march_uniform_and_bad_ids(nsl, torch_dev, reps):
    """Uniform samples of the tiny camera's pixels plus two ids past the
    keyframe store (empty rays); 40962 candidates (more samples than the
    batch takes) use the separate single-block scan, 1026 the scan inside
    the sample emission.  Counts, every offset, the statistics (rays,
    samples, kept candidates, rays with unusable depth) and the kept samples
    against the oracle's batch cut."""
    torch, dev = torch_dev
    kf = W.c1_keyframes()
    f = nsl.Field(W.C1_FIELD)
    m = upload_keyframes(nsl, torch, kf, dev)
    ids = np.concatenate([np.tile(W.c1_pixels(), reps), np.array([1024, 5000], np.uint32)])
    n = len(ids)
    cfg = nsl.step_config(W.C1_SAMPLER)
    counts, offs, t, ray, stats = _march_gpu(nsl, torch, dev, m, f, cfg, ids)
    want = np.where(ids < 1024, 32, 0)
    assert np.array_equal(counts, want)
    assert np.array_equal(offs, np.concatenate([[0], np.cumsum(want)]))
    kept, rmask = orays.batch_cut(want, W.C1_SAMPLER.max_samples)
    S = int(np.cumsum(want)[kept].max())
    pix = np.minimum(ids, 1023)
    usable = np.isfinite(kf.depth.reshape(-1)[pix]) & np.isfinite(kf.depth_var.reshape(-1)[pix]) & \
        (kf.depth_var.reshape(-1)[pix] > 0)
    assert stats.tolist() == [int(rmask.sum()), S, int(kept.sum()), int((rmask & ~usable).sum())]
    assert (reps == 1) == bool(kept.all())           # the cut applies to the larger batch
    sel = np.nonzero(rmask)[0]
    assert np.array_equal(t[:S], np.tile(orays.uniform_t(W.C1_SAMPLER), len(sel)))
    assert np.array_equal(ray[:S], np.repeat(sel, 32))


# ----------------------------------------------------------------------------
# Whole step
# ----------------------------------------------------------------------------

def _step_gpu(nsl, torch, dev, spec, sampler, kf, ids, flat, occ=None, grid_res=1, adam=None, lam=1.0,
              keep_encoding=False, mixed=False, zero_grads=True):
    f = nsl.Field(spec)
    m = upload_keyframes(nsl, torch, kf, dev, grid_res=grid_res, occ=occ)
    kw = dict(lambda_d=lam, zero_grads=zero_grads, keep_encoding=keep_encoding)
    if adam:
        kw.update(do_adam=True, lr=adam["lr"], betas=adam["betas"], eps=adam["eps"], adam_step=adam["step"])
    if mixed:
        kw.update(precision=nsl.PRECISION_MIXED,
                  scale_state=torch.tensor([2.0 ** 15, 0.0, 0.0, 0.0], dtype=torch.float32, device=dev))
    cfg = nsl.step_config(sampler, **kw)
    n = len(ids)
    ws = torch.empty(nsl.step_workspace_bytes(f, cfg, n), dtype=torch.uint8, device=dev)
    P = _t(torch, dev, flat)
    G = torch.full((f.layout["total"],), 7.0 if zero_grads else 0.0, device=dev)  # zero_grads must clear this
    M = torch.zeros_like(P) if adam else None
    V = torch.zeros_like(P) if adam else None
    loss = torch.zeros(3, device=dev)
    stats = torch.zeros(4, dtype=torch.int32, device=dev)
    rays = torch.zeros(n, 6, device=dev)
    nsl.train_step(m, f, P, G, M, V, cfg, _t(torch, dev, ids.view(np.int32)), ws, loss, stats, rays)
    torch.cuda.synchronize()
    out = dict(loss=loss.cpu().numpy(), stats=stats.cpu().numpy(), rays=rays.cpu().numpy(),
               grads=G.cpu().numpy(), params=P.cpu().numpy(), layout=f.layout)
    if adam:
        out.update(m=M.cpu().numpy(), v=V.cpu().numpy())
    return out


def _compare_step(spec, g, o, lay, tol=TOL, grad_scale=1.0):
    """Every output, loss term and gradient of a GPU step against the oracle
    step; returns the relative L2 errors of the gradients."""
    R = o["R"]
    assert g["stats"][0] == R and g["stats"][1] == o["S"]
    sel = o["sel"]
    rays = g["rays"][sel]
    check_mag("rgb", rays[:, :3], o["rgb"], o["rgb_mag"], tol)
    check_mag("depth_z", rays[:, 3], o["depth_z"], o["depth_z_mag"], tol)
    check_mag("var_z", rays[:, 4], o["var_z"], o["var_z_mag"], tol)
    check_mag("opacity", rays[:, 5], o["opacity"], o["opacity_mag"], tol)
    others = np.ones(len(g["rays"]), bool)
    others[sel] = False
    assert np.all(g["rays"][others] == 0)
    assert g["loss"][0] == pytest.approx(o["loss"], rel=tol)
    assert g["loss"][1] == pytest.approx(o["loss_rgb"], rel=tol)
    assert g["loss"][2] == pytest.approx(o["loss_d"], rel=tol)
    gtab, gws = split_grads(g["grads"] / grad_scale, lay, spec)
    covered = np.zeros(len(g["grads"]), bool)
    covered[:lay["table_floats"]] = True
    for off, (a, b) in zip(lay["w_offsets"], spec.mlp_dims()):
        covered[off:off + a * b] = True
    assert np.all(g["grads"][~covered] == 0)        # the padding between blocks is cleared as well
    rels = [check_mag("grad table", gtab, o["grad_table"], o["grad_table_mag"], tol)]
    for j in range(len(gws)):
        rels.append(check_mag(f"grad W{j}", gws[j], o["grad_w"][j], o["grad_w_mag"][j], tol))
    return rels


def worst_ratio(g, o, lay, spec, tol, grad_scale=1.0):
    """Largest |gpu - oracle| / (tol * max(magnitude, 1e-6 max magnitude)) of
    the rendered outputs, the table gradient and each weight gradient."""
    def r(a, b, m):
        a, b, m = (np.asarray(x, np.float64).ravel() for x in (a, b, m))
        m = np.abs(m)
        return float(np.max(np.abs(a - b) / (tol * np.maximum(m, 1e-6 * m.max() + 1e-300)))) if m.size else 0.0
    sel = o["sel"]
    rays = g["rays"][sel]
    gtab, gws = split_grads(g["grads"] / grad_scale, lay, spec)
    out = [("rgb", r(rays[:, :3], o["rgb"], o["rgb_mag"])), ("depth", r(rays[:, 3], o["depth_z"], o["depth_z_mag"])),
           ("var", r(rays[:, 4], o["var_z"], o["var_z_mag"])), ("table", r(gtab, o["grad_table"], o["grad_table_mag"]))]
    out += [(f"W{j}", r(gws[j], o["grad_w"][j], o["grad_w_mag"][j])) for j in range(len(gws))]
    return " ".join(f"{k} {v:.1e}" for k, v in out)


def test_step_tiny_workload(nsl, torch_dev):
    torch, dev = torch_dev
    report("step: tiny workload, 1024 rays x 32 samples")
    spec, sampler = W.C1_FIELD, W.C1_SAMPLER
    kf = W.c1_keyframes()
    ids = W.c1_pixels()
    f = nsl.Field(spec)
    flat, t64, w64 = params_for(spec, f.layout, seed=0)
    g = _step_gpu(nsl, torch, dev, spec, sampler, kf, ids, flat)
    o = ostep.train_step(spec, sampler, kf, t64, w64, ids)
    assert o["R"] == 1024 and o["S"] == 32768
    assert g["stats"][3] == 1024 - 208                # rays without a usable depth
    _compare_step(spec, g, o, f.layout)


def test_step_tiny_trained_like_field(nsl, torch_dev):
    """Same step with a larger-valued table, so density and colour vary."""
    torch, dev = torch_dev
    spec, sampler = W.C1_FIELD, W.C1_SAMPLER
    kf = W.c1_keyframes()
    ids = W.random_rays_subset(700, 1024, seed=9)
    f = nsl.Field(spec)
    flat, t64, w64 = params_for(spec, f.layout, seed=1, table_range=1.0)
    g = _step_gpu(nsl, torch, dev, spec, sampler, kf, ids, flat)
    o = ostep.train_step(spec, sampler, kf, t64, w64, ids)
    _compare_step(spec, g, o, f.layout)


@pytest.mark.slow
def test_step_paper_scale(nsl, torch_dev):
    """The full paper-scale step in FP32: 4096 candidates -> 2^18-sample cut,
    with the encoding gathered again by the backward and with it kept from
    the forward (records counted by the encoding, the scans beside the
    forward and the compositing), both against the oracle at 1e-5."""
    torch, dev = torch_dev
    scene, occ, kf = c2_inputs()
    report("step: paper scale, 16 levels x 2^19, 2^18 samples")
    spec, sampler = W.C2_FIELD, W.C2_SAMPLER
    ids = W.c2_candidates(4096)
    f = nsl.Field(spec)
    flat, t64, w64 = params_for(spec, f.layout, seed=0)
    o = ostep.train_step(spec, sampler, kf, t64, w64, ids, occupancy=occ)
    report(f"  R={o['R']} S={o['S']} ambiguous ReLU units={o['n_amb']}")
    for keep in (False, True):
        g = _step_gpu(nsl, torch, dev, spec, sampler, kf, ids, flat, occ=occ, grid_res=128, keep_encoding=keep)
        _compare_step(spec, g, o, f.layout)


@pytest.mark.slow
@pytest.mark.parametrize("table_range", [1e-4, 0.3], ids=["init", "trained-like"])
def test_mixed_step_paper_scale(nsl, torch_dev, table_range):
    """The headline configuration against the FP64 oracle: the paper-scale
    step in mixed precision (FP16 table copy, BF16 MLP on MFMA, BF16
    table-gradient records, FP32 sums) with the encoding kept from the
    forward and the gradients overwritten, loss scale 2^15; every rendered
    output, the loss terms and every table and weight gradient element at
    2e-2 of the oracle's magnitudes, the oracle's ReLU units within 2e-2 of
    their magnitude of zero taking either side."""
    torch, dev = torch_dev
    scene, occ, kf = c2_inputs()
    report(f"mixed step: paper scale, keep_encoding, table range {table_range}")
    spec, sampler = W.C2_FIELD, W.C2_SAMPLER
    ids = W.c2_candidates(4096)
    f = nsl.Field(spec)
    flat, t64, w64 = params_for(spec, f.layout, seed=0, table_range=table_range)
    g = _step_gpu(nsl, torch, dev, spec, sampler, kf, ids, flat, occ=occ, grid_res=128, keep_encoding=True,
                  mixed=True, zero_grads=True)
    o = ostep.train_step(spec, sampler, kf, t64, w64, ids, occupancy=occ, band=2e-2)
    rels = _compare_step(spec, g, o, f.layout, tol=2e-2, grad_scale=2.0 ** 15)
    units = o["S"] * (64 + 64 + 64)
    report(f"  R={o['R']} S={o['S']} ambiguous ReLU units {o['n_amb']} of {units}; rel L2 error of gradients "
           "(table, W0..W4): " + " ".join(f"{x:.2e}" for x in rels))
    # the same step against the oracle that quantises where the kernels do
    # (FP16 table, BF16 operands and records): only FP32 summation and rare
    # BF16 ties remain between the two
    q = ostep.train_step(spec, sampler, kf, t64, w64, ids, occupancy=occ, band=4e-3, quantised=True, tol=2e-2)
    _compare_step(spec, g, q, f.layout, tol=2e-2, grad_scale=2.0 ** 15)
    # relative errors against the quantised oracle whose ReLU decisions all
    # follow the FP64 sign (no midpoints): what remains is FP32 summation and
    # the decisions that FP32 took the other way
    q0 = ostep.train_step(spec, sampler, kf, t64, w64, ids, occupancy=occ, band=0.0, quantised=True, tol=2e-2)
    gtab, gws = split_grads(g["grads"] / 2.0 ** 15, f.layout, spec)
    rel = lambda a, b: float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))
    rq = [rel(gtab, q0["grad_table"])] + [rel(a, b) for a, b in zip(gws, q0["grad_w"])]
    report(f"  against the quantised oracle: ambiguous ReLU units {q['n_amb']} of {units}; largest error / "
           f"(tol * magnitude): {worst_ratio(g, q, f.layout, spec, 2e-2, 2.0 ** 15)}; rel L2 error of gradients "
           "without midpoints: " + " ".join(f"{x:.2e}" for x in rq))


@pytest.mark.parametrize("mixed", [False, True], ids=["fp32", "mixed"])
def test_step_overwrite_matches_accumulate(nsl, torch_dev, mixed):
    """A step that clears its gradients has the table-gradient reduction
    overwrite them (bins of one chunk store every entry, the others are
    cleared during placement); at paper scale, with bins of one chunk, of
    several and of none, it gives what accumulating onto a zero gradient
    gives, every entry included, up to the summation order of the
    multi-chunk bins."""
    torch, dev = torch_dev
    scene, occ, kf = c2_inputs()
    report(f"step: overwrite vs accumulate onto zeros, paper scale, {'mixed' if mixed else 'fp32'}")
    spec, sampler = W.C2_FIELD, W.C2_SAMPLER
    ids = W.c2_candidates(4096)
    f = nsl.Field(spec)
    flat, _, _ = params_for(spec, f.layout, seed=0, table_range=0.3)
    a, b = [_step_gpu(nsl, torch, dev, spec, sampler, kf, ids, flat, occ=occ, grid_res=128, keep_encoding=True,
                      mixed=mixed, zero_grads=z) for z in (True, False)]
    nt = f.layout["table_floats"]
    assert np.array_equal(a["grads"][nt:], b["grads"][nt:])
    ga, gb = a["grads"][:nt].astype(np.float64), b["grads"][:nt].astype(np.float64)
    assert np.array_equal(ga == 0, gb == 0)                       # the same entries untouched
    assert np.count_nonzero(ga) > 0.1 * nt
    assert np.allclose(ga, gb, rtol=1e-5, atol=1e-6 * np.abs(ga).max())


@pytest.mark.parametrize("log2_table", [19, 20, 21], ids=["2^19", "2^20", "2^21"])
@pytest.mark.parametrize("mixed", [False, True], ids=["fp32", "mixed"])
def test_step_keep_encoding_matches_recompute(nsl, torch_dev, mixed, log2_table):
    """With the encoding kept from the forward instead of gathered again, the
    paper-scale step gives the same forward results, loss and weight
    gradients bit for bit, and the same table gradient up to the summation
    order of its reduction.  The kept-encoding kernel counts the
    table-gradient records itself while a level spans at most 128 bins (2^20
    entries); with larger levels the scatter counts them, as it always does
    when the encoding is gathered again."""
    torch, dev = torch_dev
    scene, occ, kf = c2_inputs()
    report(f"step: keep_encoding vs recompute, paper scale, 2^{log2_table} entries a level, "
           f"{'mixed' if mixed else 'fp32'}")
    spec, sampler = dataclasses.replace(W.C2_FIELD, log2_table=log2_table), W.C2_SAMPLER
    ids = W.c2_candidates(4096)
    f = nsl.Field(spec)
    flat, _, _ = params_for(spec, f.layout, seed=0, table_range=0.3)
    a, b = [_step_gpu(nsl, torch, dev, spec, sampler, kf, ids, flat, occ=occ, grid_res=128, keep_encoding=k,
                      mixed=mixed) for k in (False, True)]
    assert np.array_equal(a["stats"], b["stats"])
    assert np.array_equal(a["rays"], b["rays"]) and np.array_equal(a["loss"], b["loss"])
    nt = f.layout["table_floats"]
    assert np.array_equal(a["grads"][nt:], b["grads"][nt:])      # fixed-order weight-gradient sums
    ga, gb = a["grads"][:nt].astype(np.float64), b["grads"][:nt].astype(np.float64)
    assert np.count_nonzero(ga) > 0.1 * nt
    assert np.allclose(ga, gb, rtol=1e-5, atol=1e-6 * np.abs(ga).max())


def test_step_with_adam(nsl, torch_dev):
    torch, dev = torch_dev
    spec, sampler = W.C1_FIELD, W.C1_SAMPLER
    kf = W.c1_keyframes()
    ids = W.c1_pixels()
    f = nsl.Field(spec)
    flat, t64, w64 = params_for(spec, f.layout, seed=0)
    adam = dict(lr=W.ADAM_LR, betas=W.ADAM_BETAS, eps=W.ADAM_EPS, step=1)
    g = _step_gpu(nsl, torch, dev, spec, sampler, kf, ids, flat, adam=adam)
    o = ostep.train_step(spec, sampler, kf, t64, w64, ids)
    gflat = ofield.pack_params(spec, o["grad_table"], o["grad_w"])
    new, m1, v1 = ostep.adam(flat.astype(np.float64), 0, 0, gflat, 1, W.ADAM_LR, *W.ADAM_BETAS, W.ADAM_EPS)
    assert np.all(g["grads"] == 0)                      # Adam clears the gradient
    # first Adam step moves each parameter by lr*sign(g) where |g| >> eps:
    # compare moves where the oracle gradient is clearly non-zero
    mag = ofield.pack_params(spec, o["grad_table_mag"], o["grad_w_mag"])
    sure = np.abs(gflat) > 1e-3 * mag
    move = g["params"].astype(np.float64) - flat
    assert np.allclose(move[sure], (new - flat)[sure], rtol=1e-4, atol=1e-7)
    check_mag("adam m", g["m"][sure], m1[sure], 0.1 * mag[sure], TOL)
