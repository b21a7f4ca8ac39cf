"""Mixed precision (FP16 tables, BF16 MLP on MFMA, FP32 accumulation, FP32
master weights, dynamic loss scaling) against the FP64 oracle at the 2e-2
tolerance, element by element relative to the oracle's magnitudes."""
import numpy as np
import pytest

import workloads as W
from oracle import field as ofield
from oracle import step as ostep
from parity import check_mag, params_for, report, split_grads, upload_keyframes

pytestmark = pytest.mark.gpu
TOL = 2e-2


def _t(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("spec,table_range", [(W.C1_FIELD, 1e-4), (W.C1_FIELD, 0.5), (W.C2_FIELD, 1e-4),
                                              (W.C2_FIELD, 0.5)], ids=["tiny", "tiny-big", "full", "full-big"])
def test_mixed_field_forward_and_adjoint(nsl, gpu, spec, table_range):
    import torch
    dev = gpu
    S = 1037
    report(f"mixed field: levels={spec.levels} S={S} table_range={table_range}")
    f = nsl.Field(spec)
    lay = f.layout
    flat, t64, w64 = params_for(spec, lay, seed=2, table_range=table_range)
    rng = np.random.default_rng(4)
    xn = rng.uniform(size=(S, 3)).astype(np.float32)
    d = rng.normal(size=(S, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    P = _t(torch, dev, flat)
    shadow = f.prepare_mixed(P)
    sig, rgb = f.fwd_mixed(shadow, _t(torch, dev, xn), _t(torch, dev, d))
    e, em, corners = ofield.encode_fwd(spec, t64, xn)
    cache = ofield.mlp_fwd(spec, w64, e, em, ofield.sh_basis(d.astype(np.float64), spec.sh_bands), band=TOL)
    r1 = check_mag("sigma", sig.cpu().numpy(), cache["sigma"], cache["sigma_mag"], TOL)
    r2 = check_mag("colour", rgb.cpu().numpy(), cache["colour"], cache["colour_mag"], TOL)
    dsig = rng.normal(size=S).astype(np.float32)
    drgb = rng.normal(size=(S, 3)).astype(np.float32)
    grads = torch.zeros(lay["total"], dtype=torch.float32, device=dev)
    ws = torch.empty(f.workspace_bytes(S), dtype=torch.uint8, device=dev)
    f.bwd_mixed(shadow, _t(torch, dev, xn), _t(torch, dev, d), _t(torch, dev, dsig), _t(torch, dev, drgb), grads, ws)
    dWs, dWm, de, dem = ofield.mlp_bwd(spec, w64, cache, dsig.astype(np.float64), np.abs(dsig).astype(np.float64),
                                       drgb.astype(np.float64), np.abs(drgb).astype(np.float64), band_tol=TOL)
    gt, gtm = ofield.encode_bwd(spec, corners, de, dem, lay["table_floats"])
    gtab, gws = split_grads(grads.cpu().numpy(), lay, spec)
    rels = [check_mag("grad table", gtab, gt, gtm, TOL)]
    for j, (a, b, m) in enumerate(zip(gws, dWs, dWm)):
        rels.append(check_mag(f"grad W{j}", a, b, m, TOL))
    report(f"  rel L2 error: sigma {r1:.2e} colour {r2:.2e} grads " + " ".join(f"{x:.2e}" for x in rels))


def _mixed_step(nsl, torch, dev, spec, sampler, kf, ids, flat, state, adam=False):
    f = nsl.Field(spec)
    m = upload_keyframes(nsl, torch, kf, dev)
    st = _t(torch, dev, np.asarray(state, np.float32))
    cfg = nsl.step_config(sampler, precision=nsl.PRECISION_MIXED, scale_state=st, do_adam=adam,
                          lr=W.ADAM_LR, betas=W.ADAM_BETAS, eps=W.ADAM_EPS, adam_step=1)
    ws = torch.empty(nsl.step_workspace_bytes(f, cfg, len(ids)), dtype=torch.uint8, device=dev)
    P = _t(torch, dev, flat)
    G = torch.zeros_like(P)
    M, V = torch.zeros_like(P), torch.zeros_like(P)
    loss = torch.zeros(3, device=dev)
    rays = torch.zeros(len(ids), 6, device=dev)
    nsl.train_step(m, f, P, G, M, V, cfg, _t(torch, dev, ids.view(np.int32)), ws, loss, None, rays)
    torch.cuda.synchronize()
    return dict(loss=loss.cpu().numpy(), grads=G.cpu().numpy(), params=P.cpu().numpy(), state=st.cpu().numpy(),
                rays=rays.cpu().numpy(), layout=f.layout)


def test_mixed_step_matches_oracle(nsl, gpu):
    import torch
    dev = gpu
    report("mixed step: tiny workload, loss scale 2^15")
    spec, sampler = W.C1_FIELD, W.C1_SAMPLER
    kf = W.c1_keyframes()
    ids = W.c1_pixels()
    f = nsl.Field(spec)
    flat, t64, w64 = params_for(spec, f.layout, seed=0, table_range=0.3)
    scale = 2.0 ** 15
    g = _mixed_step(nsl, torch, dev, spec, sampler, kf, ids, flat, [scale, 0, 0, 0])
    o = ostep.train_step(spec, sampler, kf, t64, w64, ids, band=TOL)
    assert g["state"].tolist() == [scale, 1.0, 0.0, 0.0]
    assert g["loss"][0] == pytest.approx(o["loss"], rel=TOL)
    sel = o["sel"]
    check_mag("rgb", g["rays"][sel, :3], o["rgb"], np.abs(o["rgb"]) + 1e-7, TOL)
    check_mag("depth", g["rays"][sel, 3], o["depth_z"], np.abs(o["depth_z"]) + 1e-7, TOL)
    gtab, gws = split_grads(g["grads"] / scale, f.layout, spec)
    rels = [check_mag("grad table", gtab, o["grad_table"], o["grad_table_mag"], TOL)]
    for j in range(len(gws)):
        rels.append(check_mag(f"grad W{j}", gws[j], o["grad_w"][j], o["grad_w_mag"][j], TOL))
    report("  rel L2 error of gradients: " + " ".join(f"{x:.2e}" for x in rels))


def test_dynamic_loss_scale_skips_overflow(nsl, gpu):
    """A loss scale so large that the gradients overflow: the update is
    skipped, the gradient cleared, the scale halved and the skip counted."""
    import torch
    dev = gpu
    spec, sampler = W.C1_FIELD, W.C1_SAMPLER
    kf = W.c1_keyframes()
    ids = W.random_rays_subset(128, 1024, seed=2)
    f = nsl.Field(spec)
    flat, _, _ = params_for(spec, f.layout, seed=0, table_range=0.3)
    big = 3.0e38
    g = _mixed_step(nsl, torch, dev, spec, sampler, kf, ids, flat, [big, 5, 0, 0], adam=True)
    assert np.array_equal(g["params"], flat)              # no update
    assert np.all(g["grads"] == 0)                          # gradient cleared
    st = g["state"]
    assert st[0] == np.float32(big) * np.float32(0.5) and st[1] == 0 and st[2] == 1 and st[3] == 1
    ok = _mixed_step(nsl, torch, dev, spec, sampler, kf, ids, flat, [2.0 ** 15, 1999, 0, 0], adam=True)
    assert ok["state"].tolist() == [2.0 ** 16, 0.0, 0.0, 0.0]   # 2000 clean steps: scale doubles
    assert not np.array_equal(ok["params"], flat)
