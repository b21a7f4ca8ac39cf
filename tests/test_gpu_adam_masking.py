"""Adam beyond its first step, Adam after a skipped (overflowed) step, and
the masking of unusable depth measurements, against the FP64 oracle through
the C ABI."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import field as ofield
from oracle import step as ostep
from parity import check_mag, params_for, report, split_grads, upload_keyframes

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _t(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def test_adam_chain_matches_oracle(nsl, gpu):
    """nsl_adam alone over steps t = 1..5 from non-zero moments, on random
    gradients: parameters, m and v after every step against the oracle's own
    chain (the same FP32 inputs, FP64 arithmetic), at 1e-5 of the magnitudes
    propagated along the chain.  Sizes leave a ragged tail of the 4-wide
    kernel."""
    import torch
    dev = gpu
    rng = np.random.default_rng(21)
    n = 100_003
    th = rng.normal(size=n).astype(np.float32)
    m = (0.1 * rng.normal(size=n)).astype(np.float32)
    v = rng.uniform(1e-4, 1.0, n).astype(np.float32)
    P, M, V = _t(torch, dev, th), _t(torch, dev, m), _t(torch, dev, v)
    lr, (b1, b2), eps = W.ADAM_LR, W.ADAM_BETAS, W.ADAM_EPS
    th64, m64, v64 = th.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    Mt, Mm, Mv = np.abs(th64), np.abs(m64), v64.copy()
    for t in range(1, 6):
        g = rng.normal(size=n).astype(np.float32)
        g[:100] *= 1e-6                                   # gradients near zero: the sign may not matter
        G = _t(torch, dev, g)
        nsl.adam(P, G, M, V, lr, b1, b2, eps, t)
        torch.cuda.synchronize()
        g64 = g.astype(np.float64)
        Mt, Mm, Mv = ostep.adam_magnitudes(th64, m64, v64, g64, t, lr, b1, b2, eps, Mt, Mm, Mv, np.abs(g64))
        th64, m64, v64 = ostep.adam(th64, m64, v64, g64, t, lr, b1, b2, eps)
        check_mag(f"adam t={t} params", P.cpu().numpy(), th64, Mt, TOL, floor=0.0)
        check_mag(f"adam t={t} m", M.cpu().numpy(), m64, Mm, TOL, floor=0.0)
        check_mag(f"adam t={t} v", V.cpu().numpy(), v64, Mv, TOL, floor=0.0)
        assert torch.count_nonzero(G).item() == 0        # the gradient is cleared
    report("adam chain: 5 steps from non-zero moments match the oracle")


def test_step_adam_from_nonzero_moments(nsl, gpu):
    """The fused step's Adam at step 3 (bias corrections 1 - b^3) from
    seeded non-zero moments: parameters, m and v against the oracle's Adam
    on the oracle's gradient, at 1e-5 of the propagated magnitudes."""
    import torch
    dev = gpu
    spec, sampler = W.C1_FIELD, W.C1_SAMPLER
    kf = W.c1_keyframes()
    ids = W.c1_pixels()
    f = nsl.Field(spec)
    lay = f.layout
    flat, t64, w64 = params_for(spec, lay, seed=0, table_range=0.3)
    rng = np.random.default_rng(5)
    m0 = (1e-3 * rng.normal(size=lay["total"])).astype(np.float32)
    v0 = rng.uniform(1e-7, 1e-5, lay["total"]).astype(np.float32)
    m = upload_keyframes(nsl, torch, kf, dev)
    step = 3
    cfg = nsl.step_config(sampler, do_adam=True, lr=W.ADAM_LR, betas=W.ADAM_BETAS, eps=W.ADAM_EPS,
                          adam_step=step, zero_grads=True)
    ws = torch.empty(nsl.step_workspace_bytes(f, cfg, len(ids)), dtype=torch.uint8, device=dev)
    P, M, V = _t(torch, dev, flat), _t(torch, dev, m0), _t(torch, dev, v0)
    G = torch.zeros_like(P)
    loss = torch.zeros(3, device=dev)
    nsl.train_step(m, f, P, G, M, V, cfg, _t(torch, dev, ids.view(np.int32)), ws, loss)
    torch.cuda.synchronize()
    o = ostep.train_step(spec, sampler, kf, t64, w64, ids)
    g64 = ofield.pack_params(spec, o["grad_table"], o["grad_w"])
    gm = ofield.pack_params(spec, o["grad_table_mag"], o["grad_w_mag"])
    p64, mm, vv = flat.astype(np.float64), m0.astype(np.float64), v0.astype(np.float64)
    b1, b2 = W.ADAM_BETAS
    Mt, Mm, Mv = ostep.adam_magnitudes(p64, mm, vv, g64, step, W.ADAM_LR, b1, b2, W.ADAM_EPS, np.abs(p64),
                                       np.abs(mm), vv, gm)
    new, m1, v1 = ostep.adam(p64, mm, vv, g64, step, W.ADAM_LR, b1, b2, W.ADAM_EPS)
    check_mag("step adam params", P.cpu().numpy(), new, Mt, TOL)
    check_mag("step adam m", M.cpu().numpy(), m1, Mm, TOL)
    check_mag("step adam v", V.cpu().numpy(), v1, Mv, TOL)
    assert torch.count_nonzero(G).item() == 0


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_adam_after_skipped_step(nsl, gpu, precision):
    """Dynamic loss scaling: step 1 overflows and is skipped, step 2 is
    clean.  Step 2's update is the first one made, so its bias correction is
    that of t = 1 (adam_step 2 minus one skip): parameters, m and v equal the
    oracle's Adam at t = 1 from zero moments on the oracle's gradient (at
    1e-5 in FP32; in mixed precision, where the gradient is only known to
    2e-2, at that tolerance), whereas a correction for t = 2 would move each
    parameter by about 0.74 lr instead of lr."""
    import torch
    dev = gpu
    mixed = precision == "mixed"
    tol = 2e-2 if mixed else TOL
    spec, sampler = W.C1_FIELD, W.C1_SAMPLER
    kf = W.c1_keyframes()
    ids = W.random_rays_subset(256, 1024, seed=2)
    f = nsl.Field(spec)
    lay = f.layout
    flat, t64, w64 = params_for(spec, lay, seed=0, table_range=0.3)
    m = upload_keyframes(nsl, torch, kf, dev)
    idt = _t(torch, dev, ids.view(np.int32))
    state = torch.tensor([3.0e38, 0.0, 0.0, 0.0], device=dev)
    P = _t(torch, dev, flat)
    G, M, V = torch.zeros_like(P), torch.zeros_like(P), torch.zeros_like(P)
    loss = torch.zeros(3, device=dev)
    cfg = nsl.step_config(sampler, precision=nsl.PRECISION_MIXED if mixed else nsl.PRECISION_FP32,
                          scale_state=state, do_adam=True, lr=W.ADAM_LR, betas=W.ADAM_BETAS, eps=W.ADAM_EPS,
                          adam_step=1)
    ws = torch.empty(nsl.step_workspace_bytes(f, cfg, len(ids)), dtype=torch.uint8, device=dev)
    nsl.train_step(m, f, P, G, M, V, cfg, idt, ws, loss)
    torch.cuda.synchronize()
    assert state.cpu().numpy()[2] == 1.0 and torch.equal(P, _t(torch, dev, flat))
    state[0] = 2.0 ** 15
    cfg.adam_step = 2
    nsl.train_step(m, f, P, G, M, V, cfg, idt, ws, loss)
    torch.cuda.synchronize()
    assert state.cpu().numpy().tolist() == [2.0 ** 15, 1.0, 1.0, 0.0]
    o = ostep.train_step(spec, sampler, kf, t64, w64, ids, band=tol)
    g64 = ofield.pack_params(spec, o["grad_table"], o["grad_w"])
    gm = ofield.pack_params(spec, o["grad_table_mag"], o["grad_w_mag"])
    p64 = flat.astype(np.float64)
    z = np.zeros_like(p64)
    b1, b2 = W.ADAM_BETAS
    Mt, Mm, Mv = ostep.adam_magnitudes(p64, z, z, g64, 1, W.ADAM_LR, b1, b2, W.ADAM_EPS, np.abs(p64), z, z, gm)
    new, m1, v1 = ostep.adam(p64, z, z, g64, 1, W.ADAM_LR, b1, b2, W.ADAM_EPS)
    check_mag(f"{precision} params after skip", P.cpu().numpy(), new, Mt, tol)
    check_mag(f"{precision} m after skip", M.cpu().numpy(), m1, Mm, tol)
    check_mag(f"{precision} v after skip", V.cpu().numpy(), v1, Mv, tol)
    if not mixed:                      # most parameters with a gradient moved by the full lr
        move = np.abs(P.cpu().numpy().astype(np.float64) - p64)
        nz = g64 != 0
        assert nz.sum() > 1000 and np.mean(np.isclose(move[nz], W.ADAM_LR, rtol=1e-3)) > 0.5


def test_step_masks_unusable_depth(nsl, gpu):
    """Pixels whose depth is NaN or infinite, or whose variance is negative,
    zero, NaN or infinite, carry no depth loss (precision 0) and are counted
    in n_masked; the loss terms and every gradient match the oracle."""
    import torch
    dev = gpu
    spec, sampler = W.C1_FIELD, W.C1_SAMPLER
    kf0 = W.c1_keyframes()
    depth, var = kf0.depth.copy(), kf0.depth_var.copy()
    hit = np.argwhere(np.isfinite(var[0]))              # pixels with a usable measurement
    rng = np.random.default_rng(3)
    pick = hit[rng.choice(len(hit), 60, replace=False)]
    bad = [("depth nan", np.nan, None), ("depth inf", np.inf, None), ("var negative", None, -0.04),
           ("var zero", None, 0.0), ("var nan", None, np.nan), ("var inf", None, np.inf)]
    for k, (v_, u_) in enumerate(pick):
        _, dval, vval = bad[k % len(bad)]
        if dval is not None:
            depth[0, v_, u_] = dval
        if vval is not None:
            var[0, v_, u_] = vval
    kf = dataclasses.replace(kf0, depth=depth, depth_var=var)
    ids = W.c1_pixels()
    f = nsl.Field(spec)
    lay = f.layout
    flat, t64, w64 = params_for(spec, lay, seed=1, table_range=0.3)
    m = upload_keyframes(nsl, torch, kf, dev)
    cfg = nsl.step_config(sampler, zero_grads=True)
    ws = torch.empty(nsl.step_workspace_bytes(f, cfg, len(ids)), dtype=torch.uint8, device=dev)
    P = _t(torch, dev, flat)
    G = torch.zeros_like(P)
    loss = torch.zeros(3, device=dev)
    stats = torch.zeros(4, dtype=torch.int32, device=dev)
    nsl.train_step(m, f, P, G, None, None, cfg, _t(torch, dev, ids.view(np.int32)), ws, loss, stats)
    torch.cuda.synchronize()
    o = ostep.train_step(spec, sampler, kf, t64, w64, ids)
    usable = int(np.isfinite(kf0.depth_var).sum()) - 60
    st = stats.cpu().numpy()
    assert st[3] == 1024 - usable, (st, usable)
    got = loss.cpu().numpy()
    assert np.isfinite(got).all()
    assert got[0] == pytest.approx(o["loss"], rel=TOL)
    assert got[1] == pytest.approx(o["loss_rgb"], rel=TOL)
    assert got[2] == pytest.approx(o["loss_d"], rel=TOL)
    gtab, gws = split_grads(G.cpu().numpy(), lay, spec)
    check_mag("masked grad table", gtab, o["grad_table"], o["grad_table_mag"], TOL)
    for j in range(len(gws)):
        check_mag(f"masked grad W{j}", gws[j], o["grad_w"][j], o["grad_w_mag"][j], TOL)
    report(f"masking: {1024 - usable} of 1024 rays without a usable depth, loss {got[0]:.6f}")
