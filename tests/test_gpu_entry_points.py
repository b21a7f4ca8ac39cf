"""The kernel-level entry points on their own, through the C ABI, against the
FP64 oracle: the mapping loss and its seeds (nsl_loss_fwd / nsl_loss_bwd),
the hash-grid encoding in both precisions (nsl_encode_fwd[_mixed]) and the
table-gradient scatter from a given dL/de (nsl_encode_bwd)."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import field as ofield
from oracle import render as orender
from parity import check_mag, params_for, report, split_grads

pytestmark = pytest.mark.gpu


def _t(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _loss_inputs(R, seed):
    rng = np.random.default_rng(seed)
    out = np.zeros((R, 6), np.float32)
    out[:, :3] = rng.uniform(size=(R, 3))
    out[:, 3] = rng.uniform(0.5, 3.0, R)
    out[:, 4] = rng.uniform(0, 0.1, R)
    out[:, 5] = rng.uniform(size=R)
    rgb = rng.uniform(size=(R, 3)).astype(np.float32)
    s = rng.uniform(1.0, 1.4, R).astype(np.float32)
    dz = (rng.uniform(0.5, 3.0, R) / s).astype(np.float32)
    var = np.exp(rng.uniform(np.log(1e-4), np.log(1.0), R)).astype(np.float32)
    bad = rng.choice(R, R // 10, replace=False)
    kinds = [(np.nan, None), (np.inf, None), (None, -1e-2), (None, 0.0), (None, np.nan), (None, np.inf)]
    for j, r in enumerate(bad):
        d_, v_ = kinds[j % len(kinds)]
        if d_ is not None:
            dz[r] = d_
        if v_ is not None:
            var[r] = v_
    return out, rgb, dz, var, s


@pytest.mark.parametrize("R", [1, 63, 3001])
def test_loss_entry_points_match_oracle(nsl, gpu, R):
    """L, L_rgb, L_D and the masked count of nsl_loss_fwd, and the seeds of
    nsl_loss_bwd for upstream gradients (1, 0, 0) and a random triple, against
    the oracle's loss terms and seeds (Eq. 3, 4, 7) at 1e-5."""
    import torch
    dev = gpu
    out, rgb, dz, var, s = _loss_inputs(R, seed=R)
    lam = 0.7
    T = [_t(torch, dev, a) for a in (out, rgb, dz, var, s)]
    nm = torch.zeros(1, dtype=torch.int32, device=dev)
    loss = nsl.loss_fwd(T[0], T[1], T[2], T[3], T[4], lam, n_masked=nm).cpu().numpy()
    s64 = s.astype(np.float64)
    prec, ok = orender.precision_from_variance(dz, var, s64)
    Dray = np.where(ok, dz.astype(np.float64) * s64, 0.0)
    C, D = out[:, :3].astype(np.float64), out[:, 3].astype(np.float64)
    l_rgb, l_d, gC, gD1, gCm, gD1m = orender.loss_seeds(C, D, rgb, Dray, prec, R, 1.0)
    Lr, Ld = l_rgb.sum() / R, l_d.sum() / R
    assert int(nm.item()) == int((~ok).sum())
    assert loss[1] == pytest.approx(Lr, rel=1e-5)
    assert loss[2] == pytest.approx(Ld, rel=1e-5)
    assert loss[0] == pytest.approx(Lr + lam * Ld, rel=1e-5)
    for up in (None, np.array([0.3, -1.2, 2.5], np.float32)):
        a, b, c = (1.0, 0.0, 0.0) if up is None else up.astype(np.float64)
        g = nsl.loss_bwd(T[0], T[1], T[2], T[3], T[4], lam, None if up is None else _t(torch, dev, up))
        g = g.cpu().numpy()
        check_mag("loss seed rgb", g[:, :3], (a + b) * gC, abs(a + b) * gCm + 1e-30, 1e-5)
        check_mag("loss seed depth", g[:, 3], (a * lam + c) * gD1, abs(a * lam + c) * gD1m + 1e-30, 1e-5)
        assert np.all(g[:, 4:] == 0)
    report(f"loss entry points: R={R}, {int((~ok).sum())} masked")


@pytest.mark.parametrize("spec,S", [(W.C1_FIELD, 1037), (W.C2_FIELD, 1037), (W.C2_FIELD, 65537)],
                         ids=["tiny", "full", "full-64k"])
def test_encode_entry_points_match_oracle(nsl, gpu, spec, S):
    """nsl_encode_fwd (FP32 table) at 1e-5 and nsl_encode_fwd_mixed (FP16 table
    copy, BF16 pairs) at 2e-2 of the oracle encoding's magnitudes, level-major."""
    import torch
    dev = gpu
    f = nsl.Field(spec)
    flat, t64, _ = params_for(spec, f.layout, seed=3, table_range=0.5)
    rng = np.random.default_rng(S)
    xn = rng.uniform(size=(S, 3)).astype(np.float32)
    xn[:5] = [[0, 0, 0], [1, 1, 1], [0.5, 0.5, 0.5], [1, 0, 1], [0.25, 0.75, 1.0]]
    P = _t(torch, dev, flat)
    X = _t(torch, dev, xn)
    e = nsl.encode_fwd(f, P, X).cpu().numpy()                       # [L, S, 2]
    want, mag, _ = ofield.encode_fwd(spec, t64, xn)                  # [S, 2L]
    L = spec.levels
    got = e.transpose(1, 0, 2).reshape(S, 2 * L)
    check_mag("encoding fp32", got, want, mag, 1e-5)
    shadow = f.prepare_mixed(P)
    em = nsl.encode_fwd_mixed(f, shadow, X).cpu().numpy().view(np.uint32)   # [L, S]
    lo = ((em & 0xFFFF).astype(np.uint32) << 16).view(np.float32)
    hi = (em & 0xFFFF0000).astype(np.uint32).view(np.float32)
    gotm = np.stack([lo, hi], -1).transpose(1, 0, 2).reshape(S, 2 * L)
    check_mag("encoding mixed", gotm, want, mag, 2e-2)


# The tiny network over 2^22-entry levels: a dense level of 129^3 entries
# (263 bins) and three hashed levels of 512 bins, so that a level has more
# bins than the placement has threads and each thread owns several.
LARGE_TABLE = dataclasses.replace(W.C1_FIELD, log2_table=22, base_res=128)


@pytest.mark.parametrize("spec,S,unpaired", [(W.C1_FIELD, 2049, False), (W.C2_FIELD, 4099, False),
                                             (W.C2_FIELD, 65537, False), (LARGE_TABLE, 65537, False),
                                             (W.C2_FIELD, 4099, True)],
                         ids=["tiny", "full", "full-64k", "large-table", "full-unpaired"])
def test_encode_bwd_entry_point_matches_oracle(nsl, gpu, spec, S, unpaired):
    """nsl_encode_bwd scatters a random dL/de into the table gradient: every
    table entry against the oracle's scatter at 1e-5 (FP32 records) and 2e-2
    (BF16 records), overwriting (untouched entries become 0) and
    accumulating onto a prior value; the weights' part of grads is left
    alone.  unpaired: the first 1024 samples lie in x-cell 127 of the finest
    level (2048 cells a side), whose x-neighbour corners differ in eight low
    bits of the hashed index and so travel as two records, not one paired
    record: those units hold more records than the placement stages."""
    import torch
    dev = gpu
    f = nsl.Field(spec)
    lay = f.layout
    rng = np.random.default_rng(S + 1)
    xn = rng.uniform(size=(S, 3)).astype(np.float32)
    if unpaired:
        assert spec.levels == 16 and spec.max_res == 2048
        xn[:1024, 0] = ((127.0 + rng.uniform(0.05, 0.95, 1024)) / 2048.0).astype(np.float32)
    else:
        xn[: S // 4] = np.clip(0.5 * xn[0] + 1e-3 * rng.uniform(size=(S // 4, 3)), 0, 1)   # shared cells
    de = rng.normal(size=(spec.levels, S, 2)).astype(np.float32)
    _, _, corners = ofield.encode_fwd(spec, np.zeros(lay["table_floats"]), xn)
    de_sf = de.transpose(1, 0, 2).reshape(S, 2 * spec.levels).astype(np.float64)
    gt, gtm = ofield.encode_bwd(spec, corners, de_sf, np.abs(de_sf), lay["table_floats"])
    X, DE = _t(torch, dev, xn), _t(torch, dev, de)
    nt = lay["table_floats"]
    for prec, tol in ((nsl.PRECISION_FP32, 1e-5), (nsl.PRECISION_MIXED, 2e-2)):
        G = torch.full((lay["total"],), 7.0, device=dev)
        nsl.encode_bwd(f, X, DE, G, precision=prec, overwrite=True)
        g = G.cpu().numpy()
        check_mag(f"encode bwd overwrite p{prec}", g[:nt], gt, gtm, tol)
        assert np.all(g[nt:] == 7.0)
        assert np.all(g[:nt][gtm == 0] == 0)
        G = torch.full((lay["total"],), 0.5, device=dev)
        nsl.encode_bwd(f, X, DE, G, precision=prec, overwrite=False)
        g = G.cpu().numpy().astype(np.float64)
        check_mag(f"encode bwd accumulate p{prec}", g[:nt], gt + 0.5, gtm + 0.5, tol)
        assert np.all(g[nt:] == 0.5)
    report(f"encode bwd: {spec.levels} levels, S={S}, {int(np.count_nonzero(gtm))} entries touched")


@pytest.mark.parametrize("spec,S", [(W.C1_FIELD, 1037), (W.C2_FIELD, 1037), (W.C2_FIELD, 65537)],
                         ids=["tiny", "full", "full-64k"])
def test_mlp_entry_points_match_oracle(nsl, gpu, spec, S):
    """nsl_mlp_fwd and nsl_mlp_bwd on a given level-major encoding: sigma and
    colour, dL/de and every weight gradient against the oracle's networks at
    1e-5 of their magnitudes; the weight gradients accumulate onto what
    grads held, and the table part of grads is left alone."""
    import torch
    dev = gpu
    f = nsl.Field(spec)
    lay = f.layout
    flat, _, w64 = params_for(spec, lay, seed=5, table_range=0.5)
    rng = np.random.default_rng(S + 7)
    L = spec.levels
    e = rng.normal(scale=0.3, size=(S, 2 * L)).astype(np.float32)
    e[:3] = 0.0                                     # samples whose encoding is zero
    d = rng.normal(size=(S, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    enc = np.ascontiguousarray(e.reshape(S, L, 2).transpose(1, 0, 2))
    P, E, D = _t(torch, dev, flat), _t(torch, dev, enc), _t(torch, dev, d)
    ws = torch.empty(f.workspace_bytes(S), dtype=torch.uint8, device=dev)
    sig, rgb = nsl.mlp_fwd(f, P, E, D, ws)
    e64 = e.astype(np.float64)
    cache = ofield.mlp_fwd(spec, w64, e64, np.abs(e64), ofield.sh_basis(d.astype(np.float64), spec.sh_bands))
    check_mag("mlp sigma", sig.cpu().numpy(), cache["sigma"], cache["sigma_mag"], 1e-5)
    check_mag("mlp colour", rgb.cpu().numpy(), cache["colour"], cache["colour_mag"], 1e-5)
    dsig = rng.normal(size=S).astype(np.float32)
    drgb = rng.normal(size=(S, 3)).astype(np.float32)
    G = torch.full((lay["total"],), 0.5, device=dev)
    de = nsl.mlp_bwd(f, P, E, D, _t(torch, dev, dsig), _t(torch, dev, drgb), G, ws).cpu().numpy()
    dWs, dWm, de_o, dem = ofield.mlp_bwd(spec, w64, cache, dsig.astype(np.float64), np.abs(dsig).astype(np.float64),
                                         drgb.astype(np.float64), np.abs(drgb).astype(np.float64))
    check_mag("mlp dL/de", de.transpose(1, 0, 2).reshape(S, 2 * L), de_o, dem, 1e-5)
    g = G.cpu().numpy().astype(np.float64)
    gtab, gws = split_grads(g, lay, spec)
    assert np.all(gtab == 0.5)
    for j, (a, b, m) in enumerate(zip(gws, dWs, dWm)):
        check_mag(f"mlp grad W{j}", a, b + 0.5, m + 0.5, 1e-5)
    report(f"mlp entry points: {L} levels, S={S}")
