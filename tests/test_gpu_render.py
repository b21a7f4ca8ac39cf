"""Rendering (forward only, early termination) and batched rendering of
several requests against the oracle and against themselves alone."""
import numpy as np
import pytest

import workloads as W
from oracle import step as ostep
from parity import check_mag, params_for, report

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _t(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _sampler(t_near, dt, n):
    return W.SamplerSpec(mode="uniform", t_near=t_near, t_far=t_near + n * dt, dt=dt, n_uniform=n)


def _render(nsl, torch, dev, f, P, pose, intr, H, Wd, cfg):
    ws = torch.empty(nsl.render_workspace_bytes(f, H, Wd, cfg), dtype=torch.uint8, device=dev)
    op = torch.empty(H * Wd, device=dev)
    rgb, depth, var, _ = nsl.render(f, P, _t(torch, dev, pose.reshape(12)), _t(torch, dev, intr), H, Wd, cfg, ws,
                                    opacity=op)
    torch.cuda.synchronize()
    return rgb.cpu().numpy(), depth.cpu().numpy(), var.cpu().numpy(), op.cpu().numpy()


@pytest.mark.parametrize("spec,stop_T,n,H,Wd", [(W.C1_FIELD, 0.0, 32, 18, 27), (W.C1_FIELD, 0.3, 32, 18, 27),
                                                (W.C2_FIELD, 0.0, 32, 18, 27), (W.C2_FIELD, 0.3, 32, 18, 27),
                                                (W.C1_FIELD, 0.0, 200, 18, 27), (W.C2_FIELD, 0.3, 200, 9, 11),
                                                (W.C2_FIELD, 0.0, 1024, 5, 13)],
                         ids=["tiny", "tiny-stop", "full", "full-stop", "tiny-200", "full-stop-200", "full-1024"])
def test_render_matches_oracle(nsl, gpu, spec, stop_T, n, H, Wd):
    """Rendered colour, depth, opacity and V* against the oracle's render at
    1e-5 of their magnitudes; images are not a multiple of the 64-pixel tile,
    and the sample counts include a ragged last tile (200) and the largest
    count a ray may take (1024)."""
    import torch
    dev = gpu
    report(f"render: levels={spec.levels} {Wd}x{H} n={n} stop_T={stop_T}")
    f = nsl.Field(spec)
    flat, t64, w64 = params_for(spec, f.layout, seed=8, table_range=2.0)
    pose = W.look_at_pose((1.5 * np.cos(0.4), 1.5 * np.sin(0.4), 0.2)).astype(np.float32)
    intr = np.array([0.9375 * Wd, 0.9375 * Wd, Wd / 2, H / 2], np.float32)
    t_near, dt = 0.5, 2.0 / n
    cfg = nsl.render_config(t_near, dt, n, stop_T)
    rgb, depth, var, op = _render(nsl, torch, dev, f, _t(torch, dev, flat), pose, intr, H, Wd, cfg)
    o = ostep.render_image(spec, t64, w64, pose, intr, H, Wd, _sampler(t_near, dt, n), stop_T=stop_T)
    ok = np.ones(H * Wd, bool)
    for r, alts in o["alt"].items():          # stop undecided in float32: accept either
        ok[r] = False
        cands = [dict(rgb=o["rgb"][r], depth_z=o["depth_z"][r], opacity=o["opacity"][r])] + alts
        assert any(np.allclose(rgb[r], c["rgb"], rtol=1e-4, atol=1e-6) for c in cands)
    if stop_T > 0:
        assert (o["n_used"] < n).any()         # termination actually happened
    check_mag("rgb", rgb[ok], o["rgb"][ok], o["rgb_mag"][ok], TOL)
    check_mag("depth", depth[ok], o["depth_z"][ok], o["depth_z_mag"][ok], TOL)
    check_mag("opacity", op[ok], o["opacity"][ok], o["opacity_mag"][ok], TOL)
    check_mag("var", var[ok], o["var_z"][ok], o["var_z_mag"][ok], TOL)


def test_render_batch_is_independent_of_the_mix(nsl, gpu):
    """Three requests (different sizes and parameter snapshots) in one launch,
    with ragged tiles, a tile of an unknown request and a tile past the image:
    every pixel equals the request rendered alone, bit for bit."""
    import torch
    dev = gpu
    spec = W.C1_FIELD
    f = nsl.Field(spec)
    n = 32
    cfg = nsl.render_config(0.5, 2.0 / n, n, 1e-4)
    sizes = [(13, 21), (40, 50), (7, 9)]
    snaps, reqs, outs = [], [], []
    for i, (H, Wd) in enumerate(sizes):
        flat, _, _ = params_for(spec, f.layout, seed=20 + i, table_range=1.5)
        P = _t(torch, dev, flat)
        prep = nsl.prepare(f, P)
        pose = W.look_at_pose((1.5 * np.cos(i), 1.5 * np.sin(i), 0.0)).astype(np.float32)
        intr = np.array([0.9375 * Wd, 0.9375 * Wd, Wd / 2, H / 2], np.float32)
        o = [torch.full((H * Wd, 3), -1.0, device=dev), torch.full((H * Wd,), -1.0, device=dev),
             torch.full((H * Wd,), -1.0, device=dev), torch.full((H * Wd,), -1.0, device=dev)]
        snaps.append((P, prep, pose, intr))
        outs.append(o)
        reqs.append(nsl.render_request(P, prep, pose.reshape(12), intr, H, Wd, *o))
    tiles = []
    rng = np.random.default_rng(0)
    for i, (H, Wd) in enumerate(sizes):
        p = 0
        while p < H * Wd:                       # ragged tile sizes
            k = int(rng.integers(1, 65))
            tiles.append(nsl.RenderTile(i, p, k))
            p += k
    tiles.append(nsl.RenderTile(7, 0, 64))      # unknown request: skipped
    tiles.append(nsl.RenderTile(0, 10 ** 6, 64))  # past the image: skipped
    order = rng.permutation(len(tiles))
    tiles = [tiles[i] for i in order]
    rq = nsl.records_to_device(reqs, nsl.RenderRequest, dev)
    tl = nsl.records_to_device(tiles, nsl.RenderTile, dev)
    nsl.render_batch(f, rq, len(reqs), tl, len(tiles), cfg)
    torch.cuda.synchronize()
    for i, (H, Wd) in enumerate(sizes):
        P, prep, pose, intr = snaps[i]
        alone = _render(nsl, torch, dev, f, P, pose, intr, H, Wd, cfg)
        for a, b in zip(alone, outs[i]):
            assert np.array_equal(a.reshape(-1), b.cpu().numpy().reshape(-1)), i
