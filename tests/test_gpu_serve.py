"""Serving: continuous batching of render requests interleaved with training.
Each request's pixels equal those of the same request rendered alone with
its parameter snapshot (bit for bit), and a small request matches the
oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import step as ostep
from parity import check_mag, params_for, report, upload_keyframes

pytestmark = pytest.mark.gpu


def _t(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def test_serving_mix_equals_alone_and_oracle(nsl, gpu):
    import torch
    from paper_2210_13641_amd import serve
    dev = gpu
    report("serve: two bursts of 7 requests, 40 ms apart, with training every 2 ms")
    spec = W.C1_FIELD
    f = nsl.Field(spec)
    flat, _, _ = params_for(spec, f.layout, seed=3, table_range=1.0)
    P = _t(torch, dev, flat)
    G = torch.zeros_like(P)
    M, V = torch.zeros_like(P), torch.zeros_like(P)
    kf = W.c1_keyframes()
    mapper = upload_keyframes(nsl, torch, kf, dev)
    ids = _t(torch, dev, W.c1_pixels().view(np.int32))
    scfg = nsl.step_config(W.C1_SAMPLER, zero_grads=False, do_adam=True, lr=1e-2)
    wsb = torch.empty(nsl.step_workspace_bytes(f, scfg, 1024), dtype=torch.uint8, device=dev)
    loss = torch.zeros(3, device=dev)
    step = [0]

    def train():
        step[0] += 1
        scfg.adam_step = step[0]
        nsl.train_step(mapper, f, P, G, M, V, scfg, ids, wsb, loss)

    train()                                                # first-call costs outside the loop
    torch.cuda.synchronize()
    reqs = W.serve_requests(14, seed=11, rate=2000.0)
    sizes = [(15, 20), (120, 160), (48, 64), (240, 320)]
    for i, q in enumerate(reqs):
        # two bursts 40 ms apart: requests of a burst share launches, and
        # training publishes new snapshots between the bursts
        q["arrival"] = 1e-4 * (i % 7) + (0.04 if i >= 7 else 0.0)
        q["H"], q["W"] = sizes[i % 4]
        q["intr"] = np.array([0.9375 * q["W"], 0.9375 * q["W"], q["W"] / 2, q["H"] / 2], np.float32)
        q["pose"] = q["pose"].reshape(12)
    rcfg = nsl.render_config(0.5, 2.0 / 32, 32, 1e-4)
    srv, done, stats = serve.serve(f, rcfg, dev, reqs, P, train_fn=train, train_period=2e-3,
                                   tiles_per_launch=300, keep_snapshots=True)
    report(f"  {stats}")
    assert len(done) == 14 and all(r.latency is not None and r.latency >= 0 for r in done)
    assert stats["max_requests_per_launch"] >= 2          # requests shared launches
    assert len({r.snap.version for r in done}) >= 2        # training moved the snapshot
    for r in done:
        ws = torch.empty(nsl.render_workspace_bytes(f, r.H, r.W, rcfg), dtype=torch.uint8, device=dev)
        op = torch.empty(r.H * r.W, device=dev)
        alone = nsl.render(f, r.snap.params, _t(torch, dev, np.asarray(r.pose, np.float32)),
                           _t(torch, dev, r.intr), r.H, r.W, rcfg, ws, opacity=op)
        torch.cuda.synchronize()
        for a, b in zip(alone, r.out):
            assert torch.equal(a, b), r.rid
    small = [r for r in done if r.H == 15][0]
    snap = small.snap.params.cpu().numpy()
    lay = f.layout
    t64 = snap[:lay["table_floats"]].astype(np.float64)
    w64 = [snap[o:o + a * b].astype(np.float64).reshape(a, b) for o, (a, b) in zip(lay["w_offsets"], spec.mlp_dims())]
    sampler = W.SamplerSpec(mode="uniform", t_near=0.5, t_far=2.5, dt=2.0 / 32, n_uniform=32)
    o = ostep.render_image(spec, t64, w64, np.asarray(small.pose).reshape(3, 4), small.intr, 15, 20, sampler,
                           stop_T=1e-4)
    ok = np.array([r not in o["alt"] for r in range(300)])
    got = small.out[0].cpu().numpy()
    check_mag("served rgb", got[ok], o["rgb"][ok], o["rgb_mag"][ok], 1e-5)


def test_serving_budget_queues_and_rejects(nsl, gpu):
    """A memory budget that holds one parameter snapshot and the outputs of
    two 48x64 requests: ten such requests arriving together queue (at most
    two are admitted at any time, and a request bound to a newer snapshot
    also waits until the older snapshot's requests have finished), a
    1280x960 request that can never fit is rejected with NSL_E_BUDGET while
    the others complete, and every completed request equals the same
    request rendered alone."""
    import torch
    from paper_2210_13641_amd import serve
    dev = gpu
    spec = W.C1_FIELD
    f = nsl.Field(spec)
    flat, _, _ = params_for(spec, f.layout, seed=3, table_range=1.0)
    P = _t(torch, dev, flat)
    G, M, V = torch.zeros_like(P), torch.zeros_like(P), torch.zeros_like(P)
    kf = W.c1_keyframes()
    mapper = upload_keyframes(nsl, torch, kf, dev)
    ids = _t(torch, dev, W.c1_pixels().view(np.int32))
    scfg = nsl.step_config(W.C1_SAMPLER, zero_grads=False, do_adam=True, lr=1e-2)
    wsb = torch.empty(nsl.step_workspace_bytes(f, scfg, 1024), dtype=torch.uint8, device=dev)
    loss = torch.zeros(3, device=dev)
    step = [0]

    def train():
        step[0] += 1
        scfg.adam_step = step[0]
        nsl.train_step(mapper, f, P, G, M, V, scfg, ids, wsb, loss)

    train()
    torch.cuda.synchronize()
    snap_bytes = P.numel() * 4 + nsl.prepared_bytes(f)
    out_bytes = 48 * 64 * serve.OUT_BYTES_PER_PIXEL
    budget = snap_bytes + 2 * out_bytes + out_bytes // 2
    reqs = W.serve_requests(11, seed=5, rate=2000.0)
    for i, q in enumerate(reqs):
        q["arrival"] = 1e-4 * i
        q["H"], q["W"] = (960, 1280) if i == 4 else (48, 64)
        q["intr"] = np.array([0.9375 * q["W"], 0.9375 * q["W"], q["W"] / 2, q["H"] / 2], np.float32)
        q["pose"] = q["pose"].reshape(12)
    rcfg = nsl.render_config(0.5, 2.0 / 32, 32, 1e-4)
    srv, done, stats = serve.serve(f, rcfg, dev, reqs, P, train_fn=train, train_period=1e-3, budget_bytes=budget,
                                   tiles_per_launch=16, keep_snapshots=True)
    report(f"  budget {budget} B: {stats}")
    assert [r.rid for r in srv.rejected] == [4] and srv.rejected[0].error == nsl.E_BUDGET
    assert len(done) == 10 and all(r.error == 0 and r.latency is not None for r in done)
    assert stats["peak_used_bytes"] <= budget and stats["rejected"] == 1
    held = np.array(srv.admission_log)
    assert held[:, 0].max() == 2, held            # at most two requests hold memory at once
    assert held[:, 1].max() == 1, held            # ... and then they share their snapshot
    assert len({r.snap.version for r in done}) >= 2                 # training moved the snapshot meanwhile
    assert max(r.admitted - r.arrival for r in done) > 0        # some requests queued
    for r in done:
        ws = torch.empty(nsl.render_workspace_bytes(f, r.H, r.W, rcfg), dtype=torch.uint8, device=dev)
        op = torch.empty(r.H * r.W, device=dev)
        alone = nsl.render(f, r.snap.params, _t(torch, dev, np.asarray(r.pose, np.float32)),
                           _t(torch, dev, r.intr), r.H, r.W, rcfg, ws, opacity=op)
        torch.cuda.synchronize()
        for a, b in zip(alone, r.out):
            assert torch.equal(a, b), r.rid
