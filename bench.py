"""Benchmark of the NeRF-SLAM mapping step on one MI355X.

Workload: the paper-scale step -- 16-level hash grid with 2^19 entries per
level, density net 32->64->16, colour net 32->64->64->3, 128^3 occupancy grid
of a 64-blob scene, 8 keyframes of 640x480, 4096 pixel candidates per step
cut at 2^18 samples (1..256 samples per ray).  A step is nsl_train_step:
rays + march + field forward + compositing/loss + recompute backward to
parameter gradients (headline); the full step adds Adam.  Inputs are resident
in device memory before timing starts.

Prints ONE JSON line.  Extra keys: per-phase times from HIP events recorded
between the phases on the step's stream, the roofline of the dominant kernel,
and the FP64 oracle timed on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "train samples/s (fwd+bwd) mixed vs FP32; render rays/s; p50/p99 render latency"
PEAK_HBM = 8.0e12          # B/s, MI355X HBM3E
PEAK_FP32 = 157.3e12       # FLOP/s, MI355X FP32 (matrix and vector)
N_CANDIDATES = 4096
N_SETS = 4                 # candidate sets rotated over the timed steps


def mlp_macs(spec):
    """Multiply-accumulates per sample: forward, input-gradient, weight-gradient."""
    dims = spec.mlp_dims()
    fwd = sum(a * b for a, b in dims)
    # no input gradient for the SH inputs of the first colour layer
    dx = fwd - spec.sh_bands ** 2 * dims[2][1]
    return fwd, dx, fwd


def gather_bytes(spec, elem=4):
    return 8 * spec.levels * spec.feat_per_level * elem


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-candidates", type=int, default=1536)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy first (reference kernel for HBM counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the step shards over rays; see the design notes).", file=sys.stderr)
        return 2

    import torch

    import workloads as W
    from paper_2210_13641_amd import nsl

    dev = torch.device("cuda:0")
    spec, sampler = W.C2_FIELD, W.C2_SAMPLER
    scene = W.c2_scene()
    occ = W.c2_occupancy(scene)
    kf = W.c2_keyframes(scene)
    K, H, Wd = kf.rgb.shape[:3]
    field = nsl.Field(spec)
    lay = field.layout
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    mapper = nsl.Mapper(K, H, Wd, sampler.grid_res, device=dev)
    mapper.upsert(list(range(K)), t(kf.rgb), t(kf.pose.reshape(K, 12)), t(kf.intr), t(kf.depth), t(kf.depth_var))
    mapper.set_occupancy(t(occ.view(np.int32)))
    table, ws = W.init_params(0, lay["table_floats"], spec.mlp_dims())
    flat = np.zeros(lay["total"], np.float32)
    flat[:len(table)] = table
    for off, w in zip(lay["w_offsets"], ws):
        flat[off:off + w.size] = w.ravel()
    P = t(flat)
    G = torch.zeros_like(P)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    id_sets = [t(W.c2_candidates(N_CANDIDATES, seed=3 + i).view(np.int32)) for i in range(N_SETS)]
    cfg = nsl.step_config(sampler, zero_grads=True)
    cfg_full = nsl.step_config(sampler, zero_grads=False, do_adam=True, lr=W.ADAM_LR, betas=W.ADAM_BETAS,
                               eps=W.ADAM_EPS, adam_step=1)
    wsb = torch.empty(nsl.step_workspace_bytes(field, cfg, N_CANDIDATES), dtype=torch.uint8, device=dev)
    loss = torch.zeros(3, device=dev)
    stats = torch.zeros(N_SETS, 4, dtype=torch.int32, device=dev)

    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step(i, c=cfg, stats_row=None):
        nsl.train_step(mapper, field, P, G, M, V, c, id_sets[i % N_SETS], wsb, loss,
                       stats[i % N_SETS] if stats_row is None else stats_row)

    # headline: fwd + bwd to parameter gradients
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = stats.cpu().numpy()
    S_sets = st[:, 1].astype(np.int64)
    R_sets = st[:, 0].astype(np.int64)
    samples = sum(int(S_sets[i % N_SETS]) for i in range(args.steps))
    ms_per_step = 1e3 * dt / args.steps
    value = samples / dt

    # full step with Adam (Adam clears the gradient, so no separate clearing)
    G.zero_()
    for i in range(args.warmup):
        cfg_full.adam_step = i + 1
        step(i, cfg_full)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        cfg_full.adam_step = args.warmup + i + 1
        step(i, cfg_full)
    torch.cuda.synchronize()
    dt_full = time.perf_counter() - t0
    full_value = samples / dt_full

    # phase times from HIP events on the step's stream
    n_prof = max(10, min(args.steps, 50))
    P.copy_(t(flat))
    nsl.profile_enable(True)
    for i in range(n_prof):
        cfg_full.adam_step = i + 1
        step(i, cfg_full)
    phases, n_done = nsl.profile_read()
    nsl.profile_enable(False)
    phase_ms = {k: v / n_done for k, v in phases.items()}
    S_prof = float(np.mean([S_sets[i % N_SETS] for i in range(n_prof)]))

    # roofline of the dominant kernel
    fwd_mac, dx_mac, dw_mac = mlp_macs(spec)
    gb = gather_bytes(spec)
    work = {
        "field_fwd": dict(flops=2 * fwd_mac, bytes=gb),
        "field_bwd": dict(flops=2 * (dx_mac + dw_mac), bytes=gb),   # scatter of the table gradient
    }
    dom = max(("field_fwd", "field_bwd"), key=lambda k: phase_ms[k])
    w = work[dom]
    t_s = phase_ms[dom] * 1e-3
    mfma_bound = w["flops"] / PEAK_FP32 >= w["bytes"] / PEAK_HBM
    if mfma_bound:
        achieved = w["flops"] * S_prof / t_s / 1e12
        roof = dict(bound="mfma", achieved=achieved, peak=PEAK_FP32 / 1e12, unit="TFLOP/s",
                    frac=achieved / (PEAK_FP32 / 1e12), traffic=None)
    else:
        achieved = w["bytes"] * S_prof / t_s / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=PEAK_HBM / 1e9, unit="GB/s",
                    frac=achieved / (PEAK_HBM / 1e9), traffic=None)
    roof.update(kernel=dom, per_sample=dict(flops=w["flops"], bytes=w["bytes"]), samples_per_launch=S_prof,
                launch_ms=phase_ms[dom])
    # whole fwd+bwd step against its own bound
    step_bytes = 2 * gb
    step_flops = 2 * (fwd_mac + dx_mac + dw_mac)
    t_bound = max(step_bytes / PEAK_HBM, step_flops / PEAK_FP32)
    step_roof = dict(bound_s_per_sample=t_bound, frac=(value * t_bound), per_sample=dict(
        flops=step_flops, bytes=step_bytes))

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "paper-scale FP32 mapping step: 16 levels x 2^19 hash grid, 2^18-sample cut, "
                        "8 keyframes 640x480, 128^3 occupancy (64-blob scene)",
            "candidates_per_step": N_CANDIDATES,
            "rays_per_step": float(R_sets.mean()),
            "samples_per_step": float(S_sets.mean()),
            "mean_samples_per_ray": float(S_sets.sum() / max(R_sets.sum(), 1)),
            "phase": "fwd+bwd to parameter gradients (gradient clearing included)",
        },
        "full_step_samples_per_s": full_value,
        "full_step_ms": 1e3 * dt_full / args.steps,
        "phases_ms": phase_ms,
        "roofline": roof,
        "roofline_step": step_roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, sampler, kf, occ, table, ws, lay, args.cpu_candidates)
    print(json.dumps(out), flush=True)
    return 0


def cpu_baseline(spec, sampler, kf, occ, table, ws, lay, n_cand):
    """The FP64 oracle as it stands, on the first n_cand candidates of the
    first candidate set (one step, FP32-rounded parameters)."""
    import workloads as W
    from oracle import step as ostep
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads") or 1) for i in threadpool_info()) if threadpool_info() else 1
    except Exception:                     # threadpoolctl missing: numpy's default
        threads = os.cpu_count()
    t64 = np.asarray(table, np.float32).astype(np.float64)
    w64 = [np.asarray(w, np.float32).astype(np.float64) for w in ws]
    ids = W.c2_candidates(N_CANDIDATES, seed=3)[:n_cand]
    t0 = time.perf_counter()
    r = ostep.train_step(spec, sampler, kf, t64, w64, ids, occupancy=occ)
    dt = time.perf_counter() - t0
    return dict(value=r["S"] / dt, unit="samples/s", cores=int(threads), kind="oracle",
                sample=f"one fwd+bwd step of the FP64 oracle on the first {n_cand} of the {N_CANDIDATES} "
                       f"candidates ({r['S']} samples, {r['R']} rays), {dt:.1f} s wall")


if __name__ == "__main__":
    sys.exit(main())
