"""Benchmark of the NeRF-SLAM mapping step on one MI355X.

Training workload: the paper-scale step -- 16-level hash grid with 2^19
entries per level, density net 32->64->16, colour net 32->64->64->3, 128^3
occupancy grid of a 64-blob scene, 8 keyframes of 640x480, 4096 pixel
candidates per step cut at 2^18 samples (1..256 samples per ray).  A step is
nsl_train_step: rays + march + field forward + compositing/loss + backward to
parameter gradients (the headline; gradient clearing included), and the full
step adds Adam.  The backward recomputes the MLP; the headline keeps the
encoding from the forward (keep_encoding = 1), and the variant that gathers
it again is reported beside it.  It runs in mixed precision (FP16 tables,
BF16 MLP on MFMA, FP32 accumulation and masters; the headline value) and in
plain FP32.  Inputs are resident in device memory before timing starts.

Serving workload: render requests (Poisson arrivals at 200/s, image sizes
160x120 .. 1280x960, 32 samples, early termination at T < 1e-4) against the
tiny field after 300 training steps, while training continues at one step
per 5 ms; p50/p99 latency and rays/s.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "train samples/s (fwd+bwd) mixed vs FP32; render rays/s; p50/p99 render latency"
PEAK_HBM = 8.0e12          # B/s, MI355X HBM3E
PEAK_FP32 = 157.3e12       # FLOP/s, MI355X FP32 (matrix and vector)
PEAK_BF16 = 2.5e15         # FLOP/s, MI355X dense BF16 MFMA
N_CANDIDATES = 4096
N_SETS = 4                 # candidate sets rotated over the timed steps


def mlp_macs(spec):
    """Multiply-accumulates per sample: forward, input-gradient, weight-gradient."""
    dims = spec.mlp_dims()
    fwd = sum(a * b for a, b in dims)
    dx = fwd - spec.sh_bands ** 2 * dims[2][1]      # no input gradient for the SH inputs
    return fwd, dx, fwd


def kernel_work(spec, table_bytes):
    """Algorithmic work per sample of the steps of the path, as the profiler
    phases time them (the encoding kept from the forward, keep_encoding = 1):
      encode      the table gather, 8 corners x L levels x F features;
      field_fwd   the forward MLP;
      field_bwd   the MLP recomputed and its adjoint (input and weight
                  gradients);
      table_grad  the table-gradient scatter, 8 x L x F FP32 values (two
                  kernels: placement and reduction; the encoding kernel
                  counts the records per bin as it gathers, the forward and
                  compositing launches run the column scan and the bin
                  starts, and the placement launch also sums the weight
                  gradients and the loss)."""
    fwd_mac, dx_mac, dw_mac = mlp_macs(spec)
    n = 8 * spec.levels * spec.feat_per_level
    return {"encode": dict(flops=0, bytes=n * table_bytes),
            "field_fwd": dict(flops=2 * fwd_mac, bytes=0),
            "field_bwd": dict(flops=2 * (fwd_mac + dx_mac + dw_mac), bytes=0),
            "table_grad": dict(flops=0, bytes=n * 4)}


def roofline_of(name, work, samples, ms, mlp_peak):
    t = ms * 1e-3
    if work["flops"] / mlp_peak >= work["bytes"] / PEAK_HBM:
        a = work["flops"] * samples / t / 1e12
        r = dict(bound="mfma", achieved=a, peak=mlp_peak / 1e12, unit="TFLOP/s", frac=a / (mlp_peak / 1e12))
    else:
        a = work["bytes"] * samples / t / 1e9
        r = dict(bound="hbm", achieved=a, peak=PEAK_HBM / 1e9, unit="GB/s", frac=a / (PEAK_HBM / 1e9))
    r.update(traffic=None, kernel=name, per_sample=work, samples_per_launch=samples, launch_ms=ms)
    return r


PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_traffic_paper_scale.md")
PMC_SOURCES = ("field.hip", "field_mixed.hip", "field_common.h", "net.h", "common.h", "scatter.hip", "kernels.h",
               "bins.h")
BIN_KERNELS = ["bin_place_kernel<RecBF16, NetFull>", "bin_reduce_kernel<RecBF16>"]
PMC_ROWS = {("table_grad", 2): BIN_KERNELS,
            ("field_bwd", 2): ["mixed_bwd8_kernel<NetFull>"],
            ("field_fwd", 2): ["mixed_fwd_kernel<NetFull>"],
            ("encode", 2): ["encode_levels_kernel<NetFull, _Float16, unsigned int>"]}


def measured_traffic(phase, table_bytes):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) of the
    kernels of a phase, from the committed counter summary of the mixed
    headline step, or None when the kernel sources differ from those the
    counters were taken on (or the summary lacks a kernel)."""
    import hashlib
    if table_bytes != 2:
        return None
    try:
        text = open(PMC_SUMMARY).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for name in PMC_SOURCES:
        with open(os.path.join(ROOT, "paper_2210_13641_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    if f"kernel sources sha256: {h.hexdigest()}" not in text:
        return None
    rows = {}
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 4 and cells[0].startswith("`"):
            try:
                rows[cells[0].strip("`")] = (float(cells[2]) + float(cells[3])) * 1e6
            except ValueError:
                pass
    want = PMC_ROWS.get((phase, table_bytes), [])
    if not want or any(k not in rows for k in want):
        return None
    return sum(rows[k] for k in want)


def roofline(spec, phase_ms, samples, table_bytes, mlp_peak):
    """Rooflines of the steps of the path (HIP events on the step's stream)
    and the dominant one (the slowest)."""
    work = kernel_work(spec, table_bytes)
    all_r = {}
    for k in work:
        r = roofline_of(k, work[k], samples, phase_ms[k], mlp_peak)
        r["traffic"] = measured_traffic(k, table_bytes)
        if r["traffic"] is not None:
            r["traffic_unit"] = ("HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated; "
                                 "profiles/pmc_traffic_paper_scale.md)")
            r["algorithmic_bytes"] = work[k]["bytes"] * samples
        if k == "table_grad":
            r["kernels"] = ("bin_place, bin_reduce (the records are counted by the encoding kernel, the column "
                            "scan and bin starts run beside the forward MLP and the compositing; the placement "
                            "launch also sums the weight gradients and the loss, about 19 MB of its traffic)")
        all_r[k] = r
    dom = max(work, key=lambda k: phase_ms[k])
    return all_r[dom], all_r


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-candidates", type=int, default=N_CANDIDATES)
    ap.add_argument("--serve-requests", type=int, default=2200)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-only", action="store_true", help="only the serving workload")
    ap.add_argument("--only", default="", help="comma-separated step variants to time (counter runs); the JSON "
                    "line needs all four")
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
    if args.serve_only:
        print(json.dumps({"serving": serving(nsl, torch, dev, W, args.serve_requests, args.serve_warmup)}), flush=True)
        return 0
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
    scale = t(np.array([2.0 ** 15, 0, 0, 0], np.float32))
    variants = {"fp32": (False, False), "mixed": (True, False), "fp32_keep_encoding": (False, True),
                "mixed_keep_encoding": (True, True)}
    cfgs, full = {}, {}
    for name, (mx, keep) in variants.items():
        prec = dict(precision=nsl.PRECISION_MIXED, scale_state=scale) if mx else {}
        cfgs[name] = nsl.step_config(sampler, zero_grads=True, keep_encoding=keep, **prec)
        # a training loop's step: this step's gradients replace the last (the
        # table-gradient reduction overwrites them), then Adam
        full[name] = nsl.step_config(sampler, zero_grads=True, do_adam=True, lr=W.ADAM_LR, betas=W.ADAM_BETAS,
                                     eps=W.ADAM_EPS, keep_encoding=keep, **prec)
    wsb = torch.empty(max(nsl.step_workspace_bytes(field, c, N_CANDIDATES) for c in cfgs.values()),
                      dtype=torch.uint8, device=dev)
    loss = torch.zeros(3, device=dev)
    stats = torch.zeros(N_SETS, 4, dtype=torch.int32, device=dev)

    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step(i, c):
        nsl.train_step(mapper, field, P, G, M, V, c, id_sets[i % N_SETS], wsb, loss, stats[i % N_SETS])

    def timed(c, adam):
        """Wall time of args.steps steps (synchronised on both sides) and the
        per-step HIP-event durations on the step's stream."""
        P.copy_(t(flat))
        G.zero_()
        M.zero_()
        V.zero_()
        for i in range(args.warmup):
            c.adam_step = i + 1
            step(i, c)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        for i in range(args.steps):
            c.adam_step = args.warmup + i + 1
            step(i, c)
            ev[i + 1].record()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
        return dt, per

    res = {}
    names = [v for v in args.only.split(",") if v] or list(variants)
    for name in names:
        dt, per = timed(cfgs[name], False)
        st = stats.cpu().numpy()
        S_sets = st[:, 1].astype(np.int64)
        samples = sum(int(S_sets[i % N_SETS]) for i in range(args.steps))
        dt_full, per_full = timed(full[name], True)
        # per-phase HIP events on the step's stream
        P.copy_(t(flat))
        nsl.profile_enable(True)
        n_prof = max(10, min(args.steps, 50))
        for i in range(n_prof):
            full[name].adam_step = i + 1
            step(i, full[name])
        ph, n_done = nsl.profile_read()
        nsl.profile_enable(False)
        res[name] = dict(value=samples / dt, ms=1e3 * dt / args.steps, full_value=samples / dt_full,
                         full_ms=1e3 * dt_full / args.steps, phases={k: v / n_done for k, v in ph.items()},
                         S=float(np.mean([S_sets[i % N_SETS] for i in range(n_prof)])), R=st[:, 0].astype(np.int64),
                         step_ms=distribution(per), full_step_ms=distribution(per_full))
    if args.only:
        print(json.dumps({k: {"samples_per_s": v["value"], "phases_ms": v["phases"]} for k, v in res.items()}))
        return 0
    # headline: the forward keeps the encoding for the backward (the MLP is
    # recomputed in the backward either way); the recompute-only variants are
    # reported beside it
    mixed, fp32 = res["mixed_keep_encoding"], res["fp32_keep_encoding"]
    spr = samples_per_ray(nsl, torch, mapper, field, cfgs["fp32"], id_sets, wsb, dev, sampler.max_samples)
    roof, roofs = roofline(spec, mixed["phases"], mixed["S"], 2, PEAK_BF16)
    roof_fp32, roofs_fp32 = roofline(spec, fp32["phases"], fp32["S"], 4, PEAK_FP32)

    bound = PEAK_HBM / GATHER_BYTES_MIXED
    out = {
        "metric": METRIC,
        "value": mixed["value"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": "paper-scale mapping step: 16 levels x 2^19 hash grid, 2^18-sample cut, "
                        "8 keyframes 640x480, 128^3 occupancy (64-blob scene)",
            "precision": "mixed: FP16 tables, BF16 MLP on MFMA, FP32 accumulation, FP32 master weights, "
                         "dynamic loss scale from 2^15; transmittance, variance and loss in FP32",
            "candidates_per_step": N_CANDIDATES,
            "rays_per_step": float(mixed["R"].mean()),
            "samples_per_step": mixed["S"],
            "samples_per_ray": spr,
            "phase": "fwd+bwd to parameter gradients (gradient clearing included)",
            "backward": "recompute adjoint of the MLP; the encoding kept from the forward (keep_encoding = 1)",
        },
        "step_ms_hip_events": {"mixed": mixed["step_ms"], "fp32": fp32["step_ms"],
                               "mixed_full": mixed["full_step_ms"], "fp32_full": fp32["full_step_ms"]},
        "step_roofline": {
            "note": "whole mixed fwd+bwd step against the gather-bound roofline: HBM peak / (512 B FP16 gather + "
                    "1024 B FP32 scatter per sample); the gate is half of it",
            "bound_samples_per_s": bound, "frac": mixed["value"] / bound, "gate_frac": 0.5,
            "gate_samples_per_s": 0.5 * bound, "meets_gate": bool(mixed["value"] >= 0.5 * bound)},
        "fp32_samples_per_s": fp32["value"],
        "fp32_ms_per_step": fp32["ms"],
        "mixed_vs_fp32": mixed["value"] / fp32["value"],
        "full_step_samples_per_s": {"mixed": mixed["full_value"], "fp32": fp32["full_value"]},
        "phases_ms": {"mixed": mixed["phases"], "fp32": fp32["phases"]},
        "roofline": roof,
        "roofline_fp32": roof_fp32,
        "rooflines": {"mixed": roofs, "fp32": roofs_fp32},
        "recompute_encoding": {
            "note": "keep_encoding = 0: the backward gathers the table again instead of reading the encoding "
                    "the forward kept",
            "mixed_samples_per_s": res["mixed"]["value"],
            "fp32_samples_per_s": res["fp32"]["value"],
            "full_step_samples_per_s": {"mixed": res["mixed"]["full_value"], "fp32": res["fp32"]["full_value"]},
            "phases_ms": {"mixed": res["mixed"]["phases"], "fp32": res["fp32"]["phases"]},
        },
    }
    out["peaks_measured"] = measure_peaks(nsl, torch, dev)
    add_measured_fractions(out["rooflines"], out["peaks_measured"])
    del mapper, wsb, P, G, M, V
    torch.cuda.empty_cache()
    out["tiny_field_batches"] = tiny_field_batches(nsl, torch, dev, W, args.warmup, max(10, args.steps // 2))
    if args.serve_requests > 0:
        out["serving"] = serving(nsl, torch, dev, W, args.serve_requests, args.serve_warmup)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, sampler, kf, occ, table, ws, args.cpu_candidates)
        out["cpu_baseline_more"] = cpu_baseline_more(spec, sampler, kf, occ, table, ws)
    print(json.dumps(out), flush=True)
    return 0


GATHER_BYTES_MIXED = 8 * 16 * 2 * 2 + 8 * 16 * 2 * 4    # FP16 gather + FP32 scatter per paper-scale sample


def distribution(ms):
    """median, p10, p90, min, max of per-step milliseconds"""
    ms = np.asarray(ms, np.float64)
    return {"median": float(np.median(ms)), "p10": float(np.percentile(ms, 10)),
            "p90": float(np.percentile(ms, 90)), "min": float(ms.min()), "max": float(ms.max()), "n": int(ms.size)}


def _event_ms(torch, fn, reps):
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def measure_peaks(nsl, torch, dev):
    """Measured machine peaks (the library's probe kernels, HIP events):
    HBM stream copy, random 4-byte gathers from a 2 MB table (one FP16 hash
    level: L2-resident) and a 32 MB table (Infinity-Cache resident, about the
    size of the paper-scale FP16 table), and FP32 / BF16 MFMA loops."""
    out = {}
    n = 1 << 28                                            # 1 GiB each way
    src = torch.ones(n // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    ms = _event_ms(torch, lambda: nsl.peak_copy(src, dst), 10)
    out["hbm_copy_GBps"] = 2 * n / (ms * 1e-3) / 1e9
    del src, dst
    threads, loads = 256 * 4096, 256
    o = torch.empty(threads, dtype=torch.int32, device=dev)
    for name, log2 in (("gather_l2_2MB", 19), ("gather_mall_32MB", 23)):
        tab = torch.randint(0, 1 << 30, (1 << log2,), dtype=torch.int32, device=dev)
        ms = _event_ms(torch, lambda: nsl.peak_gather(tab, log2, o, loads), 10)
        out[name + "_Gloads_per_s"] = threads * loads / (ms * 1e-3) / 1e9
        out[name + "_GBps_4B"] = 4 * threads * loads / (ms * 1e-3) / 1e9
        del tab
    wg, iters = 1024, 1000
    f = torch.empty(wg * 256, dtype=torch.float32, device=dev)
    for name, bf16, flop in (("mfma_fp32_TFLOPs", False, 2048), ("mfma_bf16_TFLOPs", True, 16384)):
        ms = _event_ms(torch, lambda: nsl.peak_mfma(bf16, f, iters), 5)
        out[name] = wg * 4 * 8 * iters * flop / (ms * 1e-3) / 1e12
    return out


def add_measured_fractions(rooflines, peaks):
    """Each phase's achieved rate against the measured peak of its bound
    (HBM copy for the byte-bound phases, the MFMA loop of its precision for
    the MLP)."""
    for prec, phases in rooflines.items():
        for r in phases.values():
            if r["bound"] == "hbm":
                p = peaks["hbm_copy_GBps"]
            else:
                p = peaks["mfma_bf16_TFLOPs"] if prec == "mixed" else peaks["mfma_fp32_TFLOPs"]
            r["measured_peak"] = p
            r["frac_of_measured_peak"] = r["achieved"] / p


def tiny_field_batches(nsl, torch, dev, W, warmup, steps):
    """The tiny field (4 levels x 2^12) on batches of 2^18 and 2^20 samples
    (8 and 32 cameras of 32x32 pixels, 32 samples per ray): fwd+bwd samples/s
    in mixed precision and FP32, each with per-step HIP-event times."""
    import dataclasses
    spec = W.C1_FIELD
    f = nsl.Field(spec)
    lay = f.layout
    table, wts = W.init_params(0, lay["table_floats"], spec.mlp_dims())
    flat = np.zeros(lay["total"], np.float32)
    flat[:len(table)] = table
    for off, w in zip(lay["w_offsets"], wts):
        flat[off:off + w.size] = w.ravel()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    out = {}
    for n_cams in (8, 32):
        kf = W.c4_keyframes(n_cams)
        m = nsl.Mapper(n_cams, 32, 32, 1, device=dev)
        m.upsert(list(range(n_cams)), t(kf.rgb), t(kf.pose.reshape(n_cams, 12)), t(kf.intr), t(kf.depth),
                 t(kf.depth_var))
        ids = t(W.c1_pixels(K=n_cams).view(np.int32))
        sampler = dataclasses.replace(W.C1_SAMPLER, max_samples=n_cams * 1024 * 32)
        S = n_cams * 1024 * 32
        P = t(flat)
        G = torch.zeros_like(P)
        loss = torch.zeros(3, device=dev)
        row = {"samples_per_step": S}
        for prec_name, prec in (("mixed", nsl.PRECISION_MIXED), ("fp32", nsl.PRECISION_FP32)):
            st = torch.tensor([2.0 ** 15, 0, 0, 0], dtype=torch.float32, device=dev)
            cfg = nsl.step_config(sampler, zero_grads=True, keep_encoding=True, precision=prec,
                                  scale_state=st if prec == nsl.PRECISION_MIXED else None)
            ws = torch.empty(nsl.step_workspace_bytes(f, cfg, ids.numel()), dtype=torch.uint8, device=dev)
            for _ in range(warmup):
                nsl.train_step(m, f, P, G, None, None, cfg, ids, ws, loss)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
            torch.cuda.synchronize()
            ev[0].record()
            for i in range(steps):
                nsl.train_step(m, f, P, G, None, None, cfg, ids, ws, loss)
                ev[i + 1].record()
            torch.cuda.synchronize()
            per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
            row[prec_name] = {"samples_per_s": S * steps / (ev[0].elapsed_time(ev[-1]) * 1e-3),
                              "step_ms": distribution(per)}
            del ws
        row["mixed_vs_fp32"] = row["mixed"]["samples_per_s"] / row["fp32"]["samples_per_s"]
        out[f"2^{int(np.log2(S))}"] = row
    return out


def samples_per_ray(nsl, torch, mapper, field, cfg, id_sets, wsb, dev, max_samples):
    """Histogram (power-of-two bins) and mean of the samples per ray of the
    batches (rays: kept candidates with at least one sample)."""
    n = []
    for ids in id_sets:
        cnt = torch.zeros(ids.numel(), dtype=torch.int32, device=dev)
        off = torch.zeros(ids.numel() + 1, dtype=torch.int32, device=dev)
        tt = torch.zeros(max_samples, dtype=torch.float32, device=dev)
        ray = torch.zeros(max_samples, dtype=torch.int32, device=dev)
        nsl.march(mapper, field, cfg, ids, wsb, cnt, off, tt, ray)
        c, o = cnt.cpu().numpy().astype(np.int64), off.cpu().numpy().astype(np.int64)
        kept = (o[1:] <= max_samples) & (c > 0)
        n.append(c[kept])
    n = np.concatenate(n)
    edges = [1, 2, 4, 8, 16, 32, 64, 128, 256, 257]
    h, _ = np.histogram(n, bins=edges)
    return {"mean": float(n.mean()), "min": int(n.min()), "max": int(n.max()),
            "hist": {f"{a}-{b - 1}": int(x) for a, b, x in zip(edges[:-1], edges[1:], h)}}


def serving(nsl, torch, dev, W, n_req, warmup):
    """Render requests against the tiny field while it keeps training."""
    from paper_2210_13641_amd import serve
    spec = W.C1_FIELD
    f = nsl.Field(spec)
    lay = f.layout
    table, ws = W.init_params(0, lay["table_floats"], spec.mlp_dims())
    flat = np.zeros(lay["total"], np.float32)
    flat[:len(table)] = table
    for off, w in zip(lay["w_offsets"], ws):
        flat[off:off + w.size] = w.ravel()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    P = t(flat)
    G, M, V = torch.zeros_like(P), torch.zeros_like(P), torch.zeros_like(P)
    kf = W.c1_keyframes()
    m = nsl.Mapper(1, 32, 32, 1, device=dev)
    m.upsert([0], t(kf.rgb), t(kf.pose.reshape(1, 12)), t(kf.intr), t(kf.depth), t(kf.depth_var))
    ids = t(W.c1_pixels().view(np.int32))
    cfg = nsl.step_config(W.C1_SAMPLER, zero_grads=False, do_adam=True, lr=W.ADAM_LR, betas=W.ADAM_BETAS,
                          eps=W.ADAM_EPS)
    wsb = torch.empty(nsl.step_workspace_bytes(f, cfg, 1024), dtype=torch.uint8, device=dev)
    loss = torch.zeros(3, device=dev)
    n_step = [0]

    def train():
        n_step[0] += 1
        cfg.adam_step = n_step[0]
        nsl.train_step(m, f, P, G, M, V, cfg, ids, wsb, loss)

    for _ in range(300):                            # the trained field that is served
        train()
    torch.cuda.synchronize()
    rcfg = nsl.render_config(0.5, 2.0 / 32, 32, 1e-4)
    capacity = render_capacity(nsl, torch, dev, W, f, P, rcfg)
    reqs = W.serve_requests(n_req, seed=7, rate=200.0)
    for q in reqs:
        q["pose"] = q["pose"].reshape(12)
    train_samples = 1024 * 32
    _, done, st = serve.serve(f, rcfg, dev, reqs, P, train_fn=train, train_period=5e-3, warmup=warmup)
    st["train_samples_per_s"] = st["train_steps"] * train_samples / st["wall_s"]
    st["render_rays_per_s_idle"] = capacity
    st["workload"] = ("Poisson 200 req/s, sizes 160x120/320x240/640x480/1280x960, 32 samples on [0.5, 2.5], "
                      "stop at T < 1e-4, tiny field trained 300 steps, training 1 step / 5 ms")
    return st


def render_capacity(nsl, torch, dev, W, f, P, rcfg, reps=20):
    """Rays/s of nsl_render_batch alone: one 1280x960 request per launch
    (19 200 tiles), nothing else on the GPU."""
    from paper_2210_13641_amd import serve
    Wd, H = 1280, 960
    prep = nsl.prepare(f, P)
    pose = W.look_at_pose((1.5, 0.0, 0.0)).astype(np.float32).reshape(12)
    intr = np.array([0.9375 * Wd, 0.9375 * Wd, Wd / 2.0, H / 2.0], np.float32)
    out = [torch.empty(H * Wd, 3, device=dev)] + [torch.empty(H * Wd, device=dev) for _ in range(3)]
    rq = nsl.records_to_device([nsl.render_request(P, prep, pose, intr, H, Wd, *out)], nsl.RenderRequest, dev)
    n_tiles = -(-H * Wd // nsl.RENDER_TILE)
    tl = nsl.bytes_to_device(serve.tile_run(0, 0, n_tiles, H * Wd).tobytes(), dev)
    for _ in range(3):
        nsl.render_batch(f, rq, 1, tl, n_tiles, rcfg)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        nsl.render_batch(f, rq, 1, tl, n_tiles, rcfg)
    b.record()
    b.synchronize()
    return reps * H * Wd / (a.elapsed_time(b) * 1e-3)


def cpu_baseline_more(spec, sampler, kf, occ, table, ws):
    """The oracle with one BLAS thread on 1024 candidates of one paper-scale
    set, and the tiny workload's full step (32 768 samples) with all threads."""
    import workloads as W
    from oracle import step as ostep
    from threadpoolctl import threadpool_limits
    t64 = np.asarray(table, np.float32).astype(np.float64)
    w64 = [np.asarray(w, np.float32).astype(np.float64) for w in ws]
    out = {}
    ids = W.c2_candidates(N_CANDIDATES, seed=3)[:1024]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        r = ostep.train_step(spec, sampler, kf, t64, w64, ids, occupancy=occ)
        dt = time.perf_counter() - t0
    out["single_thread"] = dict(value=r["S"] / dt, unit="samples/s", cores=1, kind="oracle",
                                sample=f"one fwd+bwd step of the FP64 oracle on the first 1024 candidates of one "
                                       f"paper-scale set ({r['S']} samples), {dt:.1f} s wall")
    spec1 = W.C1_FIELD
    from oracle import field as ofield
    lay = ofield.param_layout(spec1)
    tab1, ws1 = W.init_params(0, lay["table_floats"], spec1.mlp_dims())
    tab1 = np.asarray(tab1, np.float32).astype(np.float64)
    ws1 = [np.asarray(w, np.float32).astype(np.float64) for w in ws1]
    kf1 = W.c1_keyframes()
    t0 = time.perf_counter()
    r = ostep.train_step(spec1, W.C1_SAMPLER, kf1, tab1, ws1, W.c1_pixels())
    dt = time.perf_counter() - t0
    out["tiny_workload"] = dict(value=r["S"] / dt, unit="samples/s", kind="oracle",
                                sample=f"one fwd+bwd step of the FP64 oracle on the tiny workload ({r['S']} samples), "
                                       f"{dt:.2f} s wall")
    return out


def cpu_baseline(spec, sampler, kf, occ, table, ws, n_cand, n_sets=2):
    """The FP64 oracle as it stands: one fwd+bwd step on the first n_cand
    candidates of each of n_sets candidate sets (FP32-rounded parameters)."""
    import workloads as W
    from oracle import step as ostep
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        threads = max((i.get("num_threads") or 1) for i in info) if info else 1
    except Exception:
        threads = os.cpu_count()
    t64 = np.asarray(table, np.float32).astype(np.float64)
    w64 = [np.asarray(w, np.float32).astype(np.float64) for w in ws]
    samples = rays = 0
    dt = 0.0
    for k in range(n_sets):
        ids = W.c2_candidates(N_CANDIDATES, seed=3 + k)[:n_cand]
        t0 = time.perf_counter()
        r = ostep.train_step(spec, sampler, kf, t64, w64, ids, occupancy=occ)
        dt += time.perf_counter() - t0
        samples += r["S"]
        rays += r["R"]
    return dict(value=samples / dt, unit="samples/s", cores=int(threads), kind="oracle",
                sample=f"one fwd+bwd step of the FP64 oracle on each of {n_sets} candidate sets (the first {n_cand} "
                       f"of {N_CANDIDATES} candidates each; {samples} samples, {rays} rays), {dt:.1f} s wall")


if __name__ == "__main__":
    sys.exit(main())
