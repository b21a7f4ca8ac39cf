"""Shared set-up of GPU parity tests: the same seeded inputs for the HIP
path (through the C ABI) and the oracle, and the magnitude-based bound."""
from __future__ import annotations

import functools
import sys

import numpy as np

import workloads as W


def report(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check_mag(name, gpu, orc, mag, tol, floor=1e-6):
    """|gpu - orc| <= tol * max(mag, floor * max(mag)) element-wise."""
    gpu = np.asarray(gpu, np.float64).ravel()
    orc = np.asarray(orc, np.float64).ravel()
    mag = np.abs(np.asarray(mag, np.float64).ravel())
    assert gpu.shape == orc.shape == mag.shape, (name, gpu.shape, orc.shape, mag.shape)
    assert np.all(np.isfinite(gpu)), f"{name}: non-finite GPU values"
    top = mag.max() if mag.size else 0.0
    bound = tol * np.maximum(mag, floor * top)
    err = np.abs(gpu - orc)
    bad = err > bound
    rel = np.linalg.norm(gpu - orc) / max(np.linalg.norm(orc), 1e-300)
    if bad.any():
        i = int(np.argmax(err / np.maximum(bound, 1e-300)))
        raise AssertionError(
            f"{name}: {int(bad.sum())}/{bad.size} elements exceed tol {tol}; worst at {i}: "
            f"gpu {gpu[i]!r} oracle {orc[i]!r} magnitude {mag[i]!r} bound {bound[i]!r}; rel L2 {rel:.3e}")
    return rel


def params_for(spec, layout, seed=0, table_range=1e-4):
    """(flat FP32 parameter vector in the library layout, oracle table,
    oracle weights) -- the oracle gets the FP32-rounded values."""
    table, ws = W.init_params(seed, layout["table_floats"], spec.mlp_dims(), table_range)
    flat = np.zeros(layout["total"], np.float32)
    flat[:len(table)] = table
    for off, w in zip(layout["w_offsets"], ws):
        flat[off:off + w.size] = w.ravel()
    t64 = flat[:len(table)].astype(np.float64)
    w64 = [flat[o:o + w.size].astype(np.float64).reshape(w.shape) for o, w in zip(layout["w_offsets"], ws)]
    return flat, t64, w64


def split_grads(flat, layout, spec):
    g = np.asarray(flat, np.float64)
    tab = g[:layout["table_floats"]]
    ws = [g[o:o + a * b].reshape(a, b) for o, (a, b) in zip(layout["w_offsets"], spec.mlp_dims())]
    return tab, ws


@functools.lru_cache(maxsize=None)
def c2_inputs():
    scene = W.c2_scene()
    occ = W.c2_occupancy(scene)
    kf = W.c2_keyframes(scene)
    return scene, occ, kf


def upload_keyframes(nsl, torch, kf, dev, grid_res=1, occ=None):
    K, H, Wd = kf.rgb.shape[:3]
    m = nsl.Mapper(K, H, Wd, grid_res, device=dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    m.upsert(list(range(K)), t(kf.rgb), t(kf.pose.reshape(K, 12)), t(kf.intr), t(kf.depth), t(kf.depth_var))
    if occ is not None:
        m.set_occupancy(t(occ.view(np.int32)))
    return m
