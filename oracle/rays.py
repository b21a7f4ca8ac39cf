"""Camera rays, sample positions, samplers and the batch cut (test
infrastructure; see package doc).

Camera (Sec. 3.2: depth is the expected ray termination distance along each
pixel's ray; keyframe poses, images, depths and covariances arrive from
tracking, Sec. 3.3): pinhole, OpenCV axes, pose = camera-to-world [R | t].
For pixel (u, v):  d~ = ((u+1/2-c_x)/f_x, (v+1/2-c_y)/f_y, 1), s = |d~|,
origin o = t, unit direction d = R d~ / s.  The ray parameter is Euclidean
distance, so a z-depth D_z is D_z*s along the ray and a z-variance is
Sigma_z*s^2.

Sample positions decide integer quantities (occupancy cell, trilinear
cell, AABB membership, lattice range), so -- following the rule that such a
decision is taken in one precision on both sides -- they are formed in IEEE
single precision, every operation rounded separately, in this order:

    a  = ((f32(u) + 0.5) - c_x) / f_x          b = ((f32(v) + 0.5) - c_y) / f_y
    s  = sqrt((a*a + b*b) + 1)
    d_i = ((R_i0*a + R_i1*b) + R_i2) / s        o_i = t_i
    t  = t_near + (f32(i) + 0.5)*dt   (uniform)     t = (f32(k) + 0.5)*dt  (lattice)
    x_i = o_i + t*d_i
    inside  <=>  aabb_min_i <= x_i <= aabb_max_i  for every axis
    xn_i = clamp((x_i - aabb_min_i) * inv_ext_i, 0, 1),
           inv_ext_i = f32(1 / (aabb_max_i - aabb_min_i))  (FP64 quotient, rounded)
    cell_i = min(floor(xn_i * G), G - 1)

numpy float32 scalar/array operations round each operation to nearest-even,
which is exactly this definition.  Everything continuous downstream (SH of
the direction, depth scale s, the trilinear weights from xn) is FP64.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def split_pixel_ids(ids, H, W):
    ids = np.asarray(ids, np.int64)
    k = ids // (H * W)
    rem = ids % (H * W)
    return k, rem // W, rem % W


def rays_fp64(pose, intr, ids, H, W):
    """Continuous ray quantities in FP64: origin, unit direction, scale s."""
    k, v, u = split_pixel_ids(ids, H, W)
    P = np.asarray(pose, np.float64)[k]
    I = np.asarray(intr, np.float64)[k]
    a = (u + 0.5 - I[:, 2]) / I[:, 0]
    b = (v + 0.5 - I[:, 3]) / I[:, 1]
    dt = np.stack([a, b, np.ones_like(a)], -1)
    s = np.linalg.norm(dt, axis=-1)
    d = np.einsum("rij,rj->ri", P[:, :, :3], dt) / s[:, None]
    return P[:, :, 3].copy(), d, s


def rays_fp32(pose, intr, ids, H, W):
    """The single-precision ray of the position path (see module doc)."""
    k, v, u = split_pixel_ids(ids, H, W)
    P = np.asarray(pose, f32)[k]
    I = np.asarray(intr, f32)[k]
    half = f32(0.5)
    a = ((u.astype(f32) + half) - I[:, 2]) / I[:, 0]
    b = ((v.astype(f32) + half) - I[:, 3]) / I[:, 1]
    s = np.sqrt((a * a + b * b) + f32(1.0))
    d = np.empty((len(a), 3), f32)
    for i in range(3):
        d[:, i] = ((P[:, i, 0] * a + P[:, i, 1] * b) + P[:, i, 2]) / s
    o = P[:, :, 3].astype(f32)
    return o, d, s


def aabb_f32(spec):
    lo = np.asarray(spec.aabb_min, f32)
    hi = np.asarray(spec.aabb_max, f32)
    inv = (1.0 / (np.asarray(spec.aabb_max, np.float64) - np.asarray(spec.aabb_min, np.float64))).astype(f32)
    return lo, hi, inv


def positions_f32(o, d, t):
    """x = o + t*d per axis, product and sum rounded separately (FP32)."""
    return (o + (t[:, None] * d)).astype(f32)


def normalise_f32(x, lo, inv):
    xn = (x - lo) * inv
    return np.clip(xn, f32(0.0), f32(1.0)).astype(f32)


def inside_f32(x, lo, hi):
    return np.all((x >= lo) & (x <= hi), axis=-1)


def uniform_t(sampler):
    """Midpoint bins: t_i = t_n + (i+1/2)*dt, i < n_uniform (FP32)."""
    i = np.arange(sampler.n_uniform).astype(f32)
    return (f32(sampler.t_near) + (i + f32(0.5)) * f32(sampler.dt)).astype(f32)


def lattice_t(sampler):
    """Lattice t_k = (k+1/2)*dt anchored at the ray origin, restricted to
    t_near <= t_k <= t_far (FP32 comparisons)."""
    kmax = int(np.ceil(sampler.t_far / sampler.dt)) + 2
    k = np.arange(kmax).astype(f32)
    t = ((k + f32(0.5)) * f32(sampler.dt)).astype(f32)
    keep = (t >= f32(sampler.t_near)) & (t <= f32(sampler.t_far))
    return t[keep]


def occupancy_lookup(words, G, xn):
    cell = np.minimum(np.floor(xn * f32(G)), G - 1).astype(np.int64)
    bit = cell[:, 0] + G * (cell[:, 1] + G * cell[:, 2])
    w = np.asarray(words, np.uint32)
    return ((w[bit >> 5] >> (bit & 31).astype(np.uint32)) & 1).astype(bool)


def march(spec, sampler, o32, d32, words):
    """Samples of every ray.

    uniform:   all n_uniform midpoint samples.
    occupancy: lattice points inside the closed AABB whose occupancy cell bit
               is set, in order, at most max_per_ray of them.
    Returns (counts [R], list of FP32 t arrays).  delta = dt for every sample.
    """
    lo, hi, inv = aabb_f32(spec)
    R = len(o32)
    if sampler.mode == "uniform":
        t = uniform_t(sampler)
        return np.full(R, len(t), np.int64), [t.copy() for _ in range(R)]
    tl = lattice_t(sampler)
    counts = np.zeros(R, np.int64)
    ts = []
    for r in range(R):
        x = (o32[r][None, :] + tl[:, None] * d32[r][None, :]).astype(f32)
        ok = inside_f32(x, lo, hi)
        xn = normalise_f32(x[ok], lo, inv)
        occ = occupancy_lookup(words, sampler.grid_res, xn)
        tk = tl[ok][occ][:sampler.max_per_ray]
        counts[r] = len(tk)
        ts.append(tk)
    return counts, ts


def batch_cut(counts, max_samples):
    """Keep candidate r iff its inclusive sample prefix fits max_samples.
    Returns (kept mask over candidates, ray mask = kept & count > 0)."""
    incl = np.cumsum(counts)
    kept = incl <= max_samples
    return kept, kept & (counts > 0)
