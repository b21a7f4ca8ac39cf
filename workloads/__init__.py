"""Seeded synthetic inputs for the NeRF-SLAM mapping step.

This module is shared by the FP64 oracle (tests) and by the GPU path
(tests, bench, smoke).  It holds configuration numbers, camera placement,
synthetic scenes, targets and random initial parameters -- and none of the
method's arithmetic: no encoding, no network, no compositing, no loss.  The
only geometry here is scene synthesis (ray/sphere intersection for the
synthetic depth maps), written independently of both implementations.

All randomness comes from ``numpy.random.Generator(PCG64(seed))`` with the
draw order documented per function, so every consumer sees identical arrays.

The workloads stand in for the paper's datasets (Replica, Cube-Diorama;
Sec. 4), which are not available: they keep the paper's shapes -- 640x480
keyframes (Sec. 4.5), a window of 8 keyframes (Sec. 3.3), dense noisy depth
with outliers and per-pixel variances up to about 1 m^2 (Sec. 3.2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

# ----------------------------------------------------------------------------
# Configuration records (plain numbers only)
# ----------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class FieldSpec:
    """Hash-grid radiance field shape (the paper defers it to Instant-NGP,
    Sec. 3.2 and Sec. 3.4)."""
    levels: int
    log2_table: int
    base_res: int
    per_level_scale: Optional[float]   # growth factor b; None -> from max_res
    max_res: Optional[int]
    density_hidden: int
    colour_hidden: tuple               # hidden widths of the colour net
    sh_bands: int                      # 3 -> 9 coefficients, 4 -> 16
    aabb_min: tuple = (-1.0, -1.0, -1.0)
    aabb_max: tuple = (1.0, 1.0, 1.0)
    feat_per_level: int = 2
    geo_dim: int = 16

    @property
    def enc_dim(self) -> int:
        return self.levels * self.feat_per_level

    @property
    def colour_in(self) -> int:
        return self.geo_dim + self.sh_bands * self.sh_bands

    def mlp_dims(self) -> list:
        """[(fan_in, fan_out)] for every weight matrix, density net first."""
        dims = [(self.enc_dim, self.density_hidden),
                (self.density_hidden, self.geo_dim)]
        prev = self.colour_in
        for h in self.colour_hidden:
            dims.append((prev, h))
            prev = h
        dims.append((prev, 3))
        return dims


@dataclasses.dataclass(frozen=True)
class SamplerSpec:
    mode: str            # "uniform" or "occupancy"
    t_near: float
    t_far: float
    dt: float            # bin width (uniform) or lattice step (occupancy)
    n_uniform: int = 0   # samples per ray for "uniform"
    max_per_ray: int = 256
    max_samples: int = 1 << 18
    grid_res: int = 128


# C1: the tiny plain step.
C1_FIELD = FieldSpec(levels=4, log2_table=12, base_res=4, per_level_scale=2.0,
                     max_res=None, density_hidden=32, colour_hidden=(32,),
                     sh_bands=3, aabb_min=(-2.0, -2.0, -2.0),
                     aabb_max=(2.0, 2.0, 2.0))
C1_SAMPLER = SamplerSpec(mode="uniform", t_near=1.0, t_far=3.0, dt=1.0 / 16.0,
                         n_uniform=32, max_per_ray=32, max_samples=1 << 20)

# C2: the paper-scale step.
C2_FIELD = FieldSpec(levels=16, log2_table=19, base_res=16,
                     per_level_scale=None, max_res=2048, density_hidden=64,
                     colour_hidden=(64, 64), sh_bands=4)
C2_SAMPLER = SamplerSpec(mode="occupancy", t_near=0.05, t_far=4.0,
                         dt=1.0 / 128.0, max_per_ray=256,
                         max_samples=1 << 18, grid_res=128)

# Adam hyper-parameters of the differentiation workload; eps follows the
# hash-grid prior work (the paper gives none).
ADAM_LR = 1e-2
ADAM_BETAS = (0.9, 0.99)
ADAM_EPS = 1e-15
LAMBDA_D = 1.0   # Sec. 3.2, Eq. 3


# ----------------------------------------------------------------------------
# Cameras (scene synthesis): OpenCV axes, camera-to-world [R | t]
# ----------------------------------------------------------------------------

def look_at_pose(position, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)):
    """3x4 camera-to-world matrix looking from ``position`` at ``target``.

    Columns of R are the camera x (right), y (down) and z (forward) axes in
    world coordinates: z = normalize(target - position),
    x = normalize(z x up), y = z x x.
    """
    p = np.asarray(position, np.float64)
    f = np.asarray(target, np.float64) - p
    f /= np.linalg.norm(f)
    x = np.cross(f, np.asarray(up, np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    pose = np.zeros((3, 4), np.float64)
    pose[:, 0], pose[:, 1], pose[:, 2], pose[:, 3] = x, y, f, p
    return pose


def ring_poses(angles, radius, z=0.0):
    return np.stack([look_at_pose((radius * math.cos(a), radius * math.sin(a), z))
                     for a in angles])


def pixel_directions_world(pose, intr, H, W, stride=1.0):
    """World-space unit directions and z-scale of pixel centres (scene
    synthesis only: the targets are made with this, the method never is)."""
    fx, fy, cx, cy = intr
    u = (np.arange(W) + 0.5) * stride
    v = (np.arange(H) + 0.5) * stride
    uu, vv = np.meshgrid(u, v)
    cam = np.stack([(uu - cx) / fx, (vv - cy) / fy, np.ones_like(uu)], -1)
    norm = np.linalg.norm(cam, axis=-1)
    world = cam @ pose[:, :3].T
    return world / norm[..., None], norm


def pack_pixel_id(k, v, u, H, W):
    """Pixel id layout used at the boundary: k*H*W + v*W + u."""
    return (np.asarray(k, np.int64) * H * W + np.asarray(v, np.int64) * W
            + np.asarray(u, np.int64)).astype(np.uint32)


# ----------------------------------------------------------------------------
# Scenes
# ----------------------------------------------------------------------------

def sphere_hit(origins, dirs, radius=0.5, centre=(0.0, 0.0, 0.0)):
    """Entry distance of unit-direction rays into a sphere; inf on a miss."""
    oc = origins - np.asarray(centre)
    b = np.sum(oc * dirs, -1)
    c = np.sum(oc * oc, -1) - radius * radius
    disc = b * b - c
    t = -b - np.sqrt(np.maximum(disc, 0.0))
    return np.where(disc >= 0.0, t, np.inf)


@dataclasses.dataclass(frozen=True)
class BlobScene:
    centres: np.ndarray   # [n,3]
    scales: np.ndarray    # [n]
    amps: np.ndarray      # [n]
    rho_max: float = 100.0

    def density(self, x):
        x = np.asarray(x, np.float64)
        out = np.zeros(x.shape[:-1])
        for c, s, a in zip(self.centres, self.scales, self.amps):
            d2 = np.sum((x - c) ** 2, -1)
            out += a * np.exp(-d2 / (2.0 * s * s))
        return np.minimum(out, self.rho_max)

    def surface_radii(self, level=1.0):
        """Radius where one blob alone reaches ``level``."""
        return self.scales * np.sqrt(2.0 * np.log(self.amps / level))


def blob_scene(seed=0, n=64):
    """64 Gaussian density blobs: centres U[-0.8,0.8]^3, s U(0.02,0.10),
    a U(10,100); draw order centres, scales, amplitudes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(-0.8, 0.8, size=(n, 3))
    scales = rng.uniform(0.02, 0.10, size=n)
    amps = rng.uniform(10.0, 100.0, size=n)
    return BlobScene(centres, scales, amps)


def occupancy_bits(density_fn, res, aabb_min, aabb_max, threshold=1.0):
    """Bitfield of cells whose centre density exceeds ``threshold``.

    Layout: res^3 bits, cell (x,y,z) -> bit x + res*(y + res*z), packed into
    uint32 words least-significant bit first.
    """
    lo = np.asarray(aabb_min, np.float64)
    hi = np.asarray(aabb_max, np.float64)
    idx = (np.arange(res) + 0.5) / res
    occ = np.zeros(res ** 3, bool)
    zs = lo[2] + idx * (hi[2] - lo[2])
    ys = lo[1] + idx * (hi[1] - lo[1])
    xs = lo[0] + idx * (hi[0] - lo[0])
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    for z in range(res):
        pts = np.stack([xx, yy, np.full_like(xx, zs[z])], -1)
        occ[z * res * res:(z + 1) * res * res] = (density_fn(pts) > threshold).ravel()
    return pack_bits(occ)


def pack_bits(occ):
    occ = np.asarray(occ, bool).ravel()
    words = np.zeros((occ.size + 31) // 32, np.uint32)
    nz = np.nonzero(occ)[0]
    np.bitwise_or.at(words, nz >> 5, (np.uint32(1) << (nz & 31).astype(np.uint32)))
    return words


def unpack_bits(words, n):
    words = np.asarray(words, np.uint32)
    i = np.arange(n)
    return ((words[i >> 5] >> (i & 31).astype(np.uint32)) & 1).astype(bool)


# ----------------------------------------------------------------------------
# Parameters
# ----------------------------------------------------------------------------

def init_params(seed, n_table_floats, mlp_dims, table_range=1e-4):
    """Random initial field parameters.

    Draw order: the hash tables (``n_table_floats`` values, U(-r, r)), then
    each weight matrix [fan_in, fan_out] in network order, Glorot-uniform
    U(-a, a) with a = sqrt(6/(fan_in+fan_out)).  Returns (table, [W...]) in
    FP64; consumers round to their storage precision.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    table = rng.uniform(-table_range, table_range, size=n_table_floats)
    ws = []
    for fi, fo in mlp_dims:
        a = math.sqrt(6.0 / (fi + fo))
        ws.append(rng.uniform(-a, a, size=(fi, fo)))
    return table, ws


# ----------------------------------------------------------------------------
# Keyframe workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Keyframes:
    rgb: np.ndarray        # [K,H,W,3] float32 in [0,1]
    pose: np.ndarray       # [K,3,4]  float32 camera-to-world
    intr: np.ndarray       # [K,4]    float32 fx, fy, cx, cy
    depth: np.ndarray      # [K,H,W]  float32 z-depth D
    depth_var: np.ndarray  # [K,H,W]  float32 Sigma_D (variance, m^2; inf = none)

    @property
    def shape(self):
        return self.rgb.shape[:3]


def sphere_keyframes(seed, poses, H, W, f, t_far, sigma_range=(0.01, 0.5),
                     radius=0.5):
    """Keyframes of the analytic sphere scene (radius 0.5 at the origin).

    Per keyframe, draw order: RGB U(0,1) [H,W,3]; sigma = exp U(ln lo, ln hi)
    [H,W]; unit normal noise [H,W].  Depth = sphere entry z-depth + sigma*n;
    pixels that miss get Sigma_D = inf and the far-plane z-depth.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    K = len(poses)
    intr = np.array([f, f, W / 2.0, H / 2.0])
    rgb = np.empty((K, H, W, 3))
    depth = np.empty((K, H, W))
    var = np.empty((K, H, W))
    for k in range(K):
        rgb[k] = rng.uniform(0.0, 1.0, size=(H, W, 3))
        sig = np.exp(rng.uniform(math.log(sigma_range[0]), math.log(sigma_range[1]),
                                 size=(H, W)))
        noise = rng.standard_normal(size=(H, W))
        dirs, norm = pixel_directions_world(poses[k], intr, H, W)
        t = sphere_hit(np.broadcast_to(poses[k][:, 3], dirs.shape), dirs, radius)
        hit = np.isfinite(t)
        depth[k] = np.where(hit, t / norm + sig * noise, t_far / norm)
        var[k] = np.where(hit, sig * sig, np.inf)
    return Keyframes(rgb.astype(np.float32), np.asarray(poses, np.float32),
                     np.tile(intr, (K, 1)).astype(np.float32),
                     depth.astype(np.float32), var.astype(np.float32))


def blob_keyframes(seed, scene: BlobScene, poses, H=480, W=640, f=600.0,
                   lowres=(60, 80), sigma_range=(0.005, 1.0), outlier_frac=0.05,
                   background=4.0):
    """Keyframes of the blob scene, shaped like SLAM output.

    Depth is the entry z-depth of the union of the blobs' unit-density
    spheres, computed at ``lowres`` and bilinearly upsampled (dense SLAM works
    at reduced resolution), then corrupted.  Per keyframe, draw order: RGB
    U(0,1) [H,W,3]; sigma log-uniform [H,W]; unit normal noise [H,W];
    outlier mask U(0,1) [H,W]; outlier depth U(0.5,3.0) [H,W].  Outliers and
    background pixels get sigma = 1.0 m.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    K = len(poses)
    intr = np.array([f, f, W / 2.0, H / 2.0])
    rgb = np.empty((K, H, W, 3))
    depth = np.empty((K, H, W))
    var = np.empty((K, H, W))
    radii = scene.surface_radii(1.0)
    lh, lw = lowres
    stride = H / lh
    for k in range(K):
        rgb[k] = rng.uniform(0.0, 1.0, size=(H, W, 3))
        sig = np.exp(rng.uniform(math.log(sigma_range[0]), math.log(sigma_range[1]),
                                 size=(H, W)))
        noise = rng.standard_normal(size=(H, W))
        outl = rng.uniform(size=(H, W)) < outlier_frac
        outd = rng.uniform(0.5, 3.0, size=(H, W))
        dirs, norm = pixel_directions_world(poses[k], intr, lh, lw, stride=stride)
        o = np.broadcast_to(poses[k][:, 3], dirs.shape)
        t = np.full(dirs.shape[:2], np.inf)
        for c, r in zip(scene.centres, radii):
            t = np.minimum(t, sphere_hit(o, dirs, r, c))
        low = np.where(np.isfinite(t), t / norm, background)
        up = _bilinear_upsample(low, H, W)
        bg = _bilinear_upsample(np.isfinite(t).astype(np.float64), H, W) < 0.5
        d = up + sig * noise
        s = np.where(bg, 1.0, sig)
        d = np.where(outl, outd, d)
        s = np.where(outl, 1.0, s)
        depth[k], var[k] = d, s * s
    return Keyframes(rgb.astype(np.float32), np.asarray(poses, np.float32),
                     np.tile(intr, (K, 1)).astype(np.float32),
                     depth.astype(np.float32), var.astype(np.float32))


def _bilinear_upsample(img, H, W):
    h, w = img.shape
    ys = np.clip((np.arange(H) + 0.5) * h / H - 0.5, 0, h - 1)
    xs = np.clip((np.arange(W) + 0.5) * w / W - 0.5, 0, w - 1)
    y0 = np.floor(ys).astype(int)
    x0 = np.floor(xs).astype(int)
    y1 = np.minimum(y0 + 1, h - 1)
    x1 = np.minimum(x0 + 1, w - 1)
    fy = (ys - y0)[:, None]
    fx = (xs - x0)[None, :]
    a = img[y0][:, x0] * (1 - fx) + img[y0][:, x1] * fx
    b = img[y1][:, x0] * (1 - fx) + img[y1][:, x1] * fx
    return a * (1 - fy) + b * fy


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def c1_keyframes(seed=0, H=32, W=32, f=32.0):
    """Tiny step: one 32x32 camera at (0,0,-2) looking along +z (R = I)."""
    pose = np.zeros((1, 3, 4))
    pose[0, :, :3] = np.eye(3)
    pose[0, :, 3] = (0.0, 0.0, -2.0)
    return sphere_keyframes(seed, pose, H, W, f, C1_SAMPLER.t_far)


def c1_pixels(H=32, W=32, K=1):
    """All pixels of every keyframe, keyframe-major, row-major."""
    return np.arange(K * H * W, dtype=np.uint32)


def c4_keyframes(n_cams, seed=0, H=32, W=32, f=32.0, radius=2.0):
    """Mixed-precision batches: n_cams 32x32 cameras at distance 2 on the
    ring, angle 2*pi*k/n_cams, looking at the origin."""
    poses = ring_poses([2.0 * math.pi * k / n_cams for k in range(n_cams)], radius)
    return sphere_keyframes(seed, poses, H, W, f, C1_SAMPLER.t_far)


def c2_scene(seed=0):
    return blob_scene(seed)


def c2_occupancy(scene: BlobScene, res=128):
    return occupancy_bits(scene.density, res, C2_FIELD.aabb_min, C2_FIELD.aabb_max)


def c2_keyframes(scene: BlobScene, seed=1, K=8, H=480, W=640, f=600.0, radius=1.5):
    """8 keyframes at 640x480 on a ring of radius 1.5, angles U(0, 2 pi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    angles = rng.uniform(0.0, 2.0 * math.pi, size=K)
    poses = ring_poses(angles, radius)
    return blob_keyframes(seed + 1, scene, poses, H, W, f)


def c2_candidates(n, seed=3, K=8, H=480, W=640):
    """Pixel candidates drawn uniformly over all keyframes (PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, K * H * W, size=n, dtype=np.int64).astype(np.uint32)


def random_rays_subset(n, total, seed=5):
    """``n`` distinct pixel ids out of ``total`` (sorted)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(total, size=n, replace=False)).astype(np.uint32)


SERVE_SIZES = ((160, 120), (320, 240), (640, 480), (1280, 960))


def serve_requests(n, seed=7, rate=200.0, radius=1.5):
    """Render requests: Poisson arrivals (rate per second), image size drawn
    uniformly from SERVE_SIZES, f = 0.9375 W, pose on the ring.
    Draw order: inter-arrival gaps [n], size indices [n], ring angles [n]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=n)
    sizes = rng.integers(0, len(SERVE_SIZES), size=n)
    angles = rng.uniform(0.0, 2.0 * math.pi, size=n)
    out = []
    t = 0.0
    for i in range(n):
        t += gaps[i]
        W, H = SERVE_SIZES[sizes[i]]
        pose = look_at_pose((radius * math.cos(angles[i]), radius * math.sin(angles[i]), 0.0))
        intr = np.array([0.9375 * W, 0.9375 * W, W / 2.0, H / 2.0], np.float32)
        out.append(dict(arrival=t, H=H, W=W, pose=pose.astype(np.float32), intr=intr))
    return out


# ----------------------------------------------------------------------------
# Tracking Hessian of a keyframe window (input of the covariance recovery)
# ----------------------------------------------------------------------------

def ba_window(seed=0, n_kf=8, h=30, w=40, obs_per_pixel=2, gauge=1e4, pose_dim=6):
    """A synthetic dense-BA linear system of a keyframe window with the
    arrow structure of Sec. 3.1 / Eq. 1: per-pixel inverse depths (diagonal
    block P), camera poses (block C), and their coupling E.

    Every pixel of keyframe i is observed in ``obs_per_pixel`` other
    keyframes k; an observation contributes J^T W J with a 2-row Jacobian
    [J_i (2 x 6) | J_k (2 x 6) | J_d (2 x 1)] and weights W = diag(w1, w2),
    w ~ U(0.1, 1) (the flow confidences).  A prior of ``gauge`` on the first
    pose fixes the gauge.  Draw order per keyframe i: inverse depths
    U(0.2, 2) [h*w]; then per observation slot: target offsets, J_i, J_k,
    J_d, w.  Returns (C [c,c], E [c,p], P [p], inv_depth [p]) in FP64 with
    c = 6 n_kf, p = n_kf h w; pixel j of keyframe i is column i*h*w + j.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    c = pose_dim * n_kf
    npx = h * w
    p = n_kf * npx
    C = np.zeros((c, c))
    E = np.zeros((c, p))
    P = np.zeros(p)
    inv_depth = np.empty(p)
    for i in range(n_kf):
        inv_depth[i * npx:(i + 1) * npx] = rng.uniform(0.2, 2.0, npx)
        for _ in range(obs_per_pixel):
            off = rng.integers(1, n_kf, size=npx)
            k = (i + off) % n_kf
            Ji = rng.normal(size=(npx, 2, pose_dim))
            Jk = rng.normal(size=(npx, 2, pose_dim))
            Jd = rng.normal(size=(npx, 2)) * 3.0
            wt = rng.uniform(0.1, 1.0, size=(npx, 2))
            cols = i * npx + np.arange(npx)
            P[cols] += np.sum(wt * Jd * Jd, axis=1)
            si = slice(pose_dim * i, pose_dim * (i + 1))
            C[si, si] += np.einsum("nra,nr,nrb->ab", Ji, wt, Ji)
            E[si, cols] += np.einsum("nra,nr,nr->an", Ji, wt, Jd)
            for kk in range(n_kf):
                sel = k == kk
                if not sel.any():
                    continue
                sk = slice(pose_dim * kk, pose_dim * (kk + 1))
                C[sk, sk] += np.einsum("nra,nr,nrb->ab", Jk[sel], wt[sel], Jk[sel])
                cross = np.einsum("nra,nr,nrb->ab", Ji[sel], wt[sel], Jk[sel])
                C[si, sk] += cross
                C[sk, si] += cross.T
                E[sk, cols[sel]] += np.einsum("nra,nr,nr->an", Jk[sel], wt[sel], Jd[sel])
    C[:pose_dim, :pose_dim] += gauge * np.eye(pose_dim)
    return C, E, P, inv_depth
