"""Pins of the FP64 oracle against things other than itself: closed forms
(tests/golden/closed_forms.json, written with ``decimal``), invariants,
library routines, brute force and finite differences.  CPU only."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import field, rays, render, step

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


# ----------------------------------------------------------------------------
# Compositing: Eq. 5 and 6 against closed forms (P1, P2, P3) and invariants (P4)
# ----------------------------------------------------------------------------

def _uniform_ray(sigma, t0, dt, n):
    t = t0 + (np.arange(n) + 0.5) * dt
    return np.full(n, sigma), t, np.full(n, dt)


def test_homogeneous_transmittance_depth_variance():
    g = GOLD["homogeneous"]
    sig, t, dl = _uniform_ray(1.0, 1.0, 0.0625, 32)
    fw = render.composite_ray(sig, np.full((32, 3), 0.5), t, dl)
    assert fw["T"][-1] == pytest.approx(float(g["T_end"]), rel=1e-13)
    assert fw["T"][-1] == pytest.approx(math.exp(-1.0 * 2.0), rel=1e-13)   # exp(-sigma L)
    assert fw["A"] == pytest.approx(float(g["opacity"]), rel=1e-13)
    assert fw["D"] == pytest.approx(float(g["depth"]), rel=1e-13)
    assert fw["V"] == pytest.approx(float(g["var"]), rel=1e-12)
    # continuum limit of the expected depth, error O(sigma dt^2)
    L = 2.0
    cont = 1.0 * (1 - math.exp(-L)) + (1 - math.exp(-L)) - L * math.exp(-L)
    assert abs(fw["D"] - cont) < 1e-3


def test_slab_from_sphere_centre_pixel():
    """The tiny workload's centre pixel through the analytic sphere."""
    g = GOLD["slab"]
    kf = W.c1_keyframes()
    o32, d32, _ = rays.rays_fp32(kf.pose, kf.intr, np.array([16 * 32 + 16]), 32, 32)
    t = rays.uniform_t(W.C1_SAMPLER)
    x = rays.positions_f32(o32[[0] * len(t)], d32[[0] * len(t)], t).astype(np.float64)
    inside = np.linalg.norm(x, axis=-1) < 0.5
    assert np.nonzero(inside)[0].tolist() == list(range(8, 24))
    sig = np.where(inside, 50.0, 0.0)
    fw = render.composite_ray(sig, np.zeros((32, 3)), t, np.full(32, 0.0625))
    assert fw["D"] == pytest.approx(float(g["depth"]), rel=1e-13)
    assert fw["V"] == pytest.approx(float(g["var"]), rel=1e-9)
    assert fw["A"] == pytest.approx(float(g["opacity"]), rel=1e-15)
    assert fw["T"][-1] == pytest.approx(float(g["T_end"]), rel=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_composite_invariants(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    sig = rng.exponential(3.0, n) * (rng.uniform(size=n) < 0.7)
    t = np.sort(rng.uniform(0.5, 3.0, n))
    dl = rng.uniform(0.01, 0.1, n)
    c = rng.uniform(size=(n, 3))
    fw = render.composite_ray(sig, c, t, dl)
    assert np.all(fw["w"] >= 0)
    assert fw["A"] + fw["T"][-1] == pytest.approx(1.0, abs=1e-14)      # telescoping
    M2 = (fw["w"] * t * t).sum()
    assert fw["V"] == pytest.approx(M2 - fw["D"] ** 2 * (2 - fw["A"]), abs=1e-12)
    z = render.composite_ray(np.zeros(n), c, t, dl)
    assert z["A"] == 0 and z["D"] == 0 and np.all(z["C"] == 0) and z["V"] == 0


def test_single_opaque_sample():
    n, k = 10, 4
    sig = np.zeros(n)
    sig[k] = 1e4
    t = np.linspace(1, 2, n)
    c = np.random.default_rng(0).uniform(size=(n, 3))
    fw = render.composite_ray(sig, c, t, np.full(n, 0.1))
    assert fw["D"] == pytest.approx(t[k], rel=1e-12)
    assert np.allclose(fw["C"], c[k], rtol=1e-12)
    assert fw["V"] == pytest.approx(0.0, abs=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 17])
def test_composite_adjoint_by_finite_differences(n):
    """Suffix-sum adjoint formulas against central differences in sigma and c."""
    rng = np.random.default_rng(n)
    sig = rng.uniform(0.1, 5.0, n)
    t = np.sort(rng.uniform(1, 3, n))
    dl = rng.uniform(0.05, 0.2, n)
    c = rng.uniform(size=(n, 3))
    gC, gD, gV, gA = rng.normal(size=3), rng.normal(), rng.normal(), rng.normal()

    def f(s, cc):
        fw = render.composite_ray(s, cc, t, dl)
        return fw["C"] @ gC + gD * fw["D"] + gV * fw["V"] + gA * fw["A"]

    fw = render.composite_ray(sig, c, t, dl)
    ds, dc, _, _ = render.composite_ray_bwd(fw, c, t, dl, gC, gD, gV, gA=gA)
    h = 1e-6
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        fd = (f(sig + e, c) - f(sig - e, c)) / (2 * h)
        assert ds[k] == pytest.approx(fd, rel=1e-6, abs=1e-9)
        for ch in range(3):
            cc = c.copy()
            cc[k, ch] += h
            cm = c.copy()
            cm[k, ch] -= h
            assert dc[k, ch] == pytest.approx((f(sig, cc) - f(sig, cm)) / (2 * h), rel=1e-6, abs=1e-9)
    assert np.allclose(dc, fw["w"][:, None] * gC[None, :])             # dI*/dc_k = w_k


def test_early_termination_keeps_prefix():
    sig = np.full(32, 3.0)
    t = 1 + (np.arange(32) + 0.5) / 16
    fw = render.composite_ray(sig, np.ones((32, 3)), t, np.full(32, 1 / 16), stop_T=1e-2)
    T = np.exp(-np.concatenate([[0], np.cumsum(sig / 16)]))
    assert fw["n_used"] == int(np.argmax(T[:32] < 1e-2))
    assert np.all(fw["w"][fw["n_used"]:] == 0)


# ----------------------------------------------------------------------------
# Loss (Eq. 3, 4, 7) (P10)
# ----------------------------------------------------------------------------

def test_loss_reduces_to_photometric_and_is_unit_invariant():
    rng = np.random.default_rng(1)
    R = 50
    C, I = rng.uniform(size=(R, 3)), rng.uniform(size=(R, 3))
    D, Dt = rng.uniform(1, 2, R), rng.uniform(1, 2, R)
    sd = rng.uniform(0.01, 0.5, R)
    l_rgb, l_d, *_ = render.loss_seeds(C, D, I, Dt, 1 / sd ** 2, R, 1.0)
    l0_rgb, l0_d, *_ = render.loss_seeds(C, D, I, Dt, np.zeros(R), R, 1.0)
    assert np.all(l0_d == 0) and np.allclose(l0_rgb, ((C - I) ** 2).sum(-1))
    s = 3.7                                   # scale depths and std together
    _, l_d2, *_ = render.loss_seeds(C, D * s, I, Dt * s, 1 / (sd * s) ** 2, R, 1.0)
    assert np.allclose(l_d, l_d2, rtol=1e-13)
    _, l_raw, *_ = render.loss_seeds(C, D, I, Dt, np.ones(R), R, 1.0)   # Sigma_D = 1
    assert np.allclose(l_raw, (D - Dt) ** 2)


def test_precision_masks_unusable_measurements():
    D = np.array([1.0, np.nan, 1.0, 1.0, 1.0, np.inf])
    V = np.array([0.04, 0.04, 0.0, -1.0, np.inf, 0.04])
    pi, ok = render.precision_from_variance(D, V, np.ones(6))
    assert pi.tolist() == [25.0, 0, 0, 0, 0, 0] and ok.tolist() == [True] + [False] * 5


# ----------------------------------------------------------------------------
# Encoding (P5, P6, P7) and layout
# ----------------------------------------------------------------------------

def test_level_layout_of_both_fields():
    assert field.level_resolutions(W.C1_FIELD) == [4, 8, 16, 32]
    assert field.level_layout(W.C1_FIELD)[2] == [125, 729, 4096, 4096]
    res = field.level_resolutions(W.C2_FIELD)
    assert res == [16, 22, 30, 42, 58, 80, 111, 153, 212, 294, 406, 561, 776, 1072, 1482, 2048]
    _, dense, sizes, _ = field.level_layout(W.C2_FIELD)
    assert dense == [True] * 5 + [False] * 11
    assert sum(sizes) == 6098925
    # b^l must not sit on an integer, or FP64 rounding could move a floor
    b = 2048 ** (1 / 15) / 16 ** (1 / 15)
    assert min(abs(16 * b ** l - round(16 * b ** l)) for l in range(1, 15)) > 1e-3


def test_hash_matches_integer_arithmetic():
    T = 1 << 19
    v = np.array([[1, 2, 3], [2047, 0, 5], [123456, 654321, 7]])
    got = field.corner_index(v, 2048, False, T)
    want = [((a * 1) ^ (b * 2654435761) ^ (c * 805459861)) % (1 << 32) % T for a, b, c in v.tolist()]
    assert got.tolist() == want


def test_dense_index_is_bijection():
    n = 8
    g = np.stack(np.meshgrid(*[np.arange(n + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    idx = field.corner_index(g, n, True, 1 << 12)
    assert sorted(idx.tolist()) == list(range((n + 1) ** 3))


def test_trilinear_partition_of_unity_and_constant_table():
    spec = W.C1_FIELD
    xn = np.random.default_rng(0).uniform(size=(500, 3)).astype(np.float32)
    corners = field.encode_corners(spec, xn)
    for idx, w in corners:
        assert np.allclose(w.sum(0), 1.0, atol=1e-15)
        assert np.all(w >= -1e-15)
    lay = field.param_layout(spec)
    tab = np.tile([0.25, -0.5], lay["table_floats"] // 2)
    e, _, _ = field.encode_fwd(spec, tab, xn, corners)
    assert np.allclose(e[:, 0::2], 0.25, atol=1e-15) and np.allclose(e[:, 1::2], -0.5, atol=1e-15)


def test_vertex_lookup_returns_stored_feature():
    spec = W.C1_FIELD
    res, dense, sizes, offs = field.level_layout(spec)
    lay = field.param_layout(spec)
    tab = np.random.default_rng(2).normal(size=lay["table_floats"])
    rng = np.random.default_rng(3)
    for l, n in enumerate(res):
        k = rng.integers(0, n + 1, size=(64, 3))
        xn = (k / n).astype(np.float32)              # exact: n is a power of 2
        e, _, _ = field.encode_fwd(spec, tab, xn)
        idx = offs[l] + field.corner_index(k, n, dense[l], 1 << spec.log2_table)
        want = tab.reshape(-1, 2)[idx]
        assert np.array_equal(e[:, 2 * l:2 * l + 2], want)


def test_encoding_is_linear_in_table():
    spec = W.C1_FIELD
    lay = field.param_layout(spec)
    rng = np.random.default_rng(4)
    xn = rng.uniform(size=(100, 3)).astype(np.float32)
    a, b = rng.normal(size=lay["table_floats"]), rng.normal(size=lay["table_floats"])
    ea, _, c = field.encode_fwd(spec, a, xn)
    eb, _, _ = field.encode_fwd(spec, b, xn, c)
    eab, _, _ = field.encode_fwd(spec, 2 * a - 3 * b, xn, c)
    assert np.allclose(eab, 2 * ea - 3 * eb, atol=1e-12)
    # the adjoint of the encoding is its transpose: <de, E theta> = <E^T de, theta>
    de = rng.normal(size=ea.shape)
    g, _ = field.encode_bwd(spec, c, de, np.abs(de), lay["table_floats"])
    assert (de * ea).sum() == pytest.approx(g @ a, rel=1e-12)


# ----------------------------------------------------------------------------
# SH (P8)
# ----------------------------------------------------------------------------

def test_sh_orthonormal_by_quadrature():
    nt, npp = 200, 400
    th = (np.arange(nt) + 0.5) * math.pi / nt
    ph = (np.arange(npp) + 0.5) * 2 * math.pi / npp
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1).reshape(-1, 3)
    Y = field.sh_basis(d, 4)
    wq = (np.sin(TH) * (math.pi / nt) * (2 * math.pi / npp)).ravel()
    G = (Y * wq[:, None]).T @ Y
    assert np.allclose(G, np.eye(16), atol=2e-4)
    assert Y[0, 0] == pytest.approx(1 / (2 * math.sqrt(math.pi)))


def test_sh_matches_scipy_up_to_sign():
    from scipy import special
    rng = np.random.default_rng(5)
    d = rng.normal(size=(300, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    th = np.arccos(d[:, 2])
    ph = np.arctan2(d[:, 1], d[:, 0])
    Y = field.sh_basis(d, 4)
    col = 0
    for l in range(4):
        for m in range(-l, l + 1):
            c = special.sph_harm_y(l, abs(m), th, ph)
            if m > 0:
                ref = math.sqrt(2) * c.real
            elif m < 0:
                ref = math.sqrt(2) * c.imag
            else:
                ref = c.real
            sgn = np.sign(ref[np.argmax(np.abs(ref))] * Y[np.argmax(np.abs(ref)), col])
            assert np.allclose(Y[:, col], sgn * ref, atol=1e-12), (l, m)
            col += 1


# ----------------------------------------------------------------------------
# Rays, position path and marcher (P13)
# ----------------------------------------------------------------------------

def test_fp32_rays_agree_with_fp64():
    scene = W.blob_scene(0)
    poses = W.ring_poses([0.3, 2.0], 1.5)
    intr = np.array([[600, 600, 320, 240]] * 2, np.float32)
    ids = W.c2_candidates(2000, K=2)
    o32, d32, s32 = rays.rays_fp32(poses, intr, ids, 480, 640)
    o64, d64, s64 = rays.rays_fp64(poses.astype(np.float32), intr, ids, 480, 640)
    assert np.allclose(d32, d64, atol=3e-7)
    assert np.allclose(s32, s64, rtol=3e-7)
    assert np.allclose(np.linalg.norm(d64, axis=1), 1.0, atol=1e-14)


def _brute_march_fp64(spec, sampler, o, d, occ):
    """FP64 brute force over every lattice point, returns (t list, near-tie flag)."""
    out, ties = [], []
    lo, hi = np.array(spec.aabb_min), np.array(spec.aabb_max)
    G = sampler.grid_res
    k = 0
    while True:
        t = (k + 0.5) * sampler.dt
        k += 1
        if t > sampler.t_far:
            break
        if t < sampler.t_near:
            continue
        x = o + t * d
        if np.any(x < lo) or np.any(x > hi):
            ties.append(np.min(np.abs(np.concatenate([x - lo, x - hi]))) < 1e-5)
            continue
        p = (x - lo) / (hi - lo) * G
        c = np.minimum(np.floor(p), G - 1).astype(int)
        near = np.min(np.abs(p - np.round(p))) < 1e-5 or np.min(np.abs(np.concatenate([x - lo, x - hi]))) < 1e-5
        if occ[c[0] + G * (c[1] + G * c[2])]:
            out.append(t)
            ties.append(near)
        else:
            ties.append(near)
        if len(out) == sampler.max_per_ray:
            break
    return np.array(out), any(ties)


@pytest.mark.parametrize("G", [4, 8])
def test_marcher_against_brute_force(G):
    spec = W.C2_FIELD
    sampler = W.SamplerSpec(mode="occupancy", t_near=0.05, t_far=4.0, dt=1 / 64,
                            max_per_ray=40, grid_res=G)
    rng = np.random.default_rng(G)
    occ = rng.uniform(size=G ** 3) < 0.4
    words = W.pack_bits(occ)
    poses = W.ring_poses(rng.uniform(0, 2 * math.pi, 3), 1.5)
    intr = np.array([[60, 60, 32, 24]] * 3, np.float32)
    ids = W.c2_candidates(300, K=3, H=48, W=64)
    o32, d32, _ = rays.rays_fp32(poses, intr, ids, 48, 64)
    counts, ts = rays.march(spec, sampler, o32, d32, words)
    checked = 0
    for r in range(len(ids)):
        bt, tie = _brute_march_fp64(spec, sampler, o32[r].astype(np.float64), d32[r].astype(np.float64), occ)
        if tie:
            continue
        checked += 1
        assert counts[r] == len(bt)
        assert np.array_equal(ts[r].astype(np.float64), bt)
    assert checked > 250
    assert counts.max() > 0


def test_all_ones_bitfield_is_uniform_lattice_in_box():
    spec = W.C2_FIELD
    sampler = W.SamplerSpec(mode="occupancy", t_near=0.05, t_far=4.0, dt=1 / 128,
                            max_per_ray=1000, grid_res=8)
    words = W.pack_bits(np.ones(512, bool))
    poses = W.ring_poses([0.7], 1.5)
    intr = np.array([[60, 60, 32, 24]], np.float32)
    ids = np.arange(0, 48 * 64, 37, dtype=np.uint32)
    o32, d32, _ = rays.rays_fp32(poses, intr, ids, 48, 64)
    counts, ts = rays.march(spec, sampler, o32, d32, words)
    lo, hi, _ = rays.aabb_f32(spec)
    tl = rays.lattice_t(sampler)
    for r in range(len(ids)):
        x = rays.positions_f32(np.repeat(o32[r:r + 1], len(tl), 0), np.repeat(d32[r:r + 1], len(tl), 0), tl)
        assert np.array_equal(ts[r], tl[rays.inside_f32(x, lo, hi)])


def test_batch_cut():
    counts = np.array([3, 0, 5, 2, 7, 1])
    kept, rm = rays.batch_cut(counts, 10)
    assert kept.tolist() == [True, True, True, True, False, False]
    assert rm.tolist() == [True, False, True, True, False, False]


def test_occupancy_bit_layout():
    occ = np.zeros(4 ** 3, bool)
    occ[1 + 4 * (2 + 4 * 3)] = True
    words = W.pack_bits(occ)
    assert words[57 >> 5] == (1 << (57 & 31))
    assert np.array_equal(W.unpack_bits(words, 64), occ)


# ----------------------------------------------------------------------------
# Whole step: gradient by finite differences (P9, P11) and Adam (P12)
# ----------------------------------------------------------------------------

def _small_problem(seed=0, n_rays=64, table_range=0.5):
    spec = W.C1_FIELD
    lay = field.param_layout(spec)
    table, ws = W.init_params(seed, lay["table_floats"], spec.mlp_dims(), table_range)
    kf = W.c1_keyframes()
    ids = W.random_rays_subset(n_rays, 1024, seed=seed + 10)
    sampler = W.SamplerSpec(mode="uniform", t_near=1.0, t_far=3.0, dt=0.25, n_uniform=8,
                            max_per_ray=8, max_samples=1 << 20)
    return spec, lay, table, ws, kf, ids, sampler


def test_step_gradient_by_central_differences():
    spec, lay, table, ws, kf, ids, sampler = _small_problem()
    r = step.train_step(spec, sampler, kf, table, ws, ids, band=0.0)

    def loss(tab, wl):
        return step.train_step(spec, sampler, kf, tab, wl, ids, band=0.0)["loss"]

    rng = np.random.default_rng(0)
    # every weight block, a few entries each
    for li, Wl in enumerate(ws):
        for _ in range(6):
            i, j = rng.integers(0, Wl.shape[0]), rng.integers(0, Wl.shape[1])
            h = 1e-6
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[li][i, j] += h
            wm[li][i, j] -= h
            fd = (loss(table, wp) - loss(table, wm)) / (2 * h)
            an = r["grad_w"][li][i, j]
            assert an == pytest.approx(fd, rel=2e-5, abs=1e-7 * max(1, np.abs(r["grad_w"][li]).max())), (li, i, j)
    # touched table entries of every level
    touched = np.nonzero(r["grad_table"])[0]
    _, _, sizes, offs = field.level_layout(spec)
    for l in range(spec.levels):
        lo, hi = 2 * offs[l], 2 * (offs[l] + sizes[l])
        cand = touched[(touched >= lo) & (touched < hi)]
        for q in rng.choice(cand, size=min(5, len(cand)), replace=False):
            h = 1e-6
            tp, tm = table.copy(), table.copy()
            tp[q] += h
            tm[q] -= h
            fd = (loss(tp, ws) - loss(tm, ws)) / (2 * h)
            assert r["grad_table"][q] == pytest.approx(fd, rel=2e-5, abs=1e-7 * np.abs(r["grad_table"]).max())


def test_step_gradient_of_variance_seed():
    """dL/dV* path: seed g_V and compare d(sum g_V V*)/dtheta by FD."""
    spec, lay, table, ws, kf, ids, sampler = _small_problem(seed=1, n_rays=16)
    gv = np.random.default_rng(9).normal(size=16)
    lam = 0.0

    def obj(wl):
        rr = step.train_step(spec, sampler, kf, table, wl, ids, lam=lam, band=0.0)
        return rr["loss"] + (gv * rr["var_z"]).sum()

    r = step.train_step(spec, sampler, kf, table, ws, ids, lam=lam, band=0.0, g_var=gv)
    h = 1e-6
    for li in (0, len(ws) - 1):
        wp = [w.copy() for w in ws]
        wm = [w.copy() for w in ws]
        wp[li][0, 0] += h
        wm[li][0, 0] -= h
        fd = (obj(wp) - obj(wm)) / (2 * h)
        assert r["grad_w"][li][0, 0] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_mlp_adjoint_by_finite_differences():
    """dW = X^T dY and dX = dY W^T through both nets, against central
    differences of a random linear functional of (sigma, colour)."""
    spec = W.C2_FIELD
    rng = np.random.default_rng(3)
    S = 12
    _, ws = W.init_params(1, 0, spec.mlp_dims())
    e = rng.normal(size=(S, spec.enc_dim))
    d = rng.normal(size=(S, 3))
    sh = field.sh_basis(d / np.linalg.norm(d, axis=1, keepdims=True), spec.sh_bands)
    a = rng.normal(size=S)
    B = rng.normal(size=(S, 3))

    def obj(wl, ee):
        c = field.mlp_fwd(spec, wl, ee, np.abs(ee), sh, 0.0)
        return (a * c["sigma"]).sum() + (B * c["colour"]).sum()

    cache = field.mlp_fwd(spec, ws, e, np.abs(e), sh, 0.0)
    dWs, _, de, _ = field.mlp_bwd(spec, ws, cache, a, np.abs(a), B, np.abs(B), 0.0)
    h = 1e-6
    for li, Wl in enumerate(ws):
        for _ in range(4):
            i, j = rng.integers(0, Wl.shape[0]), rng.integers(0, Wl.shape[1])
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[li][i, j] += h
            wm[li][i, j] -= h
            fd = (obj(wp, e) - obj(wm, e)) / (2 * h)
            assert dWs[li][i, j] == pytest.approx(fd, rel=1e-6, abs=1e-8), (li, i, j)
    for _ in range(8):
        s_, k = rng.integers(0, S), rng.integers(0, spec.enc_dim)
        ep, em = e.copy(), e.copy()
        ep[s_, k] += h
        em[s_, k] -= h
        assert de[s_, k] == pytest.approx((obj(ws, ep) - obj(ws, em)) / (2 * h), rel=1e-6, abs=1e-8)


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(0)
    g = rng.normal(size=100)
    th = rng.normal(size=100)
    new, m, v = step.adam(th, np.zeros(100), np.zeros(100), g, 1, 1e-2, 0.9, 0.99, 1e-15)
    assert np.allclose(new - th, -1e-2 * g / (np.abs(g) + 1e-15), rtol=1e-12)
    assert np.allclose(new - th, -1e-2 * np.sign(g), rtol=1e-10)


def test_adam_matches_hand_recursion():
    g1, g2 = 0.3, -0.7
    th, m, v = step.adam(np.array([1.0]), np.zeros(1), np.zeros(1), np.array([g1]), 1, 0.1, 0.9, 0.99, 1e-8)
    th, m, v = step.adam(th, m, v, np.array([g2]), 2, 0.1, 0.9, 0.99, 1e-8)
    m2 = 0.9 * 0.1 * g1 + 0.1 * g2
    v2 = 0.99 * 0.01 * g1 ** 2 + 0.01 * g2 ** 2
    step1 = 1.0 - 0.1 * g1 / (abs(g1) + 1e-8)
    want = step1 - 0.1 * (m2 / (1 - 0.81)) / (math.sqrt(v2 / (1 - 0.9801)) + 1e-8)
    assert th[0] == pytest.approx(want, rel=1e-12)


def test_tiny_workload_shape():
    kf = W.c1_keyframes()
    assert int(np.isfinite(kf.depth_var).sum()) == 208
    spec = W.C1_FIELD
    lay = field.param_layout(spec)
    table, ws = W.init_params(0, lay["table_floats"], spec.mlp_dims())
    r = step.train_step(spec, W.C1_SAMPLER, kf, table, ws, W.c1_pixels())
    assert r["R"] == 1024 and r["S"] == 32768
    assert np.isfinite(r["loss"])
    # every gradient magnitude bounds its value
    assert np.all(np.abs(r["grad_table"]) <= r["grad_table_mag"] * (1 + 1e-12) + 1e-300)
    for g, m in zip(r["grad_w"], r["grad_w_mag"]):
        assert np.all(np.abs(g) <= m * (1 + 1e-12) + 1e-300)


def test_mlp_forward_with_constructed_weights():
    """Weights built so the nets compute a known function: selection and a
    non-symmetric permutation (a transposed square weight would pick a
    different unit)."""
    spec = W.C2_FIELD
    rng = np.random.default_rng(11)
    S = 20
    e = rng.uniform(0.1, 1.0, size=(S, 32))
    d = rng.normal(size=(S, 3))
    sh = field.sh_basis(d / np.linalg.norm(d, axis=1, keepdims=True), 4)
    W1 = np.zeros((32, 64)); W1[np.arange(32), np.arange(32)] = 1.0      # h1[:32] = e
    W2 = np.zeros((64, 16)); W2[5, 0] = 1.0; W2[7, 3] = 2.0               # o0 = e5, o3 = 2 e7
    W3 = np.zeros((32, 64)); W3[3, 10] = 1.0; W3[16, 20] = 1.0            # h3_10 = o3, h3_20 = relu(Y0)
    perm = np.roll(np.arange(64), 7)                                       # h4[perm[i]] = h3[i]
    W4 = np.zeros((64, 64)); W4[np.arange(64), perm] = 1.0
    W5 = np.zeros((64, 3)); W5[perm[10], 0] = 1.0; W5[perm[20], 2] = -1.0
    c = field.mlp_fwd(spec, [W1, W2, W3, W4, W5], e, e, sh, 0.0)
    assert np.allclose(c["sigma"], np.exp(e[:, 5]), rtol=1e-15)
    sig = lambda z: 1 / (1 + np.exp(-z))
    assert np.allclose(c["colour"][:, 0], sig(2 * e[:, 7]), rtol=1e-15)
    assert np.allclose(c["colour"][:, 1], 0.5)
    assert np.allclose(c["colour"][:, 2], sig(-np.maximum(sh[:, 0], 0)), rtol=1e-15)


# ----------------------------------------------------------------------------
# Marginal covariances (Eq. 1, 2)
# ----------------------------------------------------------------------------

def test_marginals_equal_blocks_of_the_dense_inverse():
    from oracle import covariance
    C, E, P, d = W.ba_window(seed=1, n_kf=3, h=4, w=5)
    c = C.shape[0]
    H = np.block([[C, E], [E.T, np.diag(P)]])
    Hinv = np.linalg.inv(H)
    ST, sd = covariance.marginals(C, E, P)
    assert np.allclose(ST, Hinv[:c, :c], rtol=1e-9, atol=1e-14)
    assert np.allclose(sd, np.diag(Hinv)[c:], rtol=1e-9, atol=1e-14)
    assert np.all(sd > 0) and np.all(np.linalg.eigvalsh(ST) > 0)


def test_depth_variance_is_the_delta_method():
    from oracle import covariance
    rng = np.random.default_rng(0)
    d0, s = 0.8, 0.004
    d = rng.normal(d0, s, 400000)
    mc = np.var(1.0 / d)
    assert covariance.depth_variance(s * s, d0) == pytest.approx(mc, rel=2e-2)
