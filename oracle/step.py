"""The whole mapping step in FP64 (test infrastructure; see package doc).

One step of minimising L_M = L_rgb + lambda_D L_D (Sec. 3.2, Eq. 3) over the
field parameters Theta, with poses fixed: rays from keyframe pixels, samples,
field, compositing, loss, reverse mode, and optionally Adam.  The mapping
thread minimises L_M continuously over all keyframes received (Sec. 3.2,
Sec. 3.3); one call here is one iteration of that loop.
"""
from __future__ import annotations

import numpy as np

from . import field, mixed, rays, render


def forward_samples(spec, sampler, kf, pixel_ids, occupancy=None):
    """Rays, samples and the batch cut (no field evaluation)."""
    K, H, W = kf.rgb.shape[:3]
    o32, d32, s32 = rays.rays_fp32(kf.pose, kf.intr, pixel_ids, H, W)
    counts, ts = rays.march(spec, sampler, o32, d32, occupancy)
    kept, ray_mask = rays.batch_cut(counts, sampler.max_samples)
    sel = np.nonzero(ray_mask)[0]
    return dict(o32=o32, d32=d32, counts=counts, ts=ts, kept=kept, ray_mask=ray_mask,
                sel=sel, H=H, W=W)


def sample_positions(spec, o32, d32, ts, sel):
    """Flattened FP32 t, owning ray and normalised position of all samples
    of the selected rays."""
    lo, hi, inv = rays.aabb_f32(spec)
    t_all = np.concatenate([ts[r] for r in sel]) if len(sel) else np.zeros(0, np.float32)
    ray_of = np.concatenate([np.full(len(ts[r]), i) for i, r in enumerate(sel)]) \
        if len(sel) else np.zeros(0, np.int64)
    x = rays.positions_f32(o32[sel][ray_of], d32[sel][ray_of], t_all)
    xn = rays.normalise_f32(x, lo, inv)
    return t_all, ray_of, xn


def field_forward(spec, table, ws, xn, dirs, band=1e-5):
    """sigma, colour and caches for samples at xn with view directions dirs."""
    e, e_m, corners = field.encode_fwd(spec, table, xn)
    sh = field.sh_basis(dirs, spec.sh_bands)
    cache = field.mlp_fwd(spec, ws, e, e_m, sh, band)
    cache["corners"] = corners
    return cache


def train_step(spec, sampler, kf, table, ws, pixel_ids, occupancy=None, lam=1.0,
               band=1e-5, g_var=None, quantised=False, tol=None):
    """One forward+backward pass.  Returns a dict with per-ray outputs
    (rgb, depth_z, var_z, opacity), loss terms and gradients (with
    magnitudes).  ``g_var`` optionally seeds dL/dV*_z per selected ray (the
    loss itself does not use V*).

    quantised: evaluate the field with the mixed-precision step's
    quantisation points (``oracle/mixed.py``); band is then the ReLU
    ambiguity band relative to each unit's own product sums, and tol
    (default band) the tolerance the magnitudes serve."""
    tol = band if tol is None else tol
    fs = forward_samples(spec, sampler, kf, pixel_ids, occupancy)
    sel = fs["sel"]
    R = len(sel)
    o64, d64, s64 = rays.rays_fp64(kf.pose, kf.intr, pixel_ids, fs["H"], fs["W"])
    t_all, ray_of, xn = sample_positions(spec, fs["o32"], fs["d32"], fs["ts"], sel)
    if quantised:
        e, e_m, corners = mixed.encode_fwd(spec, table, xn)
        sh = field.sh_basis(d64[sel][ray_of], spec.sh_bands)
        cache = mixed.mlp_fwd(spec, ws, e, e_m, sh, band)
        cache["corners"] = corners
    else:
        cache = field_forward(spec, table, ws, xn, d64[sel][ray_of], band)
    sigma, colour = cache["sigma"], cache["colour"]
    # targets
    k, v, u = rays.split_pixel_ids(pixel_ids, fs["H"], fs["W"])
    I = kf.rgb[k, v, u].astype(np.float64)
    Dz = kf.depth[k, v, u].astype(np.float64)
    Vz = kf.depth_var[k, v, u].astype(np.float64)
    prec, ok = render.precision_from_variance(Dz, Vz, s64)
    Dray = np.where(ok, Dz * s64, 0.0)
    offs = np.concatenate([[0], np.cumsum([len(fs["ts"][r]) for r in sel])]).astype(np.int64)
    out_rgb = np.zeros((R, 3))
    out_d = np.zeros(R)
    out_v = np.zeros(R)
    out_a = np.zeros(R)
    mags = np.zeros((R, 6))                     # magnitudes of rgb, d*, V*, A
    fws, fms = [], []
    for i in range(R):
        a, b = offs[i], offs[i + 1]
        dl = np.full(b - a, sampler.dt)
        fw = render.composite_ray(sigma[a:b], colour[a:b], t_all[a:b], dl)
        fm = render.composite_magnitudes(fw, t_all[a:b], dl, cache["sigma_mag"][a:b], colour[a:b],
                                         cache["colour_mag"][a:b], tol)
        fws.append(fw)
        fms.append(fm)
        out_rgb[i], out_d[i], out_v[i], out_a[i] = fw["C"], fw["D"], fw["V"], fw["A"]
        mags[i] = [*fm["C"], fm["D"], fm["V"], fm["A"]]
    l_rgb, l_d, gC, gD, gC_m, gD_m = render.loss_seeds(out_rgb, out_d, I[sel], Dray[sel],
                                                       prec[sel], R, lam, mags[:, :3], mags[:, 3])
    L_rgb = l_rgb.sum() / R if R else 0.0
    L_D = l_d.sum() / R if R else 0.0
    gv = np.zeros(R) if g_var is None else np.asarray(g_var, np.float64) / s64[sel] ** 2
    S = len(t_all)
    dsig = np.zeros(S)
    dsig_m = np.zeros(S)
    dcol = np.zeros((S, 3))
    dcol_m = np.zeros((S, 3))
    for i in range(R):
        a, b = offs[i], offs[i + 1]
        ds, dc, dsm, dcm = render.composite_ray_bwd(
            fws[i], colour[a:b], t_all[a:b], np.full(b - a, sampler.dt),
            gC[i], gD[i], gv[i], gC_m[i], gD_m[i], abs(gv[i]), mag=fms[i])
        dsig[a:b], dcol[a:b], dsig_m[a:b], dcol_m[a:b] = ds, dc, dsm, dcm
    if quantised:
        dWs, dWm, de, de_m = mixed.mlp_bwd(spec, cache, dsig, dsig_m, dcol, dcol_m, tol)
        gtab, gtab_m = mixed.encode_bwd(spec, cache["corners"], xn, de, de_m, len(table))
    else:
        dWs, dWm, de, de_m = field.mlp_bwd(spec, ws, cache, dsig, dsig_m, dcol, dcol_m, band)
        gtab, gtab_m = field.encode_bwd(spec, cache["corners"], de, de_m, len(table))
    return dict(
        sel=sel, counts=fs["counts"], kept=fs["kept"], ray_mask=fs["ray_mask"], R=R, S=S,
        t=t_all, ray_of=ray_of, offsets=offs, xn=xn, sigma=sigma, colour=colour,
        rgb=out_rgb, depth_z=out_d / s64[sel], var_z=out_v / s64[sel] ** 2, opacity=out_a,
        rgb_mag=mags[:, :3], depth_z_mag=mags[:, 3] / s64[sel], var_z_mag=mags[:, 4] / s64[sel] ** 2,
        opacity_mag=mags[:, 5],
        depth_ray=out_d, var_ray=out_v, scale=s64[sel],
        loss=L_rgb + lam * L_D, loss_rgb=L_rgb, loss_d=L_D,
        dsigma=dsig, dsigma_mag=dsig_m, dcolour=dcol, dcolour_mag=dcol_m,
        grad_table=gtab, grad_table_mag=gtab_m, grad_w=dWs, grad_w_mag=dWm,
        encoding=cache["e"], n_amb=int(cache["amb1"].sum() + sum(a.sum() for a in cache["ambs"])))


def adam(theta, m, v, g, t, lr, b1, b2, eps):
    """Bias-corrected Adam, step t >= 1 (dense: every parameter, every step)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def adam_magnitudes(theta, m, v, g, t, lr, b1, b2, eps, M_theta, M_m, M_v, M_g):
    """First-order running-error magnitudes of one Adam step's results
    (theta, m, v), given the magnitudes of its inputs: every factor replaced
    by its magnitude, the square root halving a relative error, and the
    sums m, v, theta - update counted term by term.  Returns (M_theta, M_m,
    M_v) for the updated values."""
    m1 = b1 * m + (1.0 - b1) * g
    v1 = b2 * v + (1.0 - b2) * g * g
    Mm = b1 * M_m + (1.0 - b1) * M_g
    Mv = b2 * M_v + (1.0 - b2) * 2.0 * np.abs(g) * M_g
    bc1, bc2 = 1.0 - b1 ** t, 1.0 - b2 ** t
    den = np.sqrt(v1 / bc2) + eps
    with np.errstate(divide="ignore", invalid="ignore"):
        rel_v = np.where(v1 > 0, Mv / np.where(v1 > 0, v1, 1.0), 0.0)
    M_upd = lr / den * (Mm / bc1 + np.abs(m1) / bc1 * (1.0 + 0.5 * rel_v * np.sqrt(v1 / bc2) / den))
    return M_theta + M_upd, Mm, Mv


def render_image(spec, table, ws, pose, intr, H, W, sampler, stop_T=0.0, pixel_ids=None,
                 band=1e-5):
    """Forward-only render of an image (or of ``pixel_ids`` of it) with
    uniform samples and optional early termination at T < stop_T.
    Returns per-pixel rgb, depth_z, var_z, opacity and the per-ray stop
    index, plus for rays whose stop is ambiguous (T within 1e-5 relative of
    stop_T at the stopping sample) the outputs with one more sample."""
    ids = np.arange(H * W, dtype=np.uint32) if pixel_ids is None else np.asarray(pixel_ids)
    pose = np.asarray(pose)[None]
    intr = np.asarray(intr)[None]
    o32, d32, _ = rays.rays_fp32(pose, intr, ids, H, W)
    _, d64, s64 = rays.rays_fp64(pose, intr, ids, H, W)
    t = rays.uniform_t(sampler)
    n = len(t)
    lo, hi, inv = rays.aabb_f32(spec)
    R = len(ids)
    rr = np.repeat(np.arange(R), n)
    tt = np.tile(t, R)
    x = rays.positions_f32(o32[rr], d32[rr], tt)
    xn = rays.normalise_f32(x, lo, inv)
    cache = field_forward(spec, table, ws, xn, d64[rr], band)
    sig = cache["sigma"].reshape(R, n)
    col = cache["colour"].reshape(R, n, 3)
    sig_m = cache["sigma_mag"].reshape(R, n)
    col_m = cache["colour_mag"].reshape(R, n, 3)
    out = dict(rgb=np.zeros((R, 3)), depth_z=np.zeros(R), var_z=np.zeros(R), opacity=np.zeros(R),
               rgb_mag=np.zeros((R, 3)), depth_z_mag=np.zeros(R), var_z_mag=np.zeros(R),
               opacity_mag=np.zeros(R), n_used=np.zeros(R, np.int64), alt=dict())
    dl = np.full(n, sampler.dt)
    for r in range(R):
        fw = render.composite_ray(sig[r], col[r], t, dl, stop_T)
        fm = render.composite_magnitudes(fw, t, dl, sig_m[r], col[r], col_m[r], band)
        out["rgb"][r], out["depth_z"][r] = fw["C"], fw["D"] / s64[r]
        out["var_z"][r], out["opacity"][r], out["n_used"][r] = fw["V"] / s64[r] ** 2, fw["A"], fw["n_used"]
        out["rgb_mag"][r], out["depth_z_mag"][r] = fm["C"], fm["D"] / s64[r]
        out["var_z_mag"][r], out["opacity_mag"][r] = fm["V"] / s64[r] ** 2, fm["A"]
        if stop_T > 0.0:
            k = fw["n_used"]
            near = [j for j in (k - 1, k) if 0 <= j < n and abs(fw["T"][j] / stop_T - 1.0) < 1e-5]
            if near:
                alts = []
                for j in near:
                    # stop decided the other way at sample j
                    m = j + 1 if fw["T"][j] < stop_T else j
                    w = fw["T"][:n] * -np.expm1(-fw["tau"])
                    w[m:] = 0.0
                    C = (w[:, None] * col[r]).sum(0)
                    D = (w * t).sum()
                    alts.append(dict(rgb=C, depth_z=D / s64[r],
                                     var_z=(w * (t - D) ** 2).sum() / s64[r] ** 2,
                                     opacity=w.sum(), n_used=m))
                out["alt"][r] = alts
    return out
