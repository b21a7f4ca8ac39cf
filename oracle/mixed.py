"""The field evaluated with the quantisation points of the mixed-precision
step made explicit, in FP64 otherwise (test infrastructure; see package doc).

The paper fixes no arithmetic precision (it trains with Instant-NGP's
kernels).  The mixed-precision step of this implementation quantises at
these points, and nowhere else:

* the hash tables are read from an FP16 copy of the FP32 masters;
* every MLP weight, and every operand of a matrix product -- the encoding,
  each hidden activation (after its ReLU), the density outputs and SH
  coefficients fed to the colour net, and every upstream gradient of the
  backward chain (after its ReLU mask) -- is rounded to BF16;
* dL/de leaves the backward rounded to BF16, and each table-gradient
  record, the sum of w_c * dL/de over a run of consecutive samples that
  share a grid cell (runs taken within aligned groups of 16 samples of the
  batch order), is rounded to BF16.

Products and sums are exact here (FP64); density, colour, compositing and
the loss are unquantised.  A quantisation point decides a discrete value,
so both sides take it in the same precision: this oracle rounds where the
kernels round.  What remains between the two is the FP32 rounding of the
kernels' sums, and rare roundings that land on the other side of a BF16 tie
because the FP32 value differs from the exact one.

Magnitudes follow ``oracle/field.py``'s running-error rules.  A ReLU unit is
ambiguous when its pre-activation lies within ``band`` of the abs-sum of its
own products (one flipped BF16 operand moves a pre-activation by at most
2^-8 of one product).
"""
from __future__ import annotations

import numpy as np

from . import field


def round_bf16(x):
    """Nearest BF16 value (8 significant bits, ties to even), as FP64."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)                       # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def round_fp16(x):
    """Nearest FP16 value (ties to even), as FP64."""
    return np.asarray(x, np.float64).astype(np.float16).astype(np.float64)


def _relu(pre, local, band):
    amb = np.abs(pre) <= band * local
    mask = np.where(amb, 0.5, np.where(pre > 0, 1.0, 0.0))
    return np.maximum(pre, 0.0), mask, amb


def encode_fwd(spec, table, xn, corners=None):
    """Encoding from the FP16 table copy, rounded to BF16 as the MLP
    consumes it.  Returns (e_bf16, magnitude, corners)."""
    e, em, corners = field.encode_fwd(spec, round_fp16(table), xn, corners)
    return round_bf16(e), em, corners


def mlp_fwd(spec, ws, e, e_mag, sh, band=4e-3, rnd=round_bf16):
    """Density and colour nets with BF16 weights and operands (``rnd`` is
    the quantiser; the identity gives the exact nets).  e must already be
    the quantised encoding.  Returns a cache like ``field.mlp_fwd``."""
    Wq = [rnd(w) for w in ws]
    aW = [np.abs(w) for w in Wq]
    pre1 = e @ Wq[0]
    loc1 = np.abs(e) @ aW[0]
    pre1_m = e_mag @ aW[0]
    r1, m1, amb1 = _relu(pre1, loc1, band)
    h1 = rnd(r1)
    h1_m = pre1_m * np.where(amb1, 2.0, m1)
    o = h1 @ Wq[1]
    o_m = h1_m @ aW[1]
    sigma = np.exp(o[:, 0])
    shq = rnd(sh)
    cur = np.concatenate([rnd(o), shq], 1)
    cur_m = np.concatenate([o_m, np.abs(shq)], 1)
    hs, hms, ms, ambs = [], [], [], []
    for Wl, al in zip(Wq[2:-1], aW[2:-1]):
        pre = cur @ Wl
        loc = np.abs(cur) @ al
        pre_m = cur_m @ al
        r, mk, amb = _relu(pre, loc, band)
        hs.append(cur)
        hms.append(cur_m)
        ms.append(mk)
        ambs.append(amb)
        cur, cur_m = rnd(r), pre_m * np.where(amb, 2.0, mk)
    z = cur @ Wq[-1]
    z_m = cur_m @ aW[-1]
    colour = 1.0 / (1.0 + np.exp(-z))
    return dict(W=Wq, e=e, e_mag=e_mag, pre1=pre1, h1=h1, h1_mag=h1_m, mask1=m1, amb1=amb1, o=o, sigma=sigma,
                hidden_in=hs, hidden_in_mag=hms, masks=ms, ambs=ambs, last_in=cur, last_in_mag=cur_m, z=z,
                colour=colour, sigma_mag=sigma * (1.0 + o_m[:, 0]), colour_mag=colour + colour * (1.0 - colour) * z_m,
                rnd=rnd)


def mlp_bwd(spec, cache, dsigma, dsigma_mag, dcol, dcol_mag, band_tol=2e-2):
    """Reverse mode with every product operand quantised as the kernels do:
    the upstream gradient of each layer is rounded once, after its ReLU
    mask, and that value feeds both the weight gradient and the next input
    gradient.  Returns (dW, dW magnitudes, dL/de rounded by the quantiser
    (the backward stores it as BF16 pairs for the table-gradient records),
    its magnitude)."""
    W, rnd = cache["W"], cache["rnd"]
    aW = [np.abs(w) for w in W]
    c = cache["colour"]
    dz = rnd(dcol * c * (1.0 - c))
    dz_m = dcol_mag * c * (1.0 - c) + np.abs(dcol) * np.abs(1.0 - 2.0 * c) * cache["colour_mag"]
    dWs, dWm = [None] * len(W), [None] * len(W)
    x = cache["last_in"]
    dWs[-1] = x.T @ dz
    dWm[-1] = np.abs(x).T @ dz_m + cache["last_in_mag"].T @ np.abs(dz)
    g = dz @ W[-1].T
    g_m = dz_m @ aW[-1].T
    for li in range(len(W) - 2, 1, -1):
        j = li - 2
        mk, amb = cache["masks"][j], cache["ambs"][j]
        g_m = field._widen(g_m, g, mk, amb, band_tol)
        g = rnd(g * mk)
        xin = cache["hidden_in"][j]
        dWs[li] = xin.T @ g
        dWm[li] = np.abs(xin).T @ g_m + cache["hidden_in_mag"][j].T @ np.abs(g)
        g, g_m = g @ W[li].T, g_m @ aW[li].T
    do = g[:, :spec.geo_dim].copy()
    do_m = g_m[:, :spec.geo_dim].copy()
    sig = cache["sigma"]
    do[:, 0] += dsigma * sig
    do_m[:, 0] += dsigma_mag * sig + np.abs(dsigma) * cache["sigma_mag"]
    do = rnd(do)
    h1 = cache["h1"]
    dWs[1] = h1.T @ do
    dWm[1] = np.abs(h1).T @ do_m + cache["h1_mag"].T @ np.abs(do)
    g = do @ W[1].T
    g_m = do_m @ aW[1].T
    mk, amb = cache["mask1"], cache["amb1"]
    g_m = field._widen(g_m, g, mk, amb, band_tol)
    g = rnd(g * mk)
    e = cache["e"]
    dWs[0] = e.T @ g
    dWm[0] = np.abs(e).T @ g_m + cache["e_mag"].T @ np.abs(g)
    return dWs, dWm, rnd(g @ W[0].T), g_m @ aW[0].T


def encode_bwd(spec, corners, xn, de, de_mag, n_table_floats, rnd=round_bf16, group=16):
    """Table gradient from BF16 records: per level, consecutive samples of an
    aligned group of ``group`` (in batch order) that share a grid cell form a
    run; the run's sum of w_c * dL/de for each corner and feature is one
    record, rounded by ``rnd``, and records are summed exactly."""
    F = spec.feat_per_level
    res, _, _, _ = field.level_layout(spec)
    n_entries = n_table_floats // F
    S = len(xn)
    g = np.zeros((n_entries, F))
    gm = np.zeros((n_entries, F))
    pos = np.arange(S)
    for l, (idx, w) in enumerate(corners):
        cell, _ = field.cell_coords(xn, res[l])
        head = pos % group == 0
        if S > 1:
            head[1:] |= np.any(cell[1:] != cell[:-1], axis=1)
        run = np.cumsum(head) - 1
        first = np.nonzero(head)[0]
        for c in range(8):
            for f in range(F):
                col = l * F + f
                v = np.bincount(run, weights=w[c] * de[:, col], minlength=len(first))
                vm = np.bincount(run, weights=w[c] * de_mag[:, col], minlength=len(first))
                g[:, f] += np.bincount(idx[c][first], weights=rnd(v), minlength=n_entries)
                gm[:, f] += np.bincount(idx[c][first], weights=vm, minlength=n_entries)
    return g.ravel(), gm.ravel()
