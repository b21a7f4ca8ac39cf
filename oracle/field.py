"""Hash-grid radiance field in FP64 (test infrastructure; see package doc).

The paper builds its map on Instant-NGP and refers there for the network
inputs (Sec. 3.2, after Eq. 5; Sec. 3.4).  The field here is:

* multiresolution grid, level l at resolution N_l = floor(N_min * b^l), with
  b given or b = exp((ln N_max - ln N_min)/(L-1)); the top level is forced to
  N_max when N_max is given.  A level is dense (one entry per vertex) when
  (N_l+1)^3 fits the table, hashed otherwise;
* trilinear interpolation of F=2 features per level from the 8 cell corners;
* density net  h = ReLU(e W1), o = h W2 (16 wide), sigma = exp(o_0);
* colour net   c = sigmoid(MLP([o_0..o_15, SH(d)])) with ReLU hidden layers;
* all layers bias-free, weights stored [fan_in, fan_out].
"""
from __future__ import annotations

import math

import numpy as np

HASH_PRIMES = (1, 2654435761, 805459861)   # prior work's spatial hash


# ----------------------------------------------------------------------------
# Layout
# ----------------------------------------------------------------------------

def level_resolutions(spec):
    """Per-level grid resolutions N_l (FP64 power, floor)."""
    L = spec.levels
    if spec.per_level_scale is not None:
        b = float(spec.per_level_scale)
    else:
        b = math.exp((math.log(spec.max_res) - math.log(spec.base_res)) / (L - 1))
    res = [int(math.floor(spec.base_res * b ** l)) for l in range(L)]
    if spec.max_res is not None:
        res[-1] = int(spec.max_res)
    return res


def level_layout(spec):
    """(resolutions, dense flags, entries per level, entry offset per level)."""
    T = 1 << spec.log2_table
    res = level_resolutions(spec)
    dense = [(n + 1) ** 3 <= T for n in res]
    sizes = [min(T, (n + 1) ** 3) for n in res]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    return res, dense, sizes, offs


ALIGN_FLOATS = 64


def _align(n, a=ALIGN_FLOATS):
    return (n + a - 1) // a * a


def param_layout(spec):
    """Flat FP32 parameter vector: the tables (level-major, entry, feature),
    then every weight matrix [fan_in, fan_out] row-major, each block start
    aligned to 64 floats.  Returns dict(table_floats, w_offsets, total)."""
    _, _, sizes, _ = level_layout(spec)
    table_floats = int(sum(sizes)) * spec.feat_per_level
    off = _align(table_floats)
    w_offsets = []
    for fi, fo in spec.mlp_dims():
        w_offsets.append(off)
        off = _align(off + fi * fo)
    return dict(table_floats=table_floats, w_offsets=w_offsets, total=off)


def pack_params(spec, table, ws):
    lay = param_layout(spec)
    flat = np.zeros(lay["total"], np.float64)
    flat[:lay["table_floats"]] = table
    for o, w in zip(lay["w_offsets"], ws):
        flat[o:o + w.size] = np.asarray(w).ravel()
    return flat


def unpack_params(spec, flat):
    lay = param_layout(spec)
    table = np.asarray(flat[:lay["table_floats"]], np.float64)
    ws = []
    for o, (fi, fo) in zip(lay["w_offsets"], spec.mlp_dims()):
        ws.append(np.asarray(flat[o:o + fi * fo], np.float64).reshape(fi, fo))
    return table, ws


# ----------------------------------------------------------------------------
# Grid indexing and trilinear encoding
# ----------------------------------------------------------------------------

def corner_index(v, n, dense, T):
    """Table index of integer vertices v [...,3] at a level of resolution n."""
    v = v.astype(np.uint64)
    if dense:
        m = np.uint64(n + 1)
        return (v[..., 0] + m * (v[..., 1] + m * v[..., 2])).astype(np.int64)
    h = (v[..., 0] * np.uint64(HASH_PRIMES[0])) ^ (v[..., 1] * np.uint64(HASH_PRIMES[1])) \
        ^ (v[..., 2] * np.uint64(HASH_PRIMES[2]))
    h &= np.uint64(0xFFFFFFFF)
    return (h % np.uint64(T)).astype(np.int64)


def cell_coords(xn, n):
    """Lower cell corner and fractional offset of normalised points at
    resolution n: p = x_n*n (exact in FP64 for FP32 x_n), i0 =
    min(floor(p), n-1), f = p - i0."""
    p = np.asarray(xn, np.float64) * n
    i0 = np.minimum(np.floor(p), n - 1)
    return i0.astype(np.int64), p - i0


CORNERS = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], np.int64)


def encode_corners(spec, xn):
    """For every level and corner: (table index [S], weight [S]).

    Returns a list over levels of (idx [8,S] global entry index, w [8,S]).
    """
    res, dense, sizes, offs = level_layout(spec)
    T = 1 << spec.log2_table
    out = []
    for l, n in enumerate(res):
        i0, f = cell_coords(xn, n)
        idx = np.empty((8, len(xn)), np.int64)
        w = np.empty((8, len(xn)))
        for c, bits in enumerate(CORNERS):
            v = i0 + bits
            idx[c] = offs[l] + corner_index(v, n, dense[l], T)
            wc = np.where(bits == 1, f, 1.0 - f)
            w[c] = wc[:, 0] * wc[:, 1] * wc[:, 2]
        out.append((idx, w))
    return out


def encode_fwd(spec, table, xn, corners=None):
    """Encoding e [S, L*F]: per level, sum over corners of w_c * theta[idx_c].
    Returns (e, magnitude of e, corners)."""
    F = spec.feat_per_level
    tab = np.asarray(table, np.float64).reshape(-1, F)
    if corners is None:
        corners = encode_corners(spec, xn)
    S = len(xn)
    e = np.zeros((S, spec.levels * F))
    m = np.zeros_like(e)
    for l, (idx, w) in enumerate(corners):
        for c in range(8):
            v = tab[idx[c]]
            e[:, l * F:(l + 1) * F] += w[c][:, None] * v
            m[:, l * F:(l + 1) * F] += w[c][:, None] * np.abs(v)
    return e, m, corners


def encode_bwd(spec, corners, de, de_mag, n_table_floats):
    """Scatter dL/de into the table gradient: theta[idx_c] += w_c * de."""
    F = spec.feat_per_level
    n_entries = n_table_floats // F
    g = np.zeros((n_entries, F))
    gm = np.zeros((n_entries, F))
    for l, (idx, w) in enumerate(corners):
        for c in range(8):
            for f in range(F):
                col = l * F + f
                g[:, f] += np.bincount(idx[c], weights=w[c] * de[:, col], minlength=n_entries)
                gm[:, f] += np.bincount(idx[c], weights=w[c] * de_mag[:, col], minlength=n_entries)
    return g.ravel(), gm.ravel()


# ----------------------------------------------------------------------------
# Spherical harmonics (real, orthonormal, no Condon-Shortley phase)
# ----------------------------------------------------------------------------

def sh_basis(d, bands):
    """Real SH of unit directions d [S,3], ordered by band l then m=-l..l."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    out = [np.full_like(x, 0.5 / math.sqrt(pi))]
    if bands > 1:
        k1 = math.sqrt(3.0 / (4.0 * pi))
        out += [k1 * y, k1 * z, k1 * x]
    if bands > 2:
        a = 0.5 * math.sqrt(15.0 / pi)
        out += [a * x * y, a * y * z, 0.25 * math.sqrt(5.0 / pi) * (3 * z * z - 1),
                a * x * z, 0.25 * math.sqrt(15.0 / pi) * (x * x - y * y)]
    if bands > 3:
        c0 = 0.25 * math.sqrt(35.0 / (2 * pi))
        c1 = 0.5 * math.sqrt(105.0 / pi)
        c2 = 0.25 * math.sqrt(21.0 / (2 * pi))
        c3 = 0.25 * math.sqrt(7.0 / pi)
        c5 = 0.25 * math.sqrt(105.0 / pi)
        out += [c0 * y * (3 * x * x - y * y), c1 * x * y * z, c2 * y * (5 * z * z - 1),
                c3 * z * (5 * z * z - 3), c2 * x * (5 * z * z - 1),
                c5 * z * (x * x - y * y), c0 * x * (x * x - 3 * y * y)]
    if bands > 4:
        raise ValueError("at most 4 SH bands")
    return np.stack(out, -1)


# ----------------------------------------------------------------------------
# Networks
# ----------------------------------------------------------------------------

def _relu_with_band(pre, pre_mag, band):
    """ReLU value, derivative mask (0, 0.5 or 1) and ambiguity flags.

    A unit is ambiguous when |pre| <= band * magnitude(pre): its float32 sign
    is not determined by the FP64 value, so either derivative is admissible.
    """
    amb = np.abs(pre) <= band * pre_mag
    mask = np.where(pre > 0, 1.0, 0.0)
    mask = np.where(amb, 0.5, mask)
    return np.maximum(pre, 0.0), mask, amb


def mlp_fwd(spec, ws, e, e_mag, sh, band=1e-5):
    """Density and colour nets.  Returns a cache dict with sigma [S],
    colour [S,3] and every activation needed by ``mlp_bwd``.

    Forward magnitudes (abs-propagated inputs times |W|) find the ambiguous
    ReLU units and bound the activations' errors.  A unit that is off passes
    no magnitude on; an ambiguous unit passes on twice its pre-activation's
    magnitude, since a float value within tol * magnitude of a pre-activation
    itself within tol * magnitude of zero may be up to twice that far from
    the exact ReLU output.
    """
    W = ws
    a = dict(e=e, e_mag=e_mag, sh=sh, band=band)
    pre1 = e @ W[0]
    pre1_m = e_mag @ np.abs(W[0])
    h1, m1, amb1 = _relu_with_band(pre1, pre1_m, band)
    h1_m = pre1_m * np.where(amb1, 2.0, m1)
    o = h1 @ W[1]
    o_m = h1_m @ np.abs(W[1])
    sigma = np.exp(o[:, 0])
    cur = np.concatenate([o, sh], 1)
    cur_m = np.concatenate([o_m, np.abs(sh)], 1)
    hs, hms, ms, ambs = [], [], [], []
    for Wl in W[2:-1]:
        pre = cur @ Wl
        pre_m = cur_m @ np.abs(Wl)
        h, mk, amb = _relu_with_band(pre, pre_m, band)
        hs.append(cur)
        hms.append(cur_m)
        ms.append(mk)
        ambs.append(amb)
        cur, cur_m = h, pre_m * np.where(amb, 2.0, mk)
    z = cur @ W[-1]
    z_m = cur_m @ np.abs(W[-1])
    colour = 1.0 / (1.0 + np.exp(-z))
    # value magnitudes of the outputs: sigma = exp(o_0) inherits the absolute
    # error of o_0 as a relative error; sigmoid damps it by c(1-c).
    sigma_mag = sigma * (1.0 + o_m[:, 0])
    colour_mag = colour + colour * (1.0 - colour) * z_m
    a.update(pre1=pre1, h1=h1, h1_mag=h1_m, mask1=m1, amb1=amb1, o=o, sigma=sigma, hidden_in=hs,
             hidden_in_mag=hms, masks=ms, ambs=ambs, last_in=cur, last_in_mag=cur_m, z=z,
             colour=colour, sigma_mag=sigma_mag, colour_mag=colour_mag)
    return a


def _widen(g_m, g, mask, amb, band_tol):
    """Magnitude after a ReLU: passed through where the unit is on, and
    widened by |g|/(2 tol) where it is ambiguous."""
    out = g_m * np.where(amb, 1.0, mask)
    if band_tol > 0:
        out = out + np.where(amb, np.abs(g) / (2 * band_tol), 0.0)
    return out


def mlp_bwd(spec, ws, cache, dsigma, dsigma_mag, dcol, dcol_mag, band_tol=1e-5):
    """Reverse mode through both nets.

    Returns (dW list, dW magnitude list, de [S, L*F], de magnitude).
    Ambiguous ReLU units carry half the gradient (midpoint of {0, g}) and a
    magnitude widened by |g| / (2 tol) so that either float32 choice passes.

    Magnitudes are first-order running-error bounds: a product x*y carries
    |x| y_mag + x_mag |y|, so the error of the forward activations (x_mag, the
    forward magnitudes) enters the weight gradients, the sigmoid derivative
    (through the colour's magnitude) and the density term (through sigma's).
    """
    W = ws
    c = cache["colour"]
    dz = dcol * c * (1.0 - c)
    dz_m = dcol_mag * c * (1.0 - c) + np.abs(dcol) * np.abs(1.0 - 2.0 * c) * cache["colour_mag"]
    dWs = [None] * len(W)
    dWm = [None] * len(W)
    x_last = cache["last_in"]
    dWs[-1] = x_last.T @ dz
    dWm[-1] = np.abs(x_last).T @ dz_m + cache["last_in_mag"].T @ np.abs(dz)
    g = dz @ W[-1].T
    g_m = dz_m @ np.abs(W[-1]).T
    for li in range(len(W) - 2, 1, -1):       # colour hidden layers, backwards
        j = li - 2
        mk = cache["masks"][j]
        amb = cache["ambs"][j]
        g_m = _widen(g_m, g, mk, amb, band_tol)
        g = g * mk
        xin = cache["hidden_in"][j]
        dWs[li] = xin.T @ g
        dWm[li] = np.abs(xin).T @ g_m + cache["hidden_in_mag"][j].T @ np.abs(g)
        g_next = g @ W[li].T
        g_m = g_m @ np.abs(W[li]).T
        g = g_next
    # g is now dL/dx for x = [o, sh]; keep the geometry slice
    do = g[:, :spec.geo_dim].copy()
    do_m = g_m[:, :spec.geo_dim].copy()
    sig = cache["sigma"]
    do[:, 0] += dsigma * sig
    do_m[:, 0] += dsigma_mag * sig + np.abs(dsigma) * cache["sigma_mag"]
    h1 = cache["h1"]
    dWs[1] = h1.T @ do
    dWm[1] = np.abs(h1).T @ do_m + cache["h1_mag"].T @ np.abs(do)
    g = do @ W[1].T
    g_m = do_m @ np.abs(W[1]).T
    mk, amb = cache["mask1"], cache["amb1"]
    g_m = _widen(g_m, g, mk, amb, band_tol)
    g = g * mk
    e = cache["e"]
    dWs[0] = e.T @ g
    dWm[0] = np.abs(e).T @ g_m + cache["e_mag"].T @ np.abs(g)
    de = g @ W[0].T
    de_m = g_m @ np.abs(W[0]).T
    return dWs, dWm, de, de_m
