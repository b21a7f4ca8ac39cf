"""Pins of the oracle's tolerance code: the ReLU ambiguity band and the
widened magnitudes of ``oracle/field.py`` and the two-pass depth-variance
magnitude of ``oracle/render.py``.  Every GPU parity bound is tol times one of
these magnitudes, so each is checked against something other than itself:
equality with the exact oracle where nothing is ambiguous, the oracles with
an ambiguous unit forced either way, exact equality with |value| where no term
cancels, tightness of the widening, and the algebraic identity that the
variance bound rests on.  CPU only."""
import contextlib

import numpy as np
import pytest

import workloads as W
from oracle import field, render


def _mlp_inputs(spec, S, seed, positive=False):
    rng = np.random.default_rng(seed)
    _, ws = W.init_params(seed, 0, spec.mlp_dims())
    e = rng.normal(size=(S, spec.enc_dim))
    d = rng.normal(size=(S, 3))
    sh = field.sh_basis(d / np.linalg.norm(d, axis=1, keepdims=True), spec.sh_bands)
    dsig = rng.normal(size=S)
    dcol = rng.normal(size=(S, 3))
    if positive:
        ws = [np.abs(w) for w in ws]
        e = np.abs(e)
        sh = np.abs(sh)
        dsig, dcol = np.abs(dsig), np.abs(dcol)
    return ws, e, sh, dsig, dcol


def _run(spec, ws, e, sh, dsig, dcol, band):
    cache = field.mlp_fwd(spec, ws, e, np.abs(e), sh, band)
    dW, dWm, de, dem = field.mlp_bwd(spec, ws, cache, dsig, np.abs(dsig), dcol, np.abs(dcol), band)
    return cache, dW, dWm, de, dem


@contextlib.contextmanager
def _forced(decisions):
    """Replace the ReLU of the oracle so that in the k-th ReLU layer (in the
    order the forward visits them) the units flagged in decisions[k] = (sel,
    on) take the decision ``on`` there (True: h = pre and derivative 1;
    False: h = 0 and derivative 0).  The forced oracle is otherwise the
    exact one: no unit is flagged ambiguous."""
    orig = field._relu_with_band
    calls = [0]

    def relu(pre, pre_mag, band):
        h, mask, amb = orig(pre, pre_mag, band)
        k = calls[0]
        calls[0] += 1
        if k in decisions:
            sel, on = decisions[k]
            mask = np.where(sel, on.astype(np.float64), np.where(pre > 0, 1.0, 0.0))
            h = np.where(sel, np.where(on, pre, 0.0), np.maximum(pre, 0.0))
        return h, mask, np.zeros_like(amb)

    field._relu_with_band = relu
    try:
        yield
    finally:
        field._relu_with_band = orig


@pytest.mark.parametrize("spec,band", [(W.C1_FIELD, 1e-5), (W.C2_FIELD, 1e-6)], ids=["tiny", "full"])
def test_band_without_ambiguity_equals_exact(spec, band):
    """Where no unit is ambiguous the band changes nothing: every value and
    every magnitude equals that of the oracle without a band, bit for bit
    (a seed and band for which no pre-activation of the 32 samples lies in
    the band)."""
    ws, e, sh, dsig, dcol = _mlp_inputs(spec, 32, seed=5)
    c0, dW0, dWm0, de0, dem0 = _run(spec, ws, e, sh, dsig, dcol, 0.0)
    c1, dW1, dWm1, de1, dem1 = _run(spec, ws, e, sh, dsig, dcol, band)
    assert not c1["amb1"].any() and not any(a.any() for a in c1["ambs"])
    for k in ("sigma", "colour", "sigma_mag", "colour_mag"):
        assert np.array_equal(c0[k], c1[k]), k
    for a, b in zip(dW0 + dWm0 + [de0, dem0], dW1 + dWm1 + [de1, dem1]):
        assert np.array_equal(a, b)


def _check_within(name, got, mid, mag, tol):
    got, mid, mag = (np.asarray(x, np.float64).ravel() for x in (got, mid, mag))
    err = np.abs(got - mid)
    ratio = err / np.maximum(tol * mag, 1e-300)
    assert np.all(err <= tol * mag * (1 + 1e-9) + 1e-300), (name, float(ratio.max()))
    return float(ratio.max())


@pytest.mark.parametrize("spec,band", [(W.C1_FIELD, 2e-2), (W.C2_FIELD, 2e-2), (W.C2_FIELD, 5e-3)],
                         ids=["tiny-2e-2", "full-2e-2", "full-5e-3"])
def test_forced_decisions_lie_within_widened_bound(spec, band):
    """Each ambiguous unit may switch either way in a lower precision.  The
    oracle with the band carries the midpoint and widened magnitudes; the
    oracles with the ambiguous units forced on, forced off, or at random must
    all lie within band times those magnitudes, for the outputs, every
    weight gradient and the encoding gradient."""
    S = 24
    ws, e, sh, dsig, dcol = _mlp_inputs(spec, S, seed=7)
    cm, dWm_, dWmag, dem_, demag = _run(spec, ws, e, sh, dsig, dcol, band)
    ambs = [cm["amb1"]] + list(cm["ambs"])
    n_amb = [int(a.sum()) for a in ambs]
    assert sum(n_amb) >= 4, n_amb          # the case exercises the band
    rng = np.random.default_rng(1)

    def full(vals):
        """decisions per layer from values over that layer's ambiguous units"""
        out = {}
        for k, (a, v) in enumerate(zip(ambs, vals)):
            on = np.zeros(a.shape, bool)
            on[a] = v
            out[k] = (a, on)
        return out

    choices = [("on", full([np.ones(n, bool) for n in n_amb])), ("off", full([np.zeros(n, bool) for n in n_amb]))]
    choices += [(f"random{i}", full([rng.random(n) < 0.5 for n in n_amb])) for i in range(4)]
    # one unit against all the others
    for k, n in enumerate(n_amb):
        for j in range(min(n, 3)):
            for val in (True, False):
                vals = [np.full(m, not val) for m in n_amb]
                vals[k][j] = val
                choices.append((f"unit{k}.{j}={val}", full(vals)))
    worst = 0.0
    for name, dec in choices:
        with _forced(dec):
            cf, dWf, _, def_, _ = _run(spec, ws, e, sh, dsig, dcol, band)
        worst = max(worst, _check_within(f"{name} sigma", cf["sigma"], cm["sigma"], cm["sigma_mag"], band))
        worst = max(worst, _check_within(f"{name} colour", cf["colour"], cm["colour"], cm["colour_mag"], band))
        for j, (a, b, m) in enumerate(zip(dWf, dWm_, dWmag)):
            worst = max(worst, _check_within(f"{name} dW{j}", a, b, m, band))
        worst = max(worst, _check_within(f"{name} de", def_, dem_, demag, band))
    # the bound is not vacuous: some forced case uses a sizeable part of it
    assert worst > 0.25, worst


def test_magnitudes_bound_input_perturbations_tightly():
    """Magnitudes against perturbed inputs.  The encoding, SH inputs and
    seeds are moved by relative amounts up to tol (errors a lower-precision
    evaluation may carry into the nets); every output and gradient must move
    by at most tol times its magnitude.  With all inputs, weights and seeds
    non-negative nothing cancels and a coherent move (every input up by
    tol) uses at least half of each weight and encoding gradient's bound, so
    a magnitude a few times too large fails; the magnitudes of sigma and the
    colour also carry their own rounding and are only checked for validity.
    The table-gradient magnitude is the scatter of the encoding-gradient
    magnitudes with the (non-negative) trilinear weights: it equals the table
    gradient when those magnitudes equal the encoding gradient."""
    spec = W.C1_FIELD
    tol = 1e-6
    for positive in (True, False):
        ws, e, sh, dsig, dcol = _mlp_inputs(spec, 40, seed=3, positive=positive)
        ws = [w * 0.25 for w in ws]      # keeps the sigmoid away from saturation
        e = e * 0.5
        c, dW, dWm, de, dem = _run(spec, ws, e, sh, dsig, dcol, 0.0)
        rng = np.random.default_rng(0)
        moves = [lambda s: np.full(s, tol)] + [lambda s: rng.uniform(-tol, tol, s) for _ in range(3)]
        for k, mv in enumerate(moves):
            c2 = field.mlp_fwd(spec, ws, e * (1 + mv(e.shape)), np.abs(e), sh * (1 + mv(sh.shape)), 0.0)
            dW2, _, de2, _ = field.mlp_bwd(spec, ws, c2, dsig * (1 + mv(dsig.shape)), np.abs(dsig),
                                           dcol * (1 + mv(dcol.shape)), np.abs(dcol), 0.0)
            for nm, a, b, m in [("sigma", c2["sigma"], c["sigma"], c["sigma_mag"]),
                                ("colour", c2["colour"], c["colour"], c["colour_mag"]), ("de", de2, de, dem)] + \
                    [(f"dW{j}", a, b, m) for j, (a, b, m) in enumerate(zip(dW2, dW, dWm))]:
                r = np.abs(a - b) / (tol * m)
                assert r.max() <= 1.0 + 1e-6, (positive, k, nm, r.max())
                if positive and k == 0 and nm not in ("sigma", "colour"):
                    assert r.min() >= 0.5, (nm, r.min())
    rng = np.random.default_rng(0)
    xn = rng.uniform(size=(40, 3))
    n = field.param_layout(spec)["table_floats"]
    _, _, corners = field.encode_fwd(spec, np.zeros(n), xn)
    dpos = np.abs(rng.normal(size=(40, spec.enc_dim)))
    gt, gtm = field.encode_bwd(spec, corners, dpos, dpos, n)
    assert np.allclose(gtm, gt, rtol=1e-13, atol=0) and gt.max() > 0


def test_widening_is_tight_for_one_unit():
    """One sample, one hidden unit of the density net whose pre-activation is
    exactly zero: switching it moves its column of dW1 by half the unit's
    gradient, and the widened magnitude allows exactly that (plus the
    rounding allowance), so the forced oracles use at least 90% of the
    bound.  A widening several times too wide would fail here."""
    spec = W.C1_FIELD
    rng = np.random.default_rng(2)
    _, ws = W.init_params(4, 0, spec.mlp_dims())
    ws = [w.copy() for w in ws]
    e = rng.uniform(0.5, 1.0, size=(1, spec.enc_dim))
    e[0, :2] = 0.75, 0.625                            # exact products, so pre is exactly zero
    u = 5
    ws[0][:, u] = 0.0
    ws[0][0, u], ws[0][1, u] = e[0, 1], -e[0, 0]      # pre = e0 e1 - e1 e0 = 0 exactly
    d = np.array([[0.3, -0.4, 0.866]])
    sh = field.sh_basis(d / np.linalg.norm(d), spec.sh_bands)
    dsig, dcol = np.array([0.7]), np.array([[0.2, -0.5, 0.9]])
    tol = 1e-5
    cm, dWm_, dWmag, _, _ = _run(spec, ws, e, sh, dsig, dcol, tol)
    assert cm["pre1"][0, u] == 0.0 and cm["amb1"][0, u]
    amb_other = cm["amb1"].sum() - 1 + sum(a.sum() for a in cm["ambs"])
    assert amb_other == 0
    for val in (True, False):
        sel = np.zeros(cm["amb1"].shape, bool)
        sel[0, u] = True
        with _forced({0: (sel, np.full(sel.shape, val))}):
            _, dWf, _, _, _ = _run(spec, ws, e, sh, dsig, dcol, tol)
        col = np.abs(dWf[0][:, u] - dWm_[0][:, u]) / (tol * dWmag[0][:, u])
        nz = dWmag[0][:, u] > 0
        assert np.all(col[nz] <= 1 + 1e-9) and np.all(col[nz] >= 0.9), col


# ----------------------------------------------------------------------------
# Depth variance magnitude (two-pass V*)
# ----------------------------------------------------------------------------

def _random_ray(rng, n, opaque):
    t = np.sort(rng.uniform(0.5, 3.0, n))
    sigma = rng.uniform(0, 60 if opaque else 0.3, n)
    colour = rng.uniform(size=(n, 3))
    return render.composite_ray(sigma, colour, t, np.full(n, 0.02)), t


def _vmag(fw, t, tol):
    """V* magnitude of a ray with exact densities and colours"""
    n = len(t)
    return render.composite_magnitudes(fw, t, np.full(n, 0.02), np.zeros(n), np.zeros((n, 3)),
                                       np.zeros((n, 3)), tol)["V"]


@pytest.mark.parametrize("opaque", [False, True])
def test_variance_shift_identity(opaque):
    """The identity the variance magnitude rests on: with the weights fixed,
    sum_i w_i (t_i - d* - e)^2 = V* - 2 e d* (1 - A) + A e^2."""
    rng = np.random.default_rng(8)
    for _ in range(20):
        fw, t = _random_ray(rng, int(rng.integers(1, 80)), opaque)
        for e in (1e-3, -2e-5, 0.1):
            direct = float((fw["w"] * (t - fw["D"] - e) ** 2).sum())
            want = fw["V"] - 2 * e * fw["D"] * (1 - fw["A"]) + fw["A"] * e * e
            assert direct == pytest.approx(want, rel=1e-10, abs=1e-15)


@pytest.mark.parametrize("opaque", [False, True])
def test_variance_magnitude_covers_fp32_two_pass(opaque):
    """An FP32 two-pass evaluation (d* first, then the sum of squares) of the
    same weights lies within 1e-5 of the magnitude; a d* off by its full
    allowance (1e-5 of its own magnitude) still does, and on transparent rays
    that shift uses a sizeable part of the bound (it is not loose).  On
    opaque rays (1 - A tiny) the first-order shift term vanishes and the
    magnitude is the weight-error term sum w_m (t - d*)^2 plus the
    second-order tol A D_m^2."""
    rng = np.random.default_rng(9)
    tol = 1e-5
    worst_shift = 0.0
    n_opaque = 0
    for _ in range(40):
        n = int(rng.integers(2, 200))
        fw, t = _random_ray(rng, n, opaque)
        fm = render.composite_magnitudes(fw, t, np.full(n, 0.02), np.zeros(n), np.zeros((n, 3)),
                                         np.zeros((n, 3)), tol)
        mag = fm["V"]
        w32, t32 = fw["w"].astype(np.float32), t.astype(np.float32)
        d32 = np.float32(0.0)
        for a, b in zip(w32, t32):
            d32 = np.float32(d32 + a * b)
        v32 = np.float32(0.0)
        for a, b in zip(w32, t32):
            r = np.float32(b - d32)
            v32 = np.float32(v32 + a * np.float32(r * r))
        assert abs(float(v32) - fw["V"]) <= tol * mag
        for sgn in (1, -1):
            e = sgn * tol * fm["D"]
            shifted = float((fw["w"] * (t - fw["D"] - e) ** 2).sum())
            assert abs(shifted - fw["V"]) <= tol * mag * (1 + 1e-9)
            worst_shift = max(worst_shift, abs(shifted - fw["V"]) / (tol * mag))
        if 1.0 - fw["A"] < 1e-9:
            want = float((fm["w"] * (t - fw["D"]) ** 2).sum()) + tol * fw["A"] * fm["D"] ** 2
            assert mag == pytest.approx(want, rel=1e-6)
            n_opaque += 1
    if opaque:
        assert n_opaque >= 10
    else:
        assert worst_shift > 0.4, worst_shift


@pytest.mark.parametrize("opaque", [False, True])
def test_composite_magnitudes_bound_field_errors(opaque):
    """Rendered outputs of a ray whose densities and colours are off by up
    to tol times their magnitudes (random and coherent moves) stay within
    tol times the composite magnitudes, and the seeds of the backward from
    those outputs likewise; the magnitudes grow with the field's."""
    rng = np.random.default_rng(12)
    tol = 1e-7
    for _ in range(30):
        n = int(rng.integers(1, 120))
        t = np.sort(rng.uniform(0.5, 3.0, n))
        sigma = rng.uniform(0, 60 if opaque else 0.5, n)
        colour = rng.uniform(size=(n, 3))
        sm = sigma * rng.uniform(1, 5, n)
        cm = colour * rng.uniform(1, 3, (n, 3))
        dl = np.full(n, 0.02)
        fw = render.composite_ray(sigma, colour, t, dl)
        fm = render.composite_magnitudes(fw, t, dl, sm, colour, cm, tol)
        base = np.concatenate([fw["C"], [fw["D"], fw["V"], fw["A"]]])
        mag = np.concatenate([fm["C"], [fm["D"], fm["V"], fm["A"]]])
        for k in range(6):
            es = np.ones(n) if k == 0 else (-np.ones(n) if k == 1 else rng.uniform(-1, 1, n))
            ec = np.ones((n, 3)) if k == 0 else (-np.ones((n, 3)) if k == 1 else rng.uniform(-1, 1, (n, 3)))
            f2 = render.composite_ray(sigma + es * tol * sm, colour + ec * tol * cm, t, dl)
            got = np.concatenate([f2["C"], [f2["D"], f2["V"], f2["A"]]])
            assert np.all(np.abs(got - base) <= tol * mag * (1 + 1e-6) + 1e-300), (k, (got - base) / (tol * mag))
        fm0 = render.composite_magnitudes(fw, t, dl, sigma, colour, colour, tol)
        assert fm["D"] >= fm0["D"] and fm["A"] >= fm0["A"] and np.all(fm["C"] >= fm0["C"])


def test_adam_magnitudes_bound_input_errors():
    """Adam's result magnitudes: moving g, m and v by up to tol times their
    magnitudes moves theta, m and v by at most tol times the magnitudes of
    the results, over five chained steps; for all-positive inputs the
    coherent move of m and v uses their whole bound (the recursions have no
    cancellation), so a magnitude too large fails."""
    from oracle import step
    rng = np.random.default_rng(4)
    n, tol = 2000, 1e-7
    lr, b1, b2, eps = 1e-2, 0.9, 0.99, 1e-15
    for positive in (False, True):
        th = rng.normal(size=n)
        m = rng.normal(size=n) * 0.1
        v = rng.uniform(0.01, 1.0, n)
        if positive:
            m = np.abs(m)
        Mt, Mm, Mv = np.abs(th), np.abs(m), v.copy()
        for t in range(1, 6):
            g = rng.normal(size=n)
            if positive:
                g = np.abs(g)
            Mg = np.abs(g)
            th1, m1, v1 = step.adam(th, m, v, g, t, lr, b1, b2, eps)
            Mt1, Mm1, Mv1 = step.adam_magnitudes(th, m, v, g, t, lr, b1, b2, eps, Mt, Mm, Mv, Mg)
            for k in range(4):
                mv = (lambda: np.ones(n)) if k == 0 else (lambda: rng.uniform(-1, 1, n))
                th2, m2, v2 = step.adam(th + mv() * tol * Mt, m + mv() * tol * Mm, v + mv() * tol * Mv,
                                        g + mv() * tol * Mg, t, lr, b1, b2, eps)
                for nm, a, b, M in (("theta", th2, th1, Mt1), ("m", m2, m1, Mm1), ("v", v2, v1, Mv1)):
                    r = np.abs(a - b) / (tol * M)
                    assert r.max() <= 1.0 + 1e-5, (positive, t, k, nm, r.max())
                    if positive and k == 0 and nm in ("m", "v"):
                        assert r.min() >= 0.99, (t, nm, r.min())
            th, m, v, Mt, Mm, Mv = th1, m1, v1, Mt1, Mm1, Mv1


# ----------------------------------------------------------------------------
# The quantised (mixed-precision) oracle
# ----------------------------------------------------------------------------

def test_bf16_rounding_matches_the_library_conversion():
    """round_bf16 equals torch's float32 -> bfloat16 conversion (round to
    nearest, ties to even) on FP32 values, ties and neighbours of ties
    included; FP16 rounding is numpy's."""
    import torch
    from oracle import mixed
    rng = np.random.default_rng(0)
    x = (rng.normal(size=20000) * np.exp(rng.uniform(-30, 30, 20000))).astype(np.float32)
    bits = x.view(np.uint32)
    ties = ((bits & ~np.uint32(0xFFFF)) | np.uint32(0x8000)).view(np.float32)      # exactly half-way
    near = np.concatenate([ties, np.nextafter(ties, np.float32(np.inf)), np.nextafter(ties, np.float32(-np.inf))])
    for v in (x, near, np.array([0.0, -0.0, 1.0, -1.0, 3.0], np.float32)):
        want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(mixed.round_bf16(v.astype(np.float64)), want)
    assert np.array_equal(mixed.round_fp16(np.array([1.0 + 2 ** -11, 1.0 + 3 * 2 ** -11])),
                          np.array([1.0, 1.0 + 2 ** -9]))                             # ties to even


def test_quantised_oracle_without_quantisation_is_the_exact_oracle():
    """With the identity as quantiser and no ambiguity band, the quantised
    nets and scatter equal the exact ones."""
    from oracle import mixed
    ident = lambda a: np.asarray(a, np.float64)
    for spec in (W.C1_FIELD, W.C2_FIELD):
        ws, e, sh, dsig, dcol = _mlp_inputs(spec, 37, seed=4)
        ce = field.mlp_fwd(spec, ws, e, np.abs(e), sh, 0.0)
        dWe, dWme, dee, deme = field.mlp_bwd(spec, ws, ce, dsig, np.abs(dsig), dcol, np.abs(dcol), 0.0)
        cq = mixed.mlp_fwd(spec, ws, e, np.abs(e), sh, 0.0, rnd=ident)
        dWq, dWmq, deq, demq = mixed.mlp_bwd(spec, cq, dsig, np.abs(dsig), dcol, np.abs(dcol), 0.0)
        for k in ("sigma", "colour", "sigma_mag", "colour_mag"):
            assert np.array_equal(ce[k], cq[k]), k
        for a, b in zip(dWe + dWme + [dee, deme], dWq + dWmq + [deq, demq]):
            assert np.allclose(a, b, rtol=1e-13, atol=0)
        if spec.levels > 4:
            continue                                      # the scatter below on the tiny table only
        rng = np.random.default_rng(1)
        xn = rng.uniform(size=(37, 3))
        xn[5:20] = xn[5]                                  # a run of samples in one cell
        n = field.param_layout(spec)["table_floats"]
        _, _, corners = field.encode_fwd(spec, np.zeros(n), xn)
        ge, gme = field.encode_bwd(spec, corners, dee, deme, n)
        gq, gmq = mixed.encode_bwd(spec, corners, xn, dee, deme, n, rnd=ident)
        assert np.allclose(gq, ge, rtol=1e-12, atol=1e-15) and np.allclose(gmq, gme, rtol=1e-12, atol=1e-15)


def test_quantised_records_against_a_sample_loop():
    """The BF16 table-gradient records, formed sample by sample: a record per
    run of consecutive samples of one aligned group of 16 that share a cell,
    its value the BF16 rounding of the run's sum."""
    from oracle import mixed
    spec = W.C1_FIELD
    rng = np.random.default_rng(6)
    S = 53
    xn = rng.uniform(size=(S, 3))
    xn[10:24] = xn[10] + 1e-4 * rng.uniform(size=(14, 3))          # crosses a group boundary at 16
    xn[40:44] = xn[40]
    de = rng.normal(size=(S, 2 * spec.levels))
    n = field.param_layout(spec)["table_floats"]
    _, _, corners = field.encode_fwd(spec, np.zeros(n), xn)
    got, _ = mixed.encode_bwd(spec, corners, xn, de, np.abs(de), n)
    res, _, _, _ = field.level_layout(spec)
    want = np.zeros(n)
    for l, (idx, w) in enumerate(corners):
        cell, _ = field.cell_coords(xn, res[l])
        s = 0
        while s < S:
            e = s + 1
            while e < S and e % 16 != 0 and np.array_equal(cell[e], cell[s]):
                e += 1
            for c in range(8):
                for f in range(2):
                    v = sum(w[c][k] * de[k, 2 * l + f] for k in range(s, e))
                    want[2 * idx[c][s] + f] += mixed.round_bf16(v)
            s = e
    assert np.allclose(got, want, rtol=1e-12, atol=1e-18)


def test_quantised_step_within_the_mixed_tolerance_of_the_exact_step():
    """Cross-check of the two oracles on the tiny workload: the quantised
    step's outputs, loss and gradients lie within 2e-2 of the exact step's
    magnitudes (whose ReLU band is 2e-2), and they differ from it (the
    quantisation is there)."""
    from oracle import step
    spec, sampler = W.C1_FIELD, W.C1_SAMPLER
    kf = W.c1_keyframes()
    ids = W.random_rays_subset(200, 1024, seed=3)
    lay = field.param_layout(spec)
    table, ws = W.init_params(2, lay["table_floats"], spec.mlp_dims(), 0.3)
    ex = step.train_step(spec, sampler, kf, table, ws, ids, band=2e-2)
    q = step.train_step(spec, sampler, kf, table, ws, ids, band=4e-3, quantised=True, tol=2e-2)
    tol = 2e-2
    for k, m in (("rgb", "rgb_mag"), ("depth_z", "depth_z_mag"), ("var_z", "var_z_mag"), ("opacity", "opacity_mag")):
        assert np.all(np.abs(q[k] - ex[k]) <= tol * ex[m] + 1e-300), k
    assert abs(q["loss"] - ex["loss"]) <= tol * ex["loss"]
    assert np.all(np.abs(q["grad_table"] - ex["grad_table"]) <= tol * ex["grad_table_mag"] + 1e-300)
    for a, b, m in zip(q["grad_w"], ex["grad_w"], ex["grad_w_mag"]):
        assert np.all(np.abs(a - b) <= tol * m + 1e-300)
    assert not np.array_equal(q["grad_table"], ex["grad_table"])
