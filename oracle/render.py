"""Volume rendering, the mapping loss and their adjoints in FP64 (test
infrastructure; see package doc).

Per ray with samples i = 0..n-1 at distances t_i, bin widths delta_i,
densities sigma_i and colours c_i:

  tau_i = sigma_i * delta_i
  T_i   = exp(-sum_{j<i} tau_j)                     (Eq. 6)
  w_i   = T_i * (1 - exp(-tau_i))
  I*    = sum_i w_i c_i                             (colour, Sec. 3.2 after Eq. 7)
  d*    = sum_i w_i t_i                             (Eq. 5, d_i = t_i)
  V*    = sum_i w_i (t_i - d*)^2                    (depth variance; not in the
                                                     paper: unnormalised, like Eq. 5)
  A     = sum_i w_i                                 (opacity)

No background colour and no division by A: Eq. 5 and the colour sum are
unnormalised.  Loss for a batch of R rays (Eq. 3, 4, 7), mean over rays:

  l_r = sum_ch (I*_ch - I_ch)^2 + lambda_D * pi_r * (d*_r - D_r)^2

where D_r is the measured depth along the ray and pi_r = 1/Sigma_D,r the
precision (0 when the measurement is unusable).  ||x||^2_Sigma is read as
the Mahalanobis norm x^2 / Sigma with Sigma a variance.

Adjoint: for a sum Q = sum_i w_i q_i with q independent of tau (q = c, t, or 1
for the opacity A),
dQ/dtau_k = T_{k+1} q_k - sum_{i>k} w_i q_i, where T_{k+1} = T_k e^{-tau_k};
dV*/dtau_k adds -2 d*(1-A) dd*/dtau_k for the d* inside the square.
"""
from __future__ import annotations

import numpy as np


def composite_ray(sigma, colour, t, delta, stop_T=0.0):
    """Forward compositing of one ray; returns a dict of per-sample and
    per-ray quantities.  With stop_T > 0 only samples with T_i >= stop_T are
    composited (early termination for rendering)."""
    sigma = np.asarray(sigma, np.float64)
    tau = sigma * np.asarray(delta, np.float64)
    n = len(tau)
    T = np.empty(n + 1)
    T[0] = 1.0
    acc = 0.0
    for i in range(n):                 # explicit sequential prefix sum
        acc += tau[i]
        T[i + 1] = np.exp(-acc)
    n_used = n
    if stop_T > 0.0:
        below = np.nonzero(T[:n] < stop_T)[0]
        n_used = int(below[0]) if len(below) else n
    alpha = -np.expm1(-tau)
    w = T[:n] * alpha
    w[n_used:] = 0.0
    c = np.asarray(colour, np.float64)
    tt = np.asarray(t, np.float64)
    C = (w[:, None] * c).sum(0) if n else np.zeros(3)
    D = float((w * tt).sum())
    A = float(w.sum())
    V = float((w * (tt - D) ** 2).sum())
    return dict(tau=tau, T=T, w=w, C=C, D=D, A=A, V=V, n_used=n_used)


def composite_magnitudes(fw, t, delta, sigma_mag, colour, colour_mag, tol):
    """Running-error magnitudes of the rendered outputs of one ray, to first
    order: a float evaluation whose densities and colours are within tol
    times ``sigma_mag`` and ``colour_mag`` of the exact ones, and that rounds
    each step, lands within tol times these magnitudes of the exact outputs.

    Each quantity's magnitude is the same expression with every factor
    replaced by its magnitude:
      tau_m = delta sigma_mag;  P_i = sum_{j<i} tau_j, P_m likewise;
      T_m   = T (1 + P + P_m)              (dT = -T dP, plus the rounding);
      alpha_m = alpha + e^{-tau} tau_m;    w_m = T_m alpha + T alpha_m;
      C_m = sum w_m |c| + w c_m;  D_m = sum w_m |t|;  A_m = sum w_m.
    V* is evaluated in two passes (d* first).  Its terms are non-negative,
    and an error e of d* enters through the identity
      sum_i w_i (t_i - d* - e)^2 = V* - 2 e d* (1 - A) + A e^2,
    which holds because sum_i w_i (t_i - d*) = d* (1 - A) (Eq. 5, A = sum w),
    so V_m = sum w_m (t - d*)^2 + 2 |d*| |1 - A| D_m + tol A D_m^2.
    Samples past the early-termination stop carry no weight."""
    tau = fw["tau"]
    n = len(tau)
    tau_m = np.asarray(delta, np.float64) * np.asarray(sigma_mag, np.float64)
    P = np.concatenate([[0.0], np.cumsum(tau)])
    Pm = np.concatenate([[0.0], np.cumsum(tau_m)])
    T_m = fw["T"] * (1.0 + P + Pm)
    alpha = -np.expm1(-tau)
    alpha_m = alpha + np.exp(-tau) * tau_m
    w_m = T_m[:n] * alpha + fw["T"][:n] * alpha_m
    w_m[fw["n_used"]:] = 0.0
    w = fw["w"]
    tt = np.abs(np.asarray(t, np.float64))
    c = np.abs(np.asarray(colour, np.float64))
    cm = np.abs(np.asarray(colour_mag, np.float64))
    C_m = (w_m[:, None] * c + w[:, None] * cm).sum(0) if n else np.zeros(3)
    D_m = float((w_m * tt).sum())
    A_m = float(w_m.sum())
    u = (np.asarray(t, np.float64) - fw["D"]) ** 2
    V_m = float((w_m * u).sum()) + 2.0 * abs(fw["D"]) * abs(1.0 - fw["A"]) * D_m + tol * fw["A"] * D_m * D_m
    return dict(C=C_m, D=D_m, A=A_m, V=V_m, T=T_m, w=w_m, c=cm)


def composite_ray_bwd(fw, colour, t, delta, gC, gD, gV, gC_m=None, gD_m=None, gV_m=None, gA=0.0, mag=None):
    """Adjoint of ``composite_ray``: (dsigma, dcolour, magnitudes).

    Magnitudes evaluate the same formulas with every factor replaced by its
    magnitude (``mag`` from ``composite_magnitudes``; without it, the values
    themselves, i.e. exact densities and colours), with each suffix sum
    sum_{i>k} counted as |Q| + |Q_{<=k}| (a float32 kernel may form it as
    total minus prefix)."""
    gC = np.asarray(gC, np.float64)
    gC_m = np.abs(gC) if gC_m is None else np.asarray(gC_m, np.float64)
    gD_m = abs(gD) if gD_m is None else gD_m
    gV_m = abs(gV) if gV_m is None else gV_m
    w, T, n_used = fw["w"], fw["T"], fw["n_used"]
    n = len(w)
    c = np.asarray(colour, np.float64)
    tt = np.asarray(t, np.float64)
    dl = np.asarray(delta, np.float64)
    D, A, V = fw["D"], fw["A"], fw["V"]
    if mag is None:
        mag = dict(C=np.abs(fw["C"]), D=abs(D), A=A, V=abs(V), T=T, w=w, c=np.abs(c))
    u = (tt - D) ** 2
    Tn = T[1:]
    act = np.arange(n) < n_used
    # inclusive prefix sums Q_{<=k}
    Cp = np.cumsum(w[:, None] * c, 0)
    Dp = np.cumsum(w * tt)
    Vp = np.cumsum(w * u)
    dC = Tn[:, None] * c - (fw["C"][None, :] - Cp)
    dD = Tn * tt - (D - Dp)
    dVraw = Tn * u - (V - Vp)
    dV = dVraw - 2.0 * D * (1.0 - A) * dD
    Ap = np.cumsum(w)
    dA = Tn - (A - Ap)
    dtau = dC @ gC + gD * dD + gV * dV + gA * dA
    Tm, wm, cm = mag["T"][1:], mag["w"], mag["c"]
    ac, at = np.abs(c), np.abs(tt)
    um = u + 2.0 * np.abs(tt - D) * mag["D"]            # (t - d*)^2 with d* in error
    mC = Tm[:, None] * ac + Tn[:, None] * cm + mag["C"][None, :] + np.cumsum(wm[:, None] * ac + w[:, None] * cm, 0)
    mD = Tm * at + mag["D"] + np.cumsum(wm * at)
    mV = Tm * u + Tn * um + mag["V"] + np.cumsum(wm * u + w * um) \
        + 2.0 * (abs(D) * (1.0 + A) * mD + (mag["D"] * (1.0 + A) + abs(D) * mag["A"]) * np.abs(dD))
    mA = Tm + mag["A"] + np.cumsum(wm)
    dtau_m = mC @ gC_m + gD_m * mD + gV_m * mV + abs(gA) * mA
    dtau = np.where(act, dtau, 0.0)
    dtau_m = np.where(act, dtau_m, 0.0)
    dsig = dl * dtau
    dsig_m = dl * dtau_m
    dcol = w[:, None] * gC[None, :]
    dcol_m = wm[:, None] * np.abs(gC)[None, :] + w[:, None] * gC_m[None, :]
    return dsig, dcol, dsig_m, dcol_m


def loss_seeds(C, D, I, Dt, prec, R, lam, C_m=None, D_m=None):
    """Per-ray loss terms and seeds for rays with rendered (C, D) and targets
    (I, Dt, precision).  Returns (l_rgb, l_d, gC, gD, gC_mag, gD_mag); the
    seed magnitudes use the magnitudes C_m, D_m of the rendered values when
    given (else their absolute values)."""
    C = np.asarray(C, np.float64)
    I = np.asarray(I, np.float64)
    er = C - I
    ed = D - Dt
    l_rgb = (er * er).sum(-1)
    l_d = prec * ed * ed
    gC = 2.0 * er / R
    gD = 2.0 * lam * prec * ed / R
    C_m = np.abs(C) if C_m is None else np.asarray(C_m, np.float64)
    D_m = np.abs(D) if D_m is None else np.asarray(D_m, np.float64)
    gC_m = 2.0 * (C_m + np.abs(I)) / R
    gD_m = 2.0 * lam * prec * (D_m + np.abs(Dt)) / R
    return l_rgb, l_d, gC, gD, gC_m, gD_m


def precision_from_variance(depth_z, var_z, s):
    """pi = 1/(Sigma_z s^2) when Sigma_z > 0 and Sigma_z, D_z are finite;
    else 0 (unusable measurement)."""
    depth_z = np.asarray(depth_z, np.float64)
    var_z = np.asarray(var_z, np.float64)
    ok = np.isfinite(depth_z) & np.isfinite(var_z) & (var_z > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        pi = np.where(ok, 1.0 / (np.where(ok, var_z, 1.0) * s * s), 0.0)
    return pi, ok
