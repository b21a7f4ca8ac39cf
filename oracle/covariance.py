"""Marginal covariances of the tracking Hessian in FP64 (test
infrastructure; see package doc).

The linear system of dense bundle adjustment is block-partitioned (Sec. 3.1,
Eq. 1) as [[C, E], [E^T, P]] with P diagonal (one inverse depth per pixel).
The reduced camera matrix is the Schur complement H_T = C - E P^{-1} E^T,
factorised as H_T = L L^T.  The marginal covariances are (Eq. 2)

    Sigma_T = (L L^T)^{-1}
    Sigma_d = P^{-1} + P^{-T} E^T Sigma_T E P^{-1}

of which the per-pixel inverse-depth variances are the diagonal of Sigma_d.
The depth loss (Eq. 4) weights the depth D = 1/d; to first order
var(D) = var(d) / d^4.
"""
from __future__ import annotations

import numpy as np


def schur(C, E, P):
    return C - (E / P[None, :]) @ E.T


def marginals(C, E, P):
    """(Sigma_T, diag Sigma_d) by Eq. 2."""
    L = np.linalg.cholesky(schur(C, E, P))
    Linv = np.linalg.inv(L)
    Sigma_T = Linv.T @ Linv              # (L L^T)^{-1}
    q = np.einsum("cj,cd,dj->j", E, Sigma_T, E)
    Pi = 1.0 / P
    return Sigma_T, Pi + Pi * Pi * q


def depth_variance(sigma_d, inv_depth):
    """First-order variance of D = 1/d."""
    return sigma_d / inv_depth ** 4
