"""Depth covariances from the tracking Hessian (Eq. 1, 2) on the GPU against
the FP64 oracle, and the failure flag for a non-positive-definite system."""
import numpy as np
import pytest

import workloads as W
from oracle import covariance as ocov
from parity import report

pytestmark = pytest.mark.gpu


def _t(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("n_kf,h,w", [(2, 3, 5), (8, 30, 40), (10, 12, 16)])
def test_covariance_matches_oracle(nsl, gpu, n_kf, h, w):
    import torch
    dev = gpu
    report(f"covariance: window {n_kf} keyframes of {w}x{h}")
    C, E, P, d = W.ba_window(seed=n_kf, n_kf=n_kf, h=h, w=w)
    sT, sd, dv, st = nsl.depth_covariance(_t(torch, dev, C), _t(torch, dev, E.T), _t(torch, dev, P),
                                          _t(torch, dev, d))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    oT, od = ocov.marginals(C, E, P)
    assert np.allclose(sT.cpu().numpy(), oT, rtol=1e-9, atol=1e-12 * np.abs(oT).max())
    assert np.allclose(sd.cpu().numpy(), od, rtol=1e-9)
    assert np.allclose(dv.cpu().numpy(), ocov.depth_variance(od, d), rtol=1e-6)


def test_covariance_flags_indefinite_system(nsl, gpu):
    import torch
    dev = gpu
    C, E, P, d = W.ba_window(seed=3, n_kf=2, h=3, w=4)
    C = C - 1e6 * np.eye(C.shape[0])          # H_T no longer positive definite
    sT, sd, dv, st = nsl.depth_covariance(_t(torch, dev, C), _t(torch, dev, E.T), _t(torch, dev, P),
                                          _t(torch, dev, d))
    torch.cuda.synchronize()
    assert int(st.item()) == 1
    assert np.isnan(sT.cpu().numpy()).all()
