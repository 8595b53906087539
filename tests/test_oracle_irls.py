"""Pins of the oracle's absolute-value objective (Equation 1 prints |r|),
minimised by iteratively reweighted least squares with per-inlier weights
w = 1 / max(|r|, delta).

* a delta above every residual makes all weights equal, and a common weight
  cancels from the Gauss-Newton step: the pose equals the squared objective's;
* the reweighting's fixed point is a stationary point of Huber's function
  with threshold delta, the function whose gradient is w r: at convergence
  sum psi(r) J = 0 with psi(r) = clip(r / delta, -1, 1) computed here from
  the oracle's per-pixel residuals and Jacobians, while the squared
  objective's gradient (psi = r) and a wrong threshold (2 delta) stay far
  from zero there (the cases are ones where the re-association settles: on
  others a pixel at a gate boundary can flip in and out every iteration and
  the iteration ends in a two-cycle of correspondence sets);
* with outlier patches (surfaces moved between sweeps) the absolute-value
  objective's pose is several times closer to the truth than the squared
  one's.
"""
import numpy as np
import pytest

import oracle as O
import synth
from synth import workloads as W


def _case(seed):
    c = W.config0()
    g = c["geom"]
    kf = O.panorama_normals(g, c["kf"])
    scan = O.panorama_normals(g, W.outlier_patches(c["scan"].astype(np.float64), seed, 0.2))
    return c, g, kf, scan


@pytest.fixture(scope="module")
def case():
    return _case(5)


def test_large_delta_equals_squared_objective(case):
    c, g, kf, scan = case
    p2 = O.IcpParams(levels=2, iters=(10, 10))
    p1 = O.IcpParams(levels=2, iters=(10, 10), irls_delta=1e3)
    a = O.register(g, scan, g, kf, np.eye(4), p2)
    b = O.register(g, scan, g, kf, np.eye(4), p1)
    rot, tr = synth.pose_error(a["T"], b["T"])
    assert rot < 1e-12 and tr < 1e-12, (rot, tr)
    # the returned normal equations carry the common weight 1 / delta
    np.testing.assert_allclose(b["JtJ"] * 1e3, a["JtJ"], rtol=1e-9, atol=1e-9)


def _gradient(r, J, psi):
    grad = (psi[:, None] * J).sum(0)
    scale = (np.abs(psi)[:, None] * np.abs(J)).sum(0)
    return np.abs(grad / scale).max()


@pytest.mark.parametrize("seed,delta", [(7, 0.01), (5, 0.03)])
def test_fixed_point_is_huber_stationary(seed, delta):
    c, g, kf, scan = _case(seed)
    res = O.register(g, scan, g, kf, np.eye(4), O.IcpParams(levels=1, iters=(40,), irls_delta=delta))
    assert res["status"] == 0 and res["last_update_norm"] < 1e-12
    rr = O.residuals(g, scan, g, kf, res["T"], d_max=0.5)
    m = rr["inlier"]
    r, J = rr["r"][m], rr["J"][m]
    assert _gradient(r, J, np.clip(r / delta, -1.0, 1.0)) < 1e-10
    assert _gradient(r, J, r) > 1e-3
    assert _gradient(r, J, np.clip(r / (2 * delta), -1.0, 1.0)) > 1e-3
    # the weighted normal equations returned at the final pose agree
    ne = O.normal_equations(g, scan, g, kf, res["T"], d_max=0.5, irls_delta=delta)
    np.testing.assert_allclose(ne["b"], res["Jtr"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ne["b"], (np.clip(r / delta, -1, 1)[:, None] * J).sum(0), rtol=1e-9, atol=1e-9)


def test_more_robust_to_outlier_patches(case):
    c, g, kf, scan = case
    errs = {}
    for delta in (0.0, 0.01):
        res = O.register(g, scan, g, kf, np.eye(4), O.IcpParams(levels=2, iters=(30, 10), irls_delta=delta))
        assert res["status"] == 0
        errs[delta] = synth.pose_error(res["T"], c["T_gt"])
    (rot2, tr2), (rot1, tr1) = errs[0.0], errs[0.01]
    assert rot1 < 0.3 * rot2 and tr1 < 0.3 * tr2, errs
