"""Host math of the sweep intake (Section III-A): the per-column transforms.

* the twist transforms equal scipy's matrix exponential of the twist (the
  generator's own per-column poses);
* gyroscope integration with a constant rate equals the twist transforms'
  rotations; with a rate that changes every 10 ms it equals a fine
  step-by-step product of scipy exponentials;
* pack() gives the float32 [cols, 12] layout of ups_splat_sweep."""
import math

import numpy as np
import scipy.linalg

from paper_2101_00585_amd import intake
from synth import workloads as W


def _expm(w):
    M = np.zeros((3, 3))
    M[:] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    return scipy.linalg.expm(M)


def test_twist_transforms_match_generator():
    c = W.moving_sweep(omega=(0.2, -0.1, math.radians(90)), velocity=(3.0, 0.5, 0.1), rows=8, cols=128)
    T = intake.twist_transforms(128, c["xi"], c["period"], c["t_ref"])
    np.testing.assert_allclose(T, c["col_T"], atol=1e-12)


def test_gyro_constant_rate_equals_twist():
    w = np.array([0.3, -0.2, 1.5])
    gt = np.arange(0.0, 0.1, 0.01)
    T = intake.gyro_transforms(256, gt, np.tile(w, (len(gt), 1)))
    ref = intake.twist_transforms(256, np.concatenate([w, [0, 0, 0]]))
    np.testing.assert_allclose(T, ref, atol=1e-12)


def test_gyro_varying_rate_fine_integration():
    rng = np.random.default_rng(3)
    gt = np.arange(0.0, 0.1, 0.01)
    gw = rng.normal(0, 1.0, (len(gt), 3))
    cols = 64
    T = intake.gyro_transforms(cols, gt, gw, period=0.1, t_ref=0.5)

    def orient(t, h=1e-4):
        R = np.eye(3)
        s = 0.0
        while s < t - 1e-15:
            k = max(0, int(np.searchsorted(gt, s, side="right")) - 1)
            nxt = gt[k + 1] if k + 1 < len(gt) else np.inf
            e = min(t, s + h, nxt)
            R = R @ _expm(gw[k] * (e - s))
            s = e
        return R

    Rr = orient(0.05)
    for j in (0, 17, 33, 63):
        np.testing.assert_allclose(T[j, :3, :3], Rr.T @ orient(j / cols * 0.1), atol=1e-10)


def test_pack_layout():
    T = intake.twist_transforms(4, [0, 0, 1.0, 1.0, 0, 0])
    p = intake.pack(T)
    assert p.dtype == np.float32 and p.shape == (4, 12)
    np.testing.assert_allclose(p[:, :9].reshape(4, 3, 3), T[:, :3, :3], atol=1e-7)
    np.testing.assert_allclose(p[:, 9:], T[:, :3, 3], atol=1e-7)
