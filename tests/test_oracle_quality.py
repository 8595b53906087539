"""Pins of the oracle's registration quality block (Section III-C: the
inlier ratio of a registration; the truncated cost that stands in for the
converged residual of the fallback rule).

At the final pose, over the level-0 scan pixels with a valid range:

* inliers / valid = the inlier ratio (valid counts ranges, not normals);
* rms = sqrt(sum of r^2 over inliers / inliers);
* truncated cost E = sum over valid pixels of min(r^2, tau^2), tau = d_max[0],
  where a pixel without an inlier correspondence (no normal, no keyframe
  pixel, rejected by Omega) counts tau^2.

A registration with zero iterations evaluates the block at its start pose, so
each pin below checks it at a chosen pose against a value derived without the
oracle's association or residual code: a brute-force nearest-pixel search on
8x32 in numpy, closed forms on the analytic box room, the scan against itself,
and a pose that leaves no correspondence.  d_max differs per level, so a tau
taken from another level fails; a tenth of the valid pixels have no normal,
so counting normal-valid instead of range-valid pixels fails.
"""
import math

import numpy as np

import oracle as O
from synth import Geom, se3, rot_x, rot_z
from synth import workloads as W

D_MAX = (0.7, 1.3, 2.9)
COS_T = math.cos(math.radians(40.0))


def _quality_at(g, scan, kf, T, d_max=D_MAX, cos_t=COS_T):
    """The oracle's quality block at pose T: three pyramid levels, no iterations."""
    p = O.IcpParams(levels=3, iters=(0, 0, 0), d_max=d_max, cos_theta_max=cos_t)
    res = O.register(g, scan, g, kf, T, p)
    assert res["iters_run"] == 0 and res["status"] == 0
    assert np.array_equal(res["T"], T)
    return res


def _rays(g):
    el = g.el_top - np.arange(g.rows) * g.d_el
    az = 2 * np.pi * np.arange(g.cols) / g.cols
    E, A = np.meshgrid(el, az, indexing="ij")
    return np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1)


def _brute_quality(g, scan, kf, T, tau, d_max, cos_t):
    """Inliers, valid count, sum of inlier r^2 and the truncated cost at T by
    exhaustive nearest-pixel search (numpy, no oracle code)."""
    U = _rays(g)
    R, t = T[:3, :3], T[:3, 3]
    el_rows = g.el_top - np.arange(g.rows) * g.d_el
    az_cols = 2 * np.pi * np.arange(g.cols) / g.cols
    n_in = n_valid = 0
    s_r2 = trunc = 0.0
    for i in range(g.rows):
        for j in range(g.cols):
            s2 = scan[i, j]
            if not (s2[3] > g.r_min and s2[3] <= g.r_max):
                continue
            n_valid += 1
            r = None
            if np.abs(s2[:3]).sum() > 0:
                q = R @ (s2[3] * U[i, j]) + t
                el = math.atan2(q[2], math.hypot(q[0], q[1]))
                az = math.atan2(q[1], q[0]) % (2 * math.pi)
                ki = int(np.argmin(np.abs(el_rows - el)))
                kj = int(np.argmin(np.abs((az_cols - az + math.pi) % (2 * math.pi) - math.pi)))
                s1 = kf[ki, kj]
                if (abs(el_rows[ki] - el) <= g.d_el / 2 and g.r_min < s1[3] <= g.r_max
                        and np.abs(s1[:3]).sum() > 0):
                    d = q - s1[3] * U[ki, kj]
                    if np.linalg.norm(d) <= d_max and (R @ s2[:3]) @ s1[:3] >= cos_t:
                        r = float(d @ s1[:3])
            if r is None:
                trunc += tau * tau
            else:
                n_in += 1
                s_r2 += r * r
                trunc += min(r * r, tau * tau)
    return n_in, n_valid, s_r2, trunc


def _random_surfels(rng, g, U):
    s = np.zeros((g.rows, g.cols, 4))
    s[..., 3] = rng.uniform(3.0, 6.0, size=(g.rows, g.cols))
    n = -U + rng.normal(size=U.shape) * 0.4
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    s[..., :3] = n
    s[rng.random((g.rows, g.cols)) < 0.1, :3] = 0.0     # valid range, no normal
    s[rng.random((g.rows, g.cols)) < 0.05, 3] = 0.0     # no return
    s[rng.random((g.rows, g.cols)) < 0.03, 3] = 60.0    # beyond r_max: not a valid range
    return s


def test_quality_brute_force_8x32():
    g = Geom(8, 32, math.radians(12.0), math.radians(24.0) / 7, 0.0, 50.0)
    U = _rays(g)
    rng = np.random.default_rng(11)
    checked_in = 0
    for trial in range(4):
        kf, scan = _random_surfels(rng, g, U), _random_surfels(rng, g, U)
        T = se3(rot_z(0.05 * (trial + 1)) @ rot_x(0.02), [0.1, -0.05 * trial, 0.02])
        res = _quality_at(g, scan, kf, T)
        n_in, n_valid, s_r2, trunc = _brute_quality(g, scan, kf, T, D_MAX[0], D_MAX[0], COS_T)
        assert res["valid"] == n_valid and res["inliers"] == n_in, (trial, res["valid"], n_valid, res["inliers"], n_in)
        assert n_valid > n_in > 10
        assert res["inlier_ratio"] == n_in / n_valid
        np.testing.assert_allclose(res["rms"], math.sqrt(s_r2 / n_in), rtol=1e-12)
        np.testing.assert_allclose(res["trunc_cost"], trunc, rtol=1e-12)
        # a tau of another level would add (tau_l^2 - tau_0^2) per non-inlier
        assert abs(res["trunc_cost"] - (trunc + (D_MAX[1] ** 2 - D_MAX[0] ** 2) * (n_valid - n_in))) > 1.0
        checked_in += n_in
    assert checked_in > 100


def _analytic_room_surfels():
    c = W.config0(noise=0.0, with_boxes=False, want_normals=True, dtype=np.float64)
    s = np.zeros(c["kf"].shape + (4,))
    s[..., :3] = c["kf_normals"]
    s[..., 3] = c["kf"]
    return c["geom"], s


def test_quality_closed_form_shifted_room():
    """The exact-normal room against itself moved by delta along x: an inlier
    whose keyframe pixel lies on the scan point's plane has r = delta * n1_x
    (the plane offset), so sum r^2 = delta^2 sum n1_x^2 over the inliers, and
    every valid pixel that is not an inlier adds tau^2 (here the scan pixels
    whose normal was cleared)."""
    g, s = _analytic_room_surfels()
    scan = s.copy()
    scan[np.random.default_rng(5).random(g.shape) < 0.1, :3] = 0.0
    delta = 0.013
    T = se3(np.eye(3), [delta, 0.0, 0.0])
    d_max = (0.5, 1.0, 2.0)
    cos_t = math.cos(math.radians(30.0))
    res = _quality_at(g, scan, s, T, d_max=d_max, cos_t=cos_t)
    idx, inl = O.correspondences(g, scan, g, s, T, d_max[0], cos_t)
    n1 = s[..., :3].reshape(-1, 3)[idx[inl]]
    valid = int(((scan[..., 3] > 0) & (scan[..., 3] <= g.r_max)).sum())
    n_in = int(inl.sum())
    s_r2 = delta ** 2 * float((n1[:, 0] ** 2).sum())
    assert res["valid"] == valid and res["inliers"] == n_in
    assert valid - n_in > 1000 and (np.abs(n1[:, 0]) > 0.99).sum() > 1000
    np.testing.assert_allclose(res["rms"], math.sqrt(s_r2 / n_in), rtol=1e-9)
    np.testing.assert_allclose(res["trunc_cost"], s_r2 + d_max[0] ** 2 * (valid - n_in), rtol=1e-12)


def test_quality_scan_against_itself():
    """At the identity every pixel with a range and a normal is its own inlier
    with r = 0: rms 0, and the truncated cost is tau^2 per valid range without
    a normal."""
    c = W.config0()
    g = c["geom"]
    s = O.panorama_normals(g, c["scan"])
    res = _quality_at(g, s, s, np.eye(4))
    rng_ok = (s[..., 3] > g.r_min) & (s[..., 3] <= g.r_max)
    has_n = np.abs(s[..., :3]).sum(-1) > 0
    assert (rng_ok & ~has_n).sum() > 50
    assert res["valid"] == rng_ok.sum() and res["inliers"] == (rng_ok & has_n).sum()
    assert res["rms"] == 0.0
    np.testing.assert_allclose(res["trunc_cost"], D_MAX[0] ** 2 * float((rng_ok & ~has_n).sum()), rtol=1e-12)


def test_quality_no_correspondence():
    """Moved 40 m up, every scan point leaves the keyframe's rows or misses
    the distance gate: no inliers, rms 0, ratio 0, tau^2 per valid range."""
    c = W.config0()
    g = c["geom"]
    s = O.panorama_normals(g, c["scan"])
    res = _quality_at(g, s, s, se3(np.eye(3), [0.0, 0.0, 40.0]))
    valid = int(((s[..., 3] > g.r_min) & (s[..., 3] <= g.r_max)).sum())
    assert res["inliers"] == 0 and res["valid"] == valid and valid > 30000
    assert res["rms"] == 0.0 and res["inlier_ratio"] == 0.0
    np.testing.assert_allclose(res["trunc_cost"], D_MAX[0] ** 2 * valid, rtol=1e-12)
