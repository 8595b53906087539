"""Pins of the oracle's keyframe update (Section III-C: each keyframe pixel is
projected onto the registered sweep, similarity-filtered, and averaged with a
weight given by its sample count, saturated at 10).

* the count sequence is 1, 2, ..., 10, 10, ... (golden fixture);
* the running average follows d_k = (c d_{k-1} + x_k)/(c + 1) where x_k is the
  exact intersection of the keyframe ray with the k-th (shifted) plane;
* fusing a scan into itself at the identity changes no range;
* fusing noise-free planar scans at the true pose changes no range;
* the fill of empty keyframe pixels picks, per pixel, the nearest scan surfel
  among those whose brute-force nearest keyframe pixel it is (8x32).
"""
import math
import os

import numpy as np

import oracle as O
from synth import Geom, lidar_geom, se3, rot_z
from synth import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rays(g):
    el = g.el_top - np.arange(g.rows) * g.d_el
    az = 2 * np.pi * np.arange(g.cols) / g.cols
    E, A = np.meshgrid(el, az, indexing="ij")
    return np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1)


def _plane_surfels(g, n, d):
    """Surfel image of the plane {x : n.x = d} (n facing away from the origin
    when d > 0), with the sensor-facing normal -n."""
    U = _rays(g)
    den = U @ n
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(den > 0.2, d / den, 0.0)
    r[r > g.r_max] = 0.0
    s = np.zeros((g.rows, g.cols, 4))
    s[..., 3] = r
    s[r > 0, :3] = -n
    return s


def _golden_counts():
    rows = []
    with open(os.path.join(GOLDEN, "fuse_count_sequence.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([int(v) for v in line.split()])
    return rows


def test_count_sequence_saturates_at_10():
    g = lidar_geom(16, 64)
    n = np.array([1.0, 0.0, 0.0])
    scan = _plane_surfels(g, n, 4.0)
    kf = np.zeros_like(scan)
    cnt = np.zeros((16, 64), np.uint16)
    has = scan[..., 3] > 0
    seq = []
    for _ in range(14):
        kf, cnt = O.fuse(g, scan, g, kf, cnt, np.eye(4))
        vals = np.unique(cnt[has])
        assert len(vals) == 1
        seq.append(int(vals[0]))
    (golden,) = _golden_counts()
    assert seq == golden
    assert (cnt[~has] == 0).all()


def test_running_average_closed_form():
    """Keyframe of the plane x = 4; then planes x = 4 + e_k are fused at the
    identity.  Every updated pixel's range must follow the count-weighted
    running average of the exact ray/plane ranges."""
    g = lidar_geom(16, 64)
    n = np.array([1.0, 0.0, 0.0])
    U = _rays(g)
    kf = np.zeros((16, 64, 4))
    cnt = np.zeros((16, 64), np.uint16)
    kf, cnt = O.fuse(g, _plane_surfels(g, n, 4.0), g, kf, cnt, np.eye(4))
    # pixels whose rays meet the plane steeply enough that every shifted
    # sample stays inside the 0.2 m distance gate (|e_a - e_b| / (u.n) < 0.2)
    has = (cnt > 0) & ((U @ n) > 0.6)
    assert has.sum() > 100
    expect = kf[..., 3].copy()
    c = np.ones((16, 64))
    offsets = [0.025, -0.015, 0.05, 0.01, -0.04, 0.0, 0.02, 0.005, -0.01, 0.03, 0.015, -0.005]
    for e in offsets:
        kf, cnt = O.fuse(g, _plane_surfels(g, n, 4.0 + e), g, kf, cnt, np.eye(4))
        x = (4.0 + e) / (U @ n)
        expect = np.where(has, (c * expect + x) / (c + 1), expect)
        c = np.minimum(c + 1, 10)
        np.testing.assert_allclose(kf[..., 3][has], expect[has], rtol=0, atol=1e-12)
        assert (cnt[has] == c[has]).all()
        np.testing.assert_allclose(kf[..., :3][has], np.tile(-n, (has.sum(), 1)), atol=1e-12)


def test_identity_self_fusion_keeps_ranges():
    c = W.config0()
    g = c["geom"]
    s = O.panorama_normals(g, c["kf"])
    kf = s.copy()
    cnt = np.where((s[..., 3] > 0) & (np.abs(s[..., :3]).sum(-1) > 0), 3, 0).astype(np.uint16)
    kf2, cnt2 = O.fuse(g, s, g, kf, cnt, np.eye(4))
    upd = cnt > 0
    np.testing.assert_array_equal(kf2[..., 3][upd], s[..., 3][upd])
    # every pixel is updated except those seen at grazing incidence (|u.n| < 0.1)
    steep = np.abs(np.einsum("ijk,ijk->ij", _rays(g), s[..., :3])) >= 0.1
    assert (cnt2[upd & steep] == 4).all()
    assert (cnt2[upd & ~steep] == 3).all()
    np.testing.assert_allclose(kf2[..., :3][upd], s[..., :3][upd], atol=1e-15)


def test_planar_scans_at_true_pose_keep_ranges():
    """Noise-free box room without boxes, exact normals, FP64 ranges: fusing
    the scan at the true pose moves no keyframe range (ray/plane is exact)."""
    c = W.config0(noise=0.0, with_boxes=False, want_normals=True, dtype=np.float64)
    g = c["geom"]

    def surf(r, n):
        s = np.zeros(r.shape + (4,))
        s[..., :3] = n
        s[..., 3] = r
        return s

    kf = surf(c["kf"], c["kf_normals"])
    scan = surf(c["scan"], c["scan_normals"])
    cnt = np.where(kf[..., 3] > 0, 1, 0).astype(np.uint16)
    kf2, cnt2 = O.fuse(g, scan, g, kf, cnt, c["T_gt"])
    upd = cnt2 == 2
    assert upd.mean() > 0.9
    np.testing.assert_allclose(kf2[..., 3][upd], kf[..., 3][upd], rtol=0, atol=1e-9)


def test_fill_brute_force_8x32():
    g = Geom(8, 32, math.radians(12.0), math.radians(24.0) / 7, 0.0, 50.0)
    rng = np.random.default_rng(11)
    U = _rays(g)
    scan = np.zeros((8, 32, 4))
    scan[..., 3] = rng.uniform(2.0, 9.0, size=(8, 32))
    nrm = -U + 0.3 * rng.normal(size=U.shape)
    scan[..., :3] = nrm / np.linalg.norm(nrm, axis=-1, keepdims=True)
    scan[rng.random((8, 32)) < 0.1, 3] = 0.0
    scan[rng.random((8, 32)) < 0.1, :3] = 0.0
    kf = np.zeros((8, 32, 4))
    cnt = np.zeros((8, 32), np.uint16)
    # some keyframe pixels already hold samples and must not be filled
    kf[2, 3] = [0.0, 0.0, 1.0, 50.0]
    cnt[2, 3] = 4
    T = se3(rot_z(0.3), [0.4, 0.2, 0.05])
    kf2, cnt2 = O.fuse(g, scan, g, kf, cnt, T)
    R, t = T[:3, :3], T[:3, 3]
    el_rows = g.el_top - np.arange(8) * g.d_el
    az_cols = 2 * np.pi * np.arange(32) / 32
    best = {}
    for i in range(8):
        for j in range(32):
            s = scan[i, j]
            if not (s[3] > 0 and np.abs(s[:3]).sum() > 0):
                continue
            q = R @ (s[3] * U[i, j]) + t
            el = math.atan2(q[2], math.hypot(q[0], q[1]))
            az = math.atan2(q[1], q[0]) % (2 * math.pi)
            ki = int(np.argmin(np.abs(el_rows - el)))
            kj = int(np.argmin(np.abs((az_cols - az + math.pi) % (2 * math.pi) - math.pi)))
            if abs(el_rows[ki] - el) > g.d_el / 2:
                continue
            key = (np.linalg.norm(q), i * 32 + j)
            if (ki, kj) not in best or key < best[(ki, kj)][0]:
                best[(ki, kj)] = (key, R @ s[:3])
    assert len(best) > 50
    for ki in range(8):
        for kj in range(32):
            if (ki, kj) == (2, 3):
                assert cnt2[ki, kj] == 4
                continue
            if (ki, kj) in best:
                (rq, _), m = best[(ki, kj)]
                assert cnt2[ki, kj] == 1
                np.testing.assert_allclose(kf2[ki, kj, 3], rq, rtol=1e-14)
                np.testing.assert_allclose(kf2[ki, kj, :3], m, atol=1e-14)
            else:
                assert cnt2[ki, kj] == 0 and (kf2[ki, kj] == 0).all()
