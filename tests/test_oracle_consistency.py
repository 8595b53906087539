"""Pins of the oracle's moving-object check across keyframes (Section III-C:
the keyframes are checked against each other when the current keyframe
changes, so that what moved between them is removed).

Reading: a sample of keyframe A is removed when keyframe B saw more than
max(margin_abs, margin_rel * range) beyond it on every ray of the 3x3
neighbourhood of its pixel in B.

* closed forms with T = I (a pixel maps onto itself): a near patch in front of
  a far background is removed exactly, minus the rows whose neighbourhood
  leaves the image; a patch within the margin stays; an invalid or
  under-counted pixel of B next to a patch pixel keeps it;
* a yaw by exactly k columns maps A's column j onto B's column j + k (the
  direction of T_ba is checked: the inverse pose moves the patch elsewhere);
* two keyframes of a static room (1 cm noise): nothing is removed;
* keyframes with person-sized boxes that moved: every removed sample belongs
  to a mover, and most movers are removed;
* the mutual check is symmetric under swapping the keyframes.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth
from synth import lidar_geom, rot_z, se3
from synth import workloads as W


def _surf(r):
    s = np.zeros(r.shape + (4,))
    s[..., 2] = 1.0
    s[..., 3] = r
    return s


G = lidar_geom(16, 64)


def _sphere(r=10.0):
    return np.full((G.rows, G.cols), r)


def test_patch_in_front_of_background_removed_exactly():
    a = _sphere()
    a[4:9, 10:20] = 5.0       # removed (10 > 5 + 0.2)
    a[4:9, 30:40] = 9.85      # inside the margin: kept
    a[4:9, 44:50] = 9.7       # 10 > 9.7 + max(0.2, 0.194): removed
    a[0, 55:60] = 5.0         # first row: the neighbourhood leaves the image, kept
    a[15, 55:60] = 5.0        # last row: kept
    a[10:14, 20:30] = 40.0    # a far wall seen by both
    a[11:13, 22:25] = 39.5    # 40 < 39.5 + max(0.2, 0.79): the relative margin keeps it
    a[11:13, 25:28] = 39.0    # 40 > 39.0 + 0.78: removed
    b = _sphere()
    b[10:14, 20:30] = 40.0
    m = O.free_space_violations(G, _surf(a), G, _surf(b), None, np.eye(4))
    want = np.zeros_like(m)
    want[4:9, 10:20] = True
    want[4:9, 44:50] = True
    want[11:13, 25:28] = True
    assert np.array_equal(m, want)


def test_invalid_or_undercounted_neighbour_keeps_sample():
    a = _sphere()
    a[6, 20] = 5.0
    a[6, 40] = 5.0
    a[6, 63] = 5.0            # column 63 wraps onto column 0
    b = _sphere()
    b[7, 21] = 0.0            # no return next to (6, 20)
    cnt = np.full((G.rows, G.cols), 3, np.uint16)
    cnt[5, 39] = 1            # one sample next to (6, 40)
    cnt[6, 0] = 1             # one sample at the wrapped neighbour of (6, 63)
    p = O.ConsistencyParams(min_count=2)
    m = O.free_space_violations(G, _surf(a), G, _surf(b), cnt, np.eye(4), p)
    assert not m.any()
    cnt[5, 39] = cnt[6, 0] = 2
    b[7, 21] = 10.0
    m = O.free_space_violations(G, _surf(a), G, _surf(b), cnt, np.eye(4), p)
    assert m[6, 20] and m[6, 40] and m[6, 63] and m.sum() == 3


def test_yaw_by_whole_columns_maps_columns():
    k = 5
    a = _sphere()
    a[6:9, 10:14] = 4.0
    # B's frame is A's turned by +k columns: a point at A's azimuth az is at
    # az - 2 pi k / W in B, i.e. B = Rz(-2 pi k / W) A
    T_ba = se3(rot_z(-2 * math.pi * k / G.cols))
    b = _sphere()
    b[6:9, 10 - k:14 - k] = 4.0      # B sees the patch too, shifted: nothing removed
    m = O.free_space_violations(G, _surf(a), G, _surf(b), None, T_ba)
    assert not m.any()
    # the same B under the opposite rotation sees through the patch
    m = O.free_space_violations(G, _surf(a), G, _surf(b), None, se3(rot_z(2 * math.pi * k / G.cols)))
    want = np.zeros_like(m)
    want[6:9, 10:14] = True
    assert np.array_equal(m, want)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_static_room_nothing_removed(seed):
    c = W.moving_objects_pair(seed)
    g = c["geom"]
    st = c["static"]
    a = O.panorama_normals(g, synth.render(st, g, c["T_world_a"], 0.01, 5))
    b = O.panorama_normals(g, synth.render(st, g, c["T_world_b"], 0.01, 6))
    assert not O.free_space_violations(g, a, g, b, None, c["T_ba"]).any()
    assert not O.free_space_violations(g, b, g, a, None, np.linalg.inv(c["T_ba"])).any()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_movers_removed_and_nothing_else(seed):
    c = W.moving_objects_pair(seed)
    g = c["geom"]
    a = O.panorama_normals(g, c["kf_a"])
    b = O.panorama_normals(g, c["kf_b"])
    a2, _, b2, _, ma, mb = O.keyframe_consistency(g, a, None, g, b, None, c["T_ba"])
    for m, truth in ((ma, c["mover_a"]), (mb, c["mover_b"])):
        assert not (m & ~truth).any()                 # no static sample removed
        assert (m & truth).sum() >= 0.3 * truth.sum()  # most movers seen through
    assert np.all(a2[ma] == 0) and np.array_equal(a2[~ma], a[~ma])
    assert np.all(b2[mb] == 0) and np.array_equal(b2[~mb], b[~mb])


def test_mutual_check_symmetric():
    c = W.moving_objects_pair(1)
    g = c["geom"]
    a = O.panorama_normals(g, c["kf_a"])
    b = O.panorama_normals(g, c["kf_b"])
    ca = np.full((g.rows, g.cols), 2, np.uint16)
    cb = np.full((g.rows, g.cols), 3, np.uint16)
    r1 = O.keyframe_consistency(g, a, ca, g, b, cb, c["T_ba"])
    r2 = O.keyframe_consistency(g, b, cb, g, a, ca, np.linalg.inv(c["T_ba"]))
    assert np.array_equal(r1[4], r2[5]) and np.array_equal(r1[5], r2[4])
    assert np.array_equal(r1[1][r1[4]], np.zeros(r1[4].sum())) and np.all(r1[1][~r1[4]] == 2)
