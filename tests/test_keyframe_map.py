"""Host logic of the keyframe map (Section III-C) with a scripted backend
(no GPU): when a sweep is fused, when a new keyframe is created, when a
strong loop closure switches the current keyframe, which edges the pose graph
records, which poses the moving-object check receives, and the two motion
priors."""
import math

import numpy as np

from paper_2101_00585_amd.keyframes import (EDGE_ODOMETRY, EDGE_STRONG, EDGE_WEAK, MOTION_ZERO_ACCELERATION,
                                            KeyframeMap, MapParams, rigid_inv)
from synth import rot_z, se3


class Scripted:
    """Registration results come from a script: ratio per sweep (odometry)
    and (ratio, class) per candidate for loop-closure searches."""

    def __init__(self, odo, loops=()):
        self.odo = list(odo)
        self.loops = list(loops)
        self.calls = []

    def normals(self, depth):
        return depth

    def new_keyframe(self, scan):
        return {"scan": scan}

    def register(self, scan, kf, init):
        self.calls.append(("register", np.array(init)))
        ratio, T = self.odo.pop(0)
        return dict(T=T, inlier_ratio=ratio, status=0)

    def fuse(self, scan, kf, T):
        self.calls.append(("fuse", np.array(T)))

    def loop_closure(self, scan, kfs, inits, threshold):
        out = self.loops.pop(0)
        self.calls.append(("loop", len(kfs), [np.array(T) for T in inits]))
        results = [dict(T=T, inlier_ratio=q, status=0) for (q, _, T) in out]
        classes = np.array([c for (_, c, _) in out])
        strong = [k for k, (q, c, _) in enumerate(out) if c == 2]
        best = max(strong, key=lambda k: (out[k][0], -k)) if strong else -1
        return results, classes, best

    def consistency(self, a, b, T_ba):
        self.calls.append(("consistency", np.array(T_ba)))
        return (3, 4)


def _step(x, yaw=0.0):
    return se3(rot_z(yaw), [x, 0.0, 0.0])


def test_fuse_then_new_keyframe_with_odometry_edge():
    T1, T2, T3 = _step(1.0), _step(2.0), _step(3.0, 0.1)
    be = Scripted([(0.9, T1), (0.8, T2), (0.5, T3)])
    m = KeyframeMap(be, MapParams(new_keyframe_ratio=0.7, search_radius=1.0))
    assert m.add_sweep("s0").event == "new_keyframe"
    s1 = m.add_sweep("s1")
    assert s1.event == "fused" and np.allclose(s1.T_world, T1)
    assert m.add_sweep("s2").event == "fused"
    s3 = m.add_sweep("s3")  # ratio 0.5 < 0.7, keyframe 0 is the current one: no candidates
    assert s3.event == "new_keyframe" and s3.keyframe == 1 and s3.removed == (3, 4)
    assert np.allclose(m.keyframes[1].T_world, T3)
    e = m.edges[-1]
    assert (e.a, e.b, e.kind) == (0, 1, EDGE_ODOMETRY) and np.allclose(e.T_ab, T3)
    # the moving-object check maps keyframe 0's frame into the new keyframe's
    cons = [c for c in be.calls if c[0] == "consistency"][-1]
    assert np.allclose(cons[1], rigid_inv(T3))
    # zero-velocity prior: each registration starts from the previous pose
    inits = [c[1] for c in be.calls if c[0] == "register"]
    assert np.allclose(inits[0], np.eye(4)) and np.allclose(inits[1], T1) and np.allclose(inits[2], T2)


def test_strong_closure_switches_and_weak_adds_edge():
    far = _step(10.0)
    back = se3(rot_z(math.pi), [10.0, 0.0, 0.0])
    be = Scripted([(0.3, far), (0.3, back)],
                  loops=[[(0.72, 1, _step(0.5)), (0.9, 2, _step(0.2))]])
    m = KeyframeMap(be, MapParams(new_keyframe_ratio=0.7, search_radius=12.0))
    m.add_sweep("s0")
    s = m.add_sweep("s1")        # nothing near but the current keyframe: new keyframe 1 at x = 10
    assert s.event == "new_keyframe" and len(m.keyframes) == 2
    # next sweep: quality drops; keyframe 0 (10 m away) is the only candidate
    m.p.search_radius = 25.0
    be.loops = [[(0.95, 2, _step(0.2))]]
    s = m.add_sweep("s2")
    assert s.event == "switched" and s.keyframe == 0 and m.current == 0
    e = m.edges[-1]
    assert e.kind == EDGE_STRONG and (e.a, e.b) == (1, 0)
    assert np.allclose(e.T_ab, back @ rigid_inv(_step(0.2)))
    # the loop-closure search started from the pose estimate in keyframe 0's frame
    loop = [c for c in be.calls if c[0] == "loop"][-1]
    assert loop[1] == 1 and np.allclose(loop[2][0], rigid_inv(np.eye(4)) @ (m.keyframes[1].T_world @ back))
    # the check runs between the old and the new current keyframe
    cons = [c for c in be.calls if c[0] == "consistency"][-1]
    assert np.allclose(cons[1], rigid_inv(e.T_ab))


def test_weak_only_creates_keyframe_and_records_edge():
    be = Scripted([(0.3, _step(5.0)), (0.3, _step(1.0))], loops=[[(0.6, 1, _step(4.0))]])
    m = KeyframeMap(be, MapParams(new_keyframe_ratio=0.7, search_radius=20.0))
    m.add_sweep("s0")
    m.add_sweep("s1")                       # keyframe 1
    s = m.add_sweep("s2")                   # keyframe 0 is a weak closure only
    assert s.event == "new_keyframe" and s.keyframe == 2
    kinds = [(e.a, e.b, e.kind) for e in m.edges]
    assert (1, 0, EDGE_WEAK) in kinds and (1, 2, EDGE_ODOMETRY) in kinds


def test_zero_acceleration_prior_extrapolates():
    T1, T2 = _step(1.0, 0.05), _step(2.1, 0.1)
    be = Scripted([(0.9, T1), (0.9, T2), (0.9, _step(3.0))])
    m = KeyframeMap(be, MapParams(motion_prior=MOTION_ZERO_ACCELERATION))
    for k in range(4):
        m.add_sweep(f"s{k}")
    inits = [c[1] for c in be.calls if c[0] == "register"]
    assert np.allclose(inits[0], np.eye(4))                       # sweep 0 is the keyframe itself
    assert np.allclose(inits[1], T1 @ T1)                         # I, T1 known: T1 (I^-1 T1)
    assert np.allclose(inits[2], T2 @ rigid_inv(T1) @ T2)          # T2 (T1^-1 T2)
