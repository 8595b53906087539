"""The keyframe map end to end on the GPU (Section III-C): a closed loop of
sweeps through the outdoor scene, 1.25 laps of a 10 m circle.  Sweeps are
fused while their quality stays above the threshold, new keyframes appear as
the sensor moves on, and on the second lap the map returns to its first
keyframe by a strong loop closure instead of creating new ones.  Poses stay
close to the rendered truth."""
import numpy as np
import pytest

import synth
from synth import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def seq():
    return W.loop_sequence(n_scans=64, radius=10.0)


def test_loop_sequence_switches_back_to_first_keyframe(gpu_lib, seq):
    from paper_2101_00585_amd.keyframes import GpuBackend, KeyframeMap, MapParams
    g = seq["geom"]
    ctx = gpu_lib.Context(0, max_pixels=g.rows * g.cols, max_batch=16, max_batch_pixels=16 * g.rows * g.cols)
    try:
        m = KeyframeMap(GpuBackend(ctx, g), MapParams(new_keyframe_ratio=0.75, search_radius=8.0))
        P0 = seq["T_world"][0]
        steps, errs = [], []
        for k, depth in enumerate(seq["scans"]):
            s = m.add_sweep(depth)
            truth = np.linalg.inv(P0) @ seq["T_world"][k]
            rot, tr = synth.pose_error(s.T_world, truth)
            steps.append(s)
            errs.append((rot, tr))
            print(f"sweep {k:2d}: {s.event:12s} kf {s.keyframe:2d} ratio {s.ratio:.3f} err {np.degrees(rot):.3f} deg "
                  f"{tr:.3f} m closures {s.closures} removed {s.removed}")
        n_kf = len(m.keyframes)
        lap = int(len(seq["scans"]) / 1.25)
        back = [k for k, s in enumerate(steps) if s.event == "switched" and s.keyframe == 0]
        print(f"keyframes {n_kf}, switches back to keyframe 0 at sweeps {back}, edges "
              f"{[(e.a, e.b, e.kind) for e in m.edges]}")
        assert n_kf >= 3
        assert any(k >= lap - 4 for k in back)
        # no keyframe is created once the loop has closed onto keyframe 0
        first_back = min(k for k in back if k >= lap - 4)
        assert all(s.event != "new_keyframe" for s in steps[first_back:first_back + 4])
        errs = np.array(errs)
        assert np.degrees(errs[:, 0]).max() < 1.0 and errs[:, 1].max() < 0.3, errs.max(axis=0)
    finally:
        ctx.close()
