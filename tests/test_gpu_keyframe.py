"""Keyframe management on the GPU against the oracle, through the C ABI:
the moving-object check between two keyframes and the loop-closure classes
(Section III-C).

Masks: closed-form cases (T = I, a pixel maps onto itself) must be
bit-exact; on rendered keyframe pairs FP32 projection and range comparisons
may flip a decision where the FP64 values sit on a pixel boundary or at the
margin, so mismatches are counted and bounded (at most 0.05 % of the
pixels).  Removal is exact: marked samples become zero with count 0, all
others keep their bits."""
import math

import numpy as np
import pytest

import oracle as O
from synth import lidar_geom, rot_z, se3
from synth import workloads as W

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0, max_pixels=128 * 2048)
    yield c
    c.close()


def _surf(r):
    s = np.zeros(r.shape + (4,), np.float32)
    s[..., 2] = 1.0
    s[..., 3] = r
    return s


def test_closed_form_masks_bit_exact(gpu_lib, ctx):
    import torch
    g = lidar_geom(16, 64)
    a = np.full((16, 64), 10.0)
    a[4:9, 10:20] = 5.0
    a[4:9, 30:40] = 9.85
    a[4:9, 44:50] = 9.7
    a[0, 55:60] = 5.0
    a[15, 55:60] = 5.0
    a[10:14, 20:30] = 40.0
    a[11:13, 22:25] = 39.5
    a[11:13, 25:28] = 39.0
    a[6, 63] = 5.0
    b = np.full((16, 64), 10.0)
    b[10:14, 20:30] = 40.0
    cnt_b = np.full((16, 64), 3, np.uint16)
    cnt_b[5, 39] = 1
    sa, sb = _surf(a), _surf(b)
    p = gpu_lib.ConsistencyParams(min_count=2)
    ref = O.free_space_violations(g, sa, g, sb, cnt_b, np.eye(4), O.ConsistencyParams(min_count=2))
    A, B = _t(sa), _t(sb)
    CB = _t(cnt_b.view(np.int16))
    ma, mb, removed = gpu_lib.keyframe_consistency(ctx, g, A, None, g, B, CB, np.eye(4), p, mutual=False)
    torch.cuda.synchronize()
    assert mb is None
    assert np.array_equal(_np(ma).astype(bool), ref)
    assert _np(removed)[0] == ref.sum()
    out = _np(A)
    assert np.all(out[ref] == 0) and np.array_equal(out[~ref], sa[~ref])
    assert np.array_equal(_np(B), sb)  # one direction: B untouched


def test_yaw_columns_bit_exact(gpu_lib, ctx):
    g = lidar_geom(16, 64)
    k = 5
    a = np.full((16, 64), 10.0)
    a[6:9, 10:14] = 4.0
    b = np.full((16, 64), 10.0)
    b[6:9, 10 - k:14 - k] = 4.0
    for T, expect_any in ((se3(rot_z(-2 * math.pi * k / 64)), False), (se3(rot_z(2 * math.pi * k / 64)), True)):
        ref = O.free_space_violations(g, _surf(a), g, _surf(b), None, T)
        ma, _, _ = gpu_lib.keyframe_consistency(ctx, g, _t(_surf(a)), None, g, _t(_surf(b)), None, T, mutual=False)
        assert np.array_equal(_np(ma).astype(bool), ref) and ref.any() == expect_any


@pytest.mark.parametrize("seed,min_count", [(0, 2), (1, 2), (2, 1), (3, 1)])
def test_moving_objects_match_oracle(gpu_lib, ctx, seed, min_count):
    import torch
    c = W.moving_objects_pair(seed)
    g = c["geom"]
    a = O.panorama_normals(g, c["kf_a"]).astype(np.float32)
    b = O.panorama_normals(g, c["kf_b"]).astype(np.float32)
    rng = np.random.default_rng(seed)
    ca = rng.integers(1, 4, size=(g.rows, g.cols)).astype(np.uint16)
    cb = rng.integers(1, 4, size=(g.rows, g.cols)).astype(np.uint16)
    p = O.ConsistencyParams(min_count=min_count)
    ra, rca, rb, rcb, ma_ref, mb_ref = O.keyframe_consistency(g, a, ca, g, b, cb, c["T_ba"], p)
    A, B, CA, CB = _t(a), _t(b), _t(ca.view(np.int16)), _t(cb.view(np.int16))
    ma, mb, removed = gpu_lib.keyframe_consistency(ctx, g, A, CA, g, B, CB, c["T_ba"],
                                                   gpu_lib.ConsistencyParams(min_count=min_count))
    torch.cuda.synchronize()
    ma, mb = _np(ma).astype(bool), _np(mb).astype(bool)
    flips = int((ma != ma_ref).sum() + (mb != mb_ref).sum())
    print(f"seed {seed}: removed A {ma.sum()} (oracle {ma_ref.sum()}), B {mb.sum()} (oracle {mb_ref.sum()}), "
          f"flips {flips}")
    assert flips <= 5e-4 * 2 * g.rows * g.cols
    assert _np(removed).tolist() == [int(ma.sum()), int(mb.sum())]
    # every removal is a mover (as in the oracle), and the removal is exact
    assert not (ma & ~c["mover_a"]).any() and not (mb & ~c["mover_b"]).any()
    oa, ob = _np(A), _np(B)
    assert np.all(oa[ma] == 0) and np.array_equal(oa[~ma], a[~ma])
    assert np.all(ob[mb] == 0) and np.array_equal(ob[~mb], b[~mb])
    oca, ocb = _np(CA).view(np.uint16), _np(CB).view(np.uint16)
    assert np.all(oca[ma] == 0) and np.array_equal(oca[~ma], ca[~ma])
    assert np.all(ocb[mb] == 0) and np.array_equal(ocb[~mb], cb[~mb])


def test_consistency_invalid_args(gpu_lib, ctx):
    g = lidar_geom(16, 64)
    A = _t(_surf(np.full((16, 64), 10.0)))
    with pytest.raises(gpu_lib.UpsError):
        gpu_lib.keyframe_consistency(ctx, g, A, None, g, A, None, np.eye(4))
    with pytest.raises(gpu_lib.UpsError):
        gpu_lib.keyframe_consistency(ctx, g, A, None, g, _t(_surf(np.full((16, 64), 10.0))), None, np.eye(4),
                                     gpu_lib.ConsistencyParams(margin_abs=-1.0))


def _results_with(gpu_lib, ratios, statuses):
    import torch
    buf = np.zeros((len(ratios), gpu_lib.RESULT_BYTES), np.uint8)
    for k, (q, st) in enumerate(zip(ratios, statuses)):
        buf[k, 112:120] = np.frombuffer(np.float64(q).tobytes(), np.uint8)
        buf[k, 140:144] = np.frombuffer(np.int32(st).tobytes(), np.uint8)
    out = torch.from_numpy(buf).cuda()
    got = gpu_lib.read_results(out)
    assert [r["inlier_ratio"] for r in got] == list(ratios) and [r["status"] for r in got] == list(statuses)
    return out


@pytest.mark.parametrize("n", [1, 7, 300, 1000])
def test_loop_closure_classes_match_oracle(gpu_lib, ctx, n):
    rng = np.random.default_rng(n)
    ratios = list(np.round(rng.uniform(0, 1, n), 2))
    ratios[0] = 0.5
    statuses = [int(s) for s in rng.integers(0, 5, n)]
    res = _results_with(gpu_lib, ratios, statuses)
    cls, best = gpu_lib.classify_loop_closures(ctx, res, 0.5)
    ref_cls, ref_best = O.loop_closure_classes(ratios, statuses, 0.5)
    assert np.array_equal(_np(cls), ref_cls)
    assert int(_np(best)[0]) == ref_best


def test_keyframes_of_different_geometries(gpu_lib, ctx):
    """A 64x1024 sweep-sized keyframe checked against a 128x2048 one (wider
    field of view), both directions, against the oracle."""
    import torch
    c = W.moving_objects_pair(2, rows=64, cols=1024)
    gb = lidar_geom(128, 2048)
    import synth
    sc_b = type(c["static"])(room=c["static"].room, boxes=np.vstack([c["static"].boxes, c["movers_b"]]), kind="room")
    kb_depth = synth.render(sc_b, gb, c["T_world_b"], 0.01, 77)
    a = O.panorama_normals(c["geom"], c["kf_a"]).astype(np.float32)
    b = O.panorama_normals(gb, kb_depth).astype(np.float32)
    _, _, _, _, ma_ref, mb_ref = O.keyframe_consistency(c["geom"], a, None, gb, b, None, c["T_ba"])
    ma, mb, removed = gpu_lib.keyframe_consistency(ctx, c["geom"], _t(a), None, gb, _t(b), None, c["T_ba"])
    torch.cuda.synchronize()
    ma, mb = _np(ma).astype(bool), _np(mb).astype(bool)
    flips = int((ma != ma_ref).sum() + (mb != mb_ref).sum())
    print(f"64x1024 vs 128x2048: removed A {ma.sum()} (oracle {ma_ref.sum()}), B {mb.sum()} (oracle {mb_ref.sum()}), "
          f"flips {flips}")
    assert ma_ref.sum() > 0 and mb_ref.sum() > 0
    assert flips <= 5e-4 * (ma.size + mb.size)
