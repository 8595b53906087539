"""Loop-closure grid search (Section III-C): candidate transforms scored by
the number of Omega inliers at a coarse pyramid level, the best one promoted
to the full-resolution batched registration.

Scores are compared with the FP64 oracle's inlier counts at the same
candidate poses on identical inputs (the oracle's surfel images, rounded to
FP32, on both sides): each integer score within the number of pixels whose
FP64 projection or gate value lies at a boundary, the winner the oracle's
wherever its margin exceeds that; the promoted registrations are compared
with identity-started ones on pairs with relative yaw up to 90 deg."""
import math

import numpy as np
import pytest

import oracle as O
import synth
from parity_checks import association_ambiguous, assert_scores_match
from synth import workloads as W

pytestmark = pytest.mark.gpu

BATCH_PARAMS = dict(levels=3, iters=(10, 10, 10), stop_update_norm=1e-6)


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _candidate(c, n_yaw, n_xy, step):
    """G_c written out from its definition (FP64, 4x4)."""
    a, u, v = c // (n_xy * n_xy), (c // n_xy) % n_xy, c % n_xy
    h = (n_xy - 1) / 2
    return synth.se3(synth.rot_z(2 * math.pi * a / n_yaw), [(u - h) * step, (v - h) * step, 0.0])


def _oracle_items(pairs):
    """Items carrying the oracle's level-0 surfel images (FP32) of each pair;
    returns the items and, per pair, the level-2 images of both (FP64 copies
    of the same FP32 values)."""
    items, lvl2 = [], []
    for p in pairs:
        g = p["geom"]
        s32 = O.panorama_normals(g, p["scan"]).astype(np.float32)
        k32 = O.panorama_normals(g, p["kf"]).astype(np.float32)
        items.append(dict(scan_geom=g, kf_geom=g, scan_surfel=_t(s32), kf_surfel=_t(k32)))
        lvl2.append((O.pyramid_level(g, s32.astype(np.float64), 2), O.pyramid_level(g, k32.astype(np.float64), 2)))
    return items, lvl2


def _check_scores(g, sl, kl, scores_k, poses, d_max):
    gl = g.level(2)
    cos_t = math.cos(math.radians(30.0))
    ref = np.array([int(O.correspondences(gl, sl, gl, kl, T, d_max, cos_t)[1].sum()) for T in poses])
    amb = np.array([int(association_ambiguous(gl, sl, gl, kl, T, d_max, cos_t).sum()) for T in poses])
    return assert_scores_match(scores_k, ref, amb)


def _items(pairs):
    import torch
    items = []
    for p in pairs:
        g = p["geom"]
        items.append(dict(scan_geom=g, kf_geom=g, scan_depth=_t(p["scan"]), kf_depth=_t(p["kf"]),
                          scan_surfel=torch.empty((g.rows, g.cols, 4), dtype=torch.float32, device="cuda"),
                          kf_surfel=torch.empty((g.rows, g.cols, 4), dtype=torch.float32, device="cuda")))
    return items


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0, max_pixels=128 * 2048, max_batch=64, max_batch_pixels=64 * 128 * 2048)
    yield c
    c.close()


# (n_yaw, n_xy): the per-yaw kernels (1 to 5 grid cells per axis, yaw chunks
# that do not divide n_yaw included) and the general kernel (6 cells per axis)
@pytest.mark.parametrize("n_yaw,n_xy", [(12, 3), (7, 1), (5, 2), (3, 4), (2, 5), (2, 6)])
def test_scores_match_oracle_counts(gpu_lib, ctx, n_yaw, n_xy):
    pairs = [W.batch_pair(k, base_seed=5_000_000, max_angle=math.radians(90.0), size=(64, 512)) for k in range(2)]
    gp = gpu_lib.GridParams(level=2, n_yaw=n_yaw, n_xy=n_xy, xy_step=0.7, d_max=2.0)
    items, lvl2 = _oracle_items(pairs)
    b = gpu_lib.Batch(ctx, items, gpu_lib.IcpParams(**BATCH_PARAMS))
    best, best_score, scores = b.grid_search(gp)
    scores = scores.cpu().numpy()
    best = best.cpu().numpy()
    best_score = best_score.cpu().numpy()
    C = n_yaw * n_xy * n_xy
    assert scores.shape == (len(pairs), C)
    for k, p in enumerate(pairs):
        sl, kl = lvl2[k]
        dev, amb = _check_scores(p["geom"], sl, kl, scores[k], [_candidate(c, n_yaw, n_xy, 0.7) for c in range(C)],
                                 2.0)
        print(f"pair {k}: {C} candidates, total |score - oracle| {dev}, ambiguous pixels {amb}")
        c_best = int(np.argmax(scores[k]))
        assert best_score[k] == scores[k].max() and np.argmax(scores[k] == scores[k].max()) == c_best
        T = np.eye(4)
        T[:3, :3] = best[k, :9].reshape(3, 3)
        T[:3, 3] = best[k, 9:]
        np.testing.assert_allclose(T, _candidate(c_best, n_yaw, n_xy, 0.7), atol=1e-12)
    b.close()


def test_grid_start_beats_identity_at_large_yaw(gpu_lib, ctx):
    import torch
    n = 32
    pairs = [W.batch_pair(k, base_seed=5_100_000, max_angle=math.radians(90.0), max_trans=2.0) for k in range(n)]
    items = _items(pairs)
    b = gpu_lib.Batch(ctx, items, gpu_lib.IcpParams(**BATCH_PARAMS))
    b.normals()
    plain = gpu_lib.read_results(b.register([np.eye(4)] * n))
    best, _, _ = b.grid_search(gpu_lib.GridParams())
    grid = gpu_lib.read_results(b.register(best))
    torch.cuda.synchronize()

    def ok(res):
        return np.array([synth.pose_error(r["T"], p["T_gt"])[0] < math.radians(1.0)
                         and synth.pose_error(r["T"], p["T_gt"])[1] < 0.05 for r, p in zip(res, pairs)])

    s_plain, s_grid = ok(plain), ok(grid)
    print(f"\ngrid search: success identity start {s_plain.sum()}/{n}, grid start {s_grid.sum()}/{n}")
    assert s_grid.sum() >= s_plain.sum() + 0.1 * n
    assert s_grid.mean() >= 0.8
    b.close()


def test_grid_search_replays_from_a_graph(gpu_lib, ctx):
    import torch
    pairs = [W.batch_pair(k, base_seed=5_200_000, max_angle=math.radians(60.0), size=(64, 512)) for k in range(4)]
    items = _items(pairs)
    b = gpu_lib.Batch(ctx, items, gpu_lib.IcpParams(**BATCH_PARAMS))
    gp = gpu_lib.GridParams(n_yaw=18)
    base = torch.stack([gpu_lib.pose_tensor(np.eye(4)) for _ in items])
    scores = torch.empty((4, 18 * 9), dtype=torch.int32, device="cuda")
    best = torch.empty((4, 12), dtype=torch.float64, device="cuda")
    bsc = torch.empty(4, dtype=torch.int32, device="cuda")
    b.normals()
    b.grid_search(gp, base, scores, best, bsc)
    torch.cuda.synchronize()
    eager = (scores.cpu().numpy().copy(), best.cpu().numpy().copy())
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        b.grid_search(gp, base, scores, best, bsc)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            b.grid_search(gp, base, scores, best, bsc)
    for _ in range(2):
        scores.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(scores.cpu().numpy(), eager[0]) and np.array_equal(best.cpu().numpy(), eager[1])
    b.close()


def test_scores_around_a_base_pose(gpu_lib, ctx):
    """The candidates are base * G_c: scores against the oracle's counts at
    base * G_c for a base pose per registration."""
    import torch
    pairs = [W.batch_pair(k, base_seed=5_100_000, max_angle=math.radians(40.0), size=(64, 512)) for k in range(2)]
    bases = [synth.se3(synth.rot_z(0.3 + k), [0.5, -0.2 * k, 0.05]) for k in range(2)]
    gp = gpu_lib.GridParams(level=2, n_yaw=4, n_xy=3, xy_step=0.5, d_max=2.0)
    items, lvl2 = _oracle_items(pairs)
    b = gpu_lib.Batch(ctx, items, gpu_lib.IcpParams(**BATCH_PARAMS))
    base_t = torch.stack([gpu_lib.pose_tensor(T) for T in bases])
    best, _, scores = b.grid_search(gp, base_t)
    scores = scores.cpu().numpy()
    for k, p in enumerate(pairs):
        sl, kl = lvl2[k]
        _check_scores(p["geom"], sl, kl, scores[k], [bases[k] @ _candidate(c, 4, 3, 0.5) for c in range(36)], 2.0)
        c_best = int(np.argmax(scores[k]))
        T = np.eye(4)
        T[:3, :3] = best.cpu().numpy()[k, :9].reshape(3, 3)
        T[:3, 3] = best.cpu().numpy()[k, 9:]
        np.testing.assert_allclose(T, bases[k] @ _candidate(c_best, 4, 3, 0.5), atol=1e-12)
    b.close()
