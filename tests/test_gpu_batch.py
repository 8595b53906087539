"""Batched registrations (many uneven panoramas per launch) against the FP64
oracle, registration by registration, and against the single-registration
path of the same library.

Inputs follow the batch workload: pairs of rendered panoramas of the box room
or the outdoor scene, sizes drawn from {64x512, 64x1024, 128x1024, 128x2048},
motions up to 10 deg / 1 m, 3 pyramid levels with up to 10/10/10 iterations
and an early exit when the update norm falls below 1e-6.
"""
import numpy as np
import pytest

import oracle as O
import synth
from synth import workloads as W
from parity_checks import assert_quality_close, pose_displacement_bound, quality_mismatches

pytestmark = pytest.mark.gpu

BATCH_PARAMS = dict(levels=3, iters=(10, 10, 10), stop_update_norm=1e-6)


def assert_status_matches(res, ref, stop_norm):
    """Equal statuses, except where the stop criterion decided them at its
    threshold: a level that needs its last allowed iteration to bring the
    update norm below stop_norm converges on one side (CONVERGED) and runs out
    of iterations on the other (MAX_ITERS), FP32 against FP64 sums; then the
    side that did not converge ended with an update norm within 10 x the
    threshold."""
    if res["status"] == ref["status"]:
        return
    pair = {res["status"], ref["status"]}
    assert pair == {0, 1}, (res["status"], ref["status"])
    unconverged = res if res["status"] == 1 else ref
    assert unconverged["last_update_norm"] < 10 * stop_norm, unconverged["last_update_norm"]


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def pairs():
    # small sizes first so the oracle stays fast; two of each kind
    sizes = [(64, 512), (64, 1024), (64, 512), (128, 1024), (64, 1024), (64, 512)]
    return [W.batch_pair(k, size=sz, max_angle=np.radians(6), max_trans=0.5) for k, sz in enumerate(sizes)]


@pytest.fixture(scope="module")
def bctx(gpu_lib):
    c = gpu_lib.Context(0, max_pixels=128 * 2048, max_batch=512, max_batch_pixels=300 * 128 * 2048)
    yield c
    c.close()


def _items_from_depth(gpu_lib, pairs):
    import torch
    items = []
    for p in pairs:
        g = p["geom"]
        items.append(dict(scan_geom=g, kf_geom=g, scan_depth=_t(p["scan"]), kf_depth=_t(p["kf"]),
                          scan_surfel=torch.empty((g.rows, g.cols, 4), dtype=torch.float32, device="cuda"),
                          kf_surfel=torch.empty((g.rows, g.cols, 4), dtype=torch.float32, device="cuda")))
    return items


def test_batch_normals_equal_single(gpu_lib, bctx, pairs):
    items = _items_from_depth(gpu_lib, pairs)
    b = gpu_lib.Batch(bctx, items, gpu_lib.IcpParams(**BATCH_PARAMS))
    b.normals()
    for it in items:
        g = it["scan_geom"]
        single = gpu_lib.panorama_normals(bctx, g, it["scan_depth"])
        assert np.array_equal(_np(single), _np(it["scan_surfel"]))
        single = gpu_lib.panorama_normals(bctx, g, it["kf_depth"])
        assert np.array_equal(_np(single), _np(it["kf_surfel"]))
    b.close()


def test_batch_normals_scans_only(gpu_lib, bctx, pairs):
    """Items without keyframe depth: only the scans' surfels are written, the
    resident keyframe surfel images are left as they were."""
    import torch
    items = _items_from_depth(gpu_lib, pairs[:4])
    for it in items:
        del it["kf_depth"]
        it["kf_surfel"].fill_(7.0)
    b = gpu_lib.Batch(bctx, items, gpu_lib.IcpParams(**BATCH_PARAMS))
    b.normals()
    for it in items:
        single = gpu_lib.panorama_normals(bctx, it["scan_geom"], it["scan_depth"])
        assert np.array_equal(_np(single), _np(it["scan_surfel"]))
        assert bool((it["kf_surfel"] == 7.0).all())
    b.close()


@pytest.mark.parametrize("persistent", [False, True], ids=["launches", "persistent"])
def test_batch_matches_oracle_per_registration(gpu_lib, bctx, pairs, persistent):
    import torch
    items, surf = [], []
    for p in pairs:
        g = p["geom"]
        kf = O.panorama_normals(g, p["kf"]).astype(np.float32)
        scan = O.panorama_normals(g, p["scan"]).astype(np.float32)
        surf.append((kf, scan))
        items.append(dict(scan_geom=g, kf_geom=g, scan_surfel=_t(scan), kf_surfel=_t(kf)))
    b = gpu_lib.Batch(bctx, items, gpu_lib.IcpParams(**BATCH_PARAMS))
    b.set_scheduler(persistent)
    res = gpu_lib.read_results(b.register([np.eye(4)] * len(items)))
    for k, (p, (kf, scan)) in enumerate(zip(pairs, surf)):
        g = p["geom"]
        ref = O.register(g, scan, g, kf, np.eye(4), O.IcpParams(**BATCH_PARAMS))
        rot, tr = synth.pose_error(res[k]["T"], ref["T"])
        print(f"pair {k} {g.rows}x{g.cols} {p['kind']}: GPU vs oracle {rot:.2e} rad {tr:.2e} m, "
              f"iters {res[k]['iters_run']} / {ref['iters_run']}, status {res[k]['status']} / {ref['status']}")
        assert rot < 1e-5 and tr < 1e-5, (k, rot, tr)
        assert_status_matches(res[k], ref, BATCH_PARAMS["stop_update_norm"])
        assert abs(res[k]["iters_run"] - ref["iters_run"]) <= 2
        assert sum(res[k]["level_iters"]) == res[k]["iters_run"]
        assert abs(res[k]["inliers"] - ref["inliers"]) <= 2e-3 * ref["valid"]
        # and the registration found the true motion
        rot_gt, tr_gt = synth.pose_error(res[k]["T"], p["T_gt"])
        assert rot_gt < 2e-3 and tr_gt < 2e-2, (k, rot_gt, tr_gt)
    b.close()


def test_batch_equals_single_registration(gpu_lib, bctx, pairs):
    """Batch and single launches differ only in pixels per thread (hence the
    order of FP32 sums): poses agree far inside the oracle tolerance."""
    items = []
    for p in pairs[:3]:
        g = p["geom"]
        items.append(dict(scan_geom=g, kf_geom=g,
                          scan_surfel=gpu_lib.panorama_normals(bctx, g, _t(p["scan"])),
                          kf_surfel=gpu_lib.panorama_normals(bctx, g, _t(p["kf"]))))
    params = gpu_lib.IcpParams(**BATCH_PARAMS)
    b = gpu_lib.Batch(bctx, items, params)
    res = gpu_lib.read_results(b.register([np.eye(4)] * len(items)))
    for k, it in enumerate(items):
        g = it["scan_geom"]
        r1 = gpu_lib.read_result(gpu_lib.register_scan(bctx, g, it["scan_surfel"], g, it["kf_surfel"], np.eye(4),
                                                       params))
        rot, tr = synth.pose_error(res[k]["T"], r1["T"])
        assert rot < 1e-6 and tr < 1e-6, (k, rot, tr)
        assert res[k]["status"] == r1["status"]
    b.close()


@pytest.mark.parametrize("persistent", [False, True], ids=["launches", "persistent"])
def test_batch_graph_replays_match_eager(gpu_lib, bctx, pairs, persistent):
    """The whole batched call captured in a HIP graph: each of several
    replays, with eager work in between, reproduces the eager result bitwise."""
    import torch
    items = _items_from_depth(gpu_lib, pairs[:4])
    b = gpu_lib.Batch(bctx, items, gpu_lib.IcpParams(**BATCH_PARAMS))
    b.set_scheduler(persistent)
    init = torch.stack([gpu_lib.pose_tensor(np.eye(4)) for _ in items])
    results = torch.zeros((len(items), gpu_lib.RESULT_BYTES), dtype=torch.uint8, device="cuda")
    b.normals()
    b.register(init, results)
    torch.cuda.synchronize()
    eager = _np(results).copy()
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        b.normals()
        b.register(init, results)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            b.normals()
            b.register(init, results)
    for rep in range(3):
        results.zero_()
        # unrelated eager work between replays
        gpu_lib.panorama_normals(bctx, items[0]["scan_geom"], items[0]["scan_depth"])
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(_np(results), eager), rep
    b.close()


@pytest.mark.parametrize("persistent", [False, True], ids=["launches", "persistent"])
def test_batch_failures_isolated(gpu_lib, bctx, pairs, persistent):
    """An empty registration (no returns) stops with NO_INLIERS without
    disturbing its neighbours in the batch."""
    import torch
    items = _items_from_depth(gpu_lib, pairs[:3])
    g = items[1]["scan_geom"]
    items[1]["scan_depth"] = torch.zeros((g.rows, g.cols), dtype=torch.float32, device="cuda")
    b = gpu_lib.Batch(bctx, items, gpu_lib.IcpParams(**BATCH_PARAMS))
    b.set_scheduler(persistent)
    b.normals()
    res = gpu_lib.read_results(b.register([np.eye(4)] * 3))
    assert res[1]["status"] == 3 and res[1]["iters_run"] == 0
    for k in (0, 2):
        assert res[k]["status"] in (0, 1)  # converged, or the 1e-6 criterion not met in 10 iterations
        assert sum(res[k]["level_iters"]) == res[k]["iters_run"] > 0
        rot, tr = synth.pose_error(res[k]["T"], pairs[k]["T_gt"])
        assert rot < 2e-3 and tr < 2e-2
    b.close()


@pytest.mark.parametrize("persistent", [False, True], ids=["launches", "persistent"])
def test_fallback_reruns_only_poor_starts(gpu_lib, bctx, pairs, persistent):
    """Registrations started 60 deg away end with a low inlier ratio and are
    rerun from the identity; the fallback's result replaces theirs (status
    FALLBACK_USED) and matches a plain identity-started registration, while
    the others keep their results bit for bit.  Under the launch scheduler the
    rerun subset is tiled with fewer pixels per thread than the whole batch
    (more, shorter tiles for a few registrations): the same registration with
    its sums partitioned differently, so the match is to rounding (pose within
    1e-6, inliers within 2, truncated cost within those 2 pixels' tau^2);
    under the persistent scheduler the subset keeps the batch's tiling and
    matches bit for bit."""
    import torch
    items = _items_from_depth(gpu_lib, pairs[:4])
    b = gpu_lib.Batch(bctx, items, gpu_lib.IcpParams(**BATCH_PARAMS))
    b.set_scheduler(persistent)
    b.normals()
    plain = _np(b.register([np.eye(4)] * 4)).copy()
    bad = synth.se3(synth.rot_z(np.radians(60.0)), [1.5, -1.0, 0.0])
    init = [bad, np.eye(4), bad, np.eye(4)]
    res = b.register(init)
    torch.cuda.synchronize()
    first = gpu_lib.read_results(res)
    before = _np(res).copy()
    b.fallback(res, 0.5)
    torch.cuda.synchronize()
    after = gpu_lib.read_results(res)
    ref = gpu_lib.read_results(torch.from_numpy(plain))
    for k in (0, 2):
        assert first[k]["inlier_ratio"] < 0.5
        assert after[k]["status"] == gpu_lib.STATUS_FALLBACK_USED
        if persistent:
            assert np.array_equal(after[k]["T"], ref[k]["T"])
            assert after[k]["trunc_cost"] == ref[k]["trunc_cost"]
        else:
            rot, tr = synth.pose_error(after[k]["T"], ref[k]["T"])
            print(f"\nfallback {k} vs plain: {rot:.2e} rad {tr:.2e} m, inliers {after[k]['inliers']} vs {ref[k]['inliers']}")
            assert rot < 1e-6 and tr < 1e-6
            assert abs(after[k]["inliers"] - ref[k]["inliers"]) <= 2
            tau2 = 0.5 ** 2  # level-0 d_max of the parameters
            assert abs(after[k]["trunc_cost"] - ref[k]["trunc_cost"]) <= 2 * tau2 + 1e-6 * ref[k]["trunc_cost"]
    for k in (1, 3):
        assert first[k]["inlier_ratio"] >= 0.5
        assert np.array_equal(_np(res)[k], before[k])
    b.close()


def test_autotune_roundtrip(gpu_lib, bctx, tmp_path):
    path = str(tmp_path / "tune.json")
    gpu_lib.autotune(bctx, path)
    txt = open(path).read()
    assert '"arch": "gfx950' in txt and '"k": ' in txt
    # a second context loads the cache instead of measuring
    c2 = gpu_lib.Context(0, max_pixels=1 << 16, max_batch=4, max_batch_pixels=1 << 20)
    gpu_lib.autotune(c2, path)
    c2.close()


@pytest.mark.gpu
def test_benchmark_batch_sampled_against_oracle(gpu_lib, bctx):
    """The benchmark's own batch (the 256 pairs of the batch workload, its
    parameters and its autotuned pixels per thread: the launch configuration
    it times), with one registration of every size and scene kind compared
    with the oracle.  The sampled pairs get oracle surfels on both sides (the
    oracle's inputs never come from the GPU); the others GPU surfels, which
    only fill the launches.  The iteration at which a level stops (update
    norm below 1e-6) is not unique across FP32 and FP64 near the threshold,
    so the counts are only checked for validity; the pose, the status and the
    inlier count are compared."""
    import os
    import torch
    pairs = W.batch(256)
    sample = {}
    for k, p in enumerate(pairs):
        sample.setdefault((p["geom"].rows, p["geom"].cols, p["kind"]), k)
    assert len(sample) == 8  # 4 sizes x 2 scene kinds
    tune = os.path.join(os.path.dirname(gpu_lib.__file__), "autotune_gfx950.json")
    gpu_lib.autotune(bctx, tune)
    dev = torch.device("cuda:0")
    items, ref_in = [], {}
    for k, p in enumerate(pairs):
        g = p["geom"]
        if k in sample.values():
            kf = O.panorama_normals(g, p["kf"]).astype(np.float32)
            scan = O.panorama_normals(g, p["scan"]).astype(np.float32)
            ref_in[k] = (kf, scan)
            items.append(dict(scan_geom=g, kf_geom=g, scan_surfel=_t(scan), kf_surfel=_t(kf)))
        else:
            items.append(dict(scan_geom=g, kf_geom=g,
                              scan_surfel=gpu_lib.panorama_normals(bctx, g, torch.from_numpy(p["scan"]).to(dev)),
                              kf_surfel=gpu_lib.panorama_normals(bctx, g, torch.from_numpy(p["kf"]).to(dev))))
    b = gpu_lib.Batch(bctx, items, gpu_lib.IcpParams(**BATCH_PARAMS))
    res = gpu_lib.read_results(b.register([np.eye(4)] * len(items)))
    b.close()
    for (rows, cols, kind), k in sorted(sample.items()):
        g = pairs[k]["geom"]
        kf, scan = ref_in[k]
        ref = O.register(g, scan, g, kf, np.eye(4), O.IcpParams(**BATCH_PARAMS))
        rot, tr = synth.pose_error(res[k]["T"], ref["T"])
        print(f"pair {k} {rows}x{cols} {kind}: GPU vs oracle {rot:.2e} rad {tr:.2e} m, "
              f"iters {res[k]['iters_run']} / {ref['iters_run']}, status {res[k]['status']} / {ref['status']}",
              flush=True)
        assert rot < 1e-5 and tr < 1e-5, (k, rot, tr)
        assert_status_matches(res[k], ref, BATCH_PARAMS["stop_update_norm"])
        assert 1 <= res[k]["iters_run"] <= 30 and sum(res[k]["level_iters"]) == res[k]["iters_run"]
        assert abs(res[k]["inliers"] - ref["inliers"]) <= 2e-3 * ref["valid"]
        # the quality block (inlier ratio, rms, truncated cost) at the two final poses
        mism = quality_mismatches(gpu_lib, bctx, g, scan, kf, res[k]["T"], ref["T"])
        rr = O.residuals(g, scan, g, kf, ref["T"])
        dr = pose_displacement_bound(res[k]["T"], ref["T"], float(scan[..., 3].max()))
        print(f"   truncated cost {res[k]['trunc_cost']:.6f} / {ref['trunc_cost']:.6f}, mismatches {mism}", flush=True)
        assert_quality_close(res[k], ref, mism, 0.5, dr, float(np.abs(rr["r"][rr["inlier"]]).sum()))


def test_pyramids_built_by_normals_give_the_same_results(gpu_lib, bctx, pairs):
    """UPS_PYR_IN_NORMALS: the normals' last pass writes the pyramids of the
    images it computes (every scan, the keyframes with depth), and register
    and grid search build only those of the keyframes given as surfels.
    Results bitwise those of the default mode (both batches alive at once, so
    the second's pyramid memory is fresh), also from a captured graph
    replayed three times, and grid-search scores equal."""
    import torch
    items = _items_from_depth(gpu_lib, pairs)
    # every other keyframe resident (surfels only): its pyramid comes from the side stream
    for k, it in enumerate(items):
        gpu_lib.panorama_normals(bctx, it["kf_geom"], it["kf_depth"], it["kf_surfel"])
    items2 = [dict(it) for it in items]
    for k, it in enumerate(items2):
        it["scan_surfel"] = torch.empty_like(it["scan_surfel"])
        if k % 2:
            it.pop("kf_depth")
        else:
            it["kf_surfel"] = torch.empty_like(it["kf_surfel"])
    params = gpu_lib.IcpParams(**BATCH_PARAMS)
    ref_b = gpu_lib.Batch(bctx, items, params)
    b = gpu_lib.Batch(bctx, items2, params)
    b.set_pyramid_mode(True)
    n = len(items)
    init = torch.stack([gpu_lib.pose_tensor(np.eye(4)) for _ in items])
    ref_b.normals()
    ref = _np(ref_b.register(init)).copy()
    def grid(batch):
        _, _, scores = batch.grid_search(base=init)
        torch.cuda.synchronize()
        return _np(scores)
    ref_scores = grid(ref_b)
    b.normals()
    got = _np(b.register(init))
    assert np.array_equal(got, ref)
    assert np.array_equal(grid(b), ref_scores)
    # captured: normals (writing the pyramids) and register
    res = torch.zeros_like(torch.from_numpy(ref)).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.normals()
        b.register(init, res)
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr, stream=s):
        b.normals()
        b.register(init, res)
    for rep in range(3):
        res.zero_()
        for it in items2:
            it["scan_surfel"].zero_()
        torch.cuda.synchronize()
        print(f"replay {rep}", flush=True)
        with torch.cuda.stream(s):
            gr.replay()
        torch.cuda.synchronize()
        assert np.array_equal(_np(res), ref), rep
    # the persistent scheduler reads the same pyramids
    for batch in (ref_b, b):
        batch.set_scheduler(True)
    ref_p = _np(ref_b.register(init)).copy()
    b.normals()
    assert np.array_equal(_np(b.register(init)), ref_p)
    b.close()
    ref_b.close()
