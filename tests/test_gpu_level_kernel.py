"""Failure handling of the one-XCD level kernel (the Gauss-Newton iterations
of Section III-B for a coarse level of a single registration in one launch,
its workgroups waiting for each other between iterations), forced from the
host: with a limit of zero unsuccessful polls, a workgroup that finds the
others not yet arrived gives up, every other one gives up at its next poll,
and the registration ends as DEGENERATE instead of going on from a sum that
lacks a tile.  Every kernel still exits normally.  The next call with the
default limit must give bitwise the result of a call before the failure (the
counters and partials the failed call left behind are not read)."""
import numpy as np
import pytest

import synth
from synth import workloads as W

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0, max_pixels=128 * 1024)
    yield c
    c.close()


@pytest.fixture
def spin_limit(gpu_lib):
    """Set the level kernel's poll limit for the test, restore the default afterwards."""
    yield gpu_lib.debug_level_spin_limit
    gpu_lib.debug_level_spin_limit(-1)


@pytest.mark.parametrize("size", [(128, 1024), (64, 512)], ids=["128x1024", "64x512"])
def test_level_kernel_give_up_ends_degenerate(gpu_lib, ctx, spin_limit, size):
    import torch
    c = W.config0(rows=size[0], cols=size[1])
    g = c["geom"]
    kf = gpu_lib.panorama_normals(ctx, g, _t(c["kf"].astype(np.float32)))
    scan = gpu_lib.panorama_normals(ctx, g, _t(c["scan"].astype(np.float32)))
    p = gpu_lib.IcpParams(levels=3, iters=(10, 10, 10))
    init = synth.se3(synth.rot_z(0.02), [0.1, -0.05, 0.0])
    print(f"\n{size}: reference call", flush=True)
    ref = gpu_lib.register_scan(ctx, g, scan, g, kf, init, p)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy().copy()
    r0 = gpu_lib.read_result(torch.from_numpy(ref))
    assert r0["status"] == gpu_lib.STATUS_CONVERGED and r0["iters_run"] == 30
    print("zero-poll limit", flush=True)
    spin_limit(0)
    bad = gpu_lib.register_scan(ctx, g, scan, g, kf, init, p)
    torch.cuda.synchronize()
    rb = gpu_lib.read_result(bad)
    print(f"gave up: status {rb['status']}, iterations {rb['iters_run']}, per level {rb['level_iters']}")
    assert rb["status"] == gpu_lib.STATUS_DEGENERATE
    # a coarse level gave up: no update at level 0 (it never runs in one launch)
    assert rb["iters_run"] < 30 and rb["level_iters"][0] == 0
    print("default limit again", flush=True)
    spin_limit(-1)
    again = gpu_lib.register_scan(ctx, g, scan, g, kf, init, p)
    torch.cuda.synchronize()
    assert np.array_equal(again.cpu().numpy(), ref)


def test_level_spin_limit_rejects_out_of_range(gpu_lib):
    with pytest.raises(Exception):
        gpu_lib.debug_level_spin_limit(1 << 32)


def test_level_kernels_on_concurrent_streams(gpu_lib):
    """Four registrations, each in its own context, replayed from graphs on
    four streams at once: their one-XCD level kernels run concurrently (on
    different XCDs: the host rotates the XCD that takes the tiles), and each
    result is bitwise the sequential one, three replays in a row."""
    import torch
    n = 4
    ctxs = [gpu_lib.Context(0, max_pixels=128 * 1024) for _ in range(n)]
    try:
        c = W.config0(rows=128, cols=1024)
        g = c["geom"]
        kf = gpu_lib.panorama_normals(ctxs[0], g, _t(c["kf"].astype(np.float32)))
        scan = gpu_lib.panorama_normals(ctxs[0], g, _t(c["scan"].astype(np.float32)))
        p = gpu_lib.IcpParams(levels=3, iters=(10, 10, 10))
        init = synth.se3(synth.rot_z(0.02), [0.1, -0.05, 0.0])
        ref = gpu_lib.register_scan(ctxs[0], g, scan, g, kf, init, p)
        torch.cuda.synchronize()
        ref = ref.cpu().numpy().copy()
        dev = torch.device("cuda:0")
        streams = [torch.cuda.Stream() for _ in range(n)]
        graphs, results, inits = [], [], []
        for k in range(n):
            res = gpu_lib.new_result(dev)
            init_d = gpu_lib.pose_tensor(init, dev)
            with torch.cuda.stream(streams[k]):
                gpu_lib.register_scan(ctxs[k], g, scan, g, kf, init_d, p, res)
            torch.cuda.synchronize()
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr, stream=streams[k]):
                gpu_lib.register_scan(ctxs[k], g, scan, g, kf, init_d, p, res)
            graphs.append(gr)
            results.append(res)
            inits.append(init_d)
        for rep in range(3):
            for r in results:
                r.zero_()
            torch.cuda.synchronize()
            print(f"replay {rep}", flush=True)
            for k in range(n):
                with torch.cuda.stream(streams[k]):
                    graphs[k].replay()
            torch.cuda.synchronize()
            for k in range(n):
                assert np.array_equal(results[k].cpu().numpy(), ref), (rep, k)
    finally:
        torch.cuda.synchronize()
        for cx in ctxs:
            cx.close()


@pytest.mark.parametrize("variant", ["squared", "irls", "world"])
def test_level_kernel_variants_match_oracle(gpu_lib, ctx, variant):
    """The instantiations of the one-XCD level kernel (squared objective,
    IRLS, world-frame arithmetic) on a 64x512 pair, whose levels 2 and 1 each
    run in one launch, against the oracle's registration on the same FP32
    surfels: the same iterations per level, the pose within 1e-5 rad / m."""
    import oracle as O
    c = W.config0()
    g = c["geom"]
    kf = O.panorama_normals(g, c["kf"]).astype(np.float32)
    scan = O.panorama_normals(g, c["scan"]).astype(np.float32)
    delta = 0.01 if variant == "irls" else 0.0
    world = c["T_world_kf"] if variant == "world" else None
    p = gpu_lib.IcpParams(levels=3, iters=(10, 10, 10), irls_delta=delta)
    res = gpu_lib.read_result(gpu_lib.register_scan(ctx, g, _t(scan), g, _t(kf), np.eye(4), p, world_kf=world))
    ref = O.register(g, scan.astype(np.float64), g, kf.astype(np.float64), np.eye(4),
                     O.IcpParams(levels=3, iters=(10, 10, 10), irls_delta=delta))
    rot, tr = synth.pose_error(res["T"], ref["T"])
    print(f"\n{variant}: {rot:.2e} rad {tr:.2e} m, iterations per level {res['level_iters']}")
    assert res["status"] == ref["status"]
    assert list(res["level_iters"][:3]) == list(ref["level_iters"][:3])
    assert rot < 1e-5 and tr < 1e-5


def test_level_kernel_beside_a_batch_on_another_stream(gpu_lib):
    """A single registration (its coarsest level in the one-XCD level kernel,
    whose workgroups wait for each other) replayed on one stream while a
    batch of 16 registrations is replayed on another, so that the batch's
    launches hold the CUs the level kernel's workgroups wait for: both
    results are bitwise the ones each gives alone, five rounds in a row."""
    import torch
    ctx1 = gpu_lib.Context(0, max_pixels=128 * 1024)
    ctx2 = gpu_lib.Context(0, max_pixels=128 * 1024, max_batch=16, max_batch_pixels=16 * 128 * 1024)
    try:
        dev = torch.device("cuda:0")
        c = W.config0(rows=128, cols=1024)
        g = c["geom"]
        kf = gpu_lib.panorama_normals(ctx1, g, _t(c["kf"].astype(np.float32)))
        scan = gpu_lib.panorama_normals(ctx1, g, _t(c["scan"].astype(np.float32)))
        p = gpu_lib.IcpParams(levels=3, iters=(10, 10, 10))
        init_d = gpu_lib.pose_tensor(synth.se3(synth.rot_z(0.02), [0.1, -0.05, 0.0]), dev)
        items = []
        for k in range(16):
            q = W.batch_pair(k, size=(128, 1024), max_angle=np.radians(6), max_trans=0.5)
            items.append(dict(scan_geom=q["geom"], kf_geom=q["geom"],
                              scan_surfel=gpu_lib.panorama_normals(ctx2, q["geom"], _t(q["scan"].astype(np.float32))),
                              kf_surfel=gpu_lib.panorama_normals(ctx2, q["geom"], _t(q["kf"].astype(np.float32)))))
        b = gpu_lib.Batch(ctx2, items, gpu_lib.IcpParams(levels=3, iters=(10, 10, 10), stop_update_norm=1e-6))
        binit = torch.stack([gpu_lib.pose_tensor(np.eye(4), dev) for _ in items])
        r1 = gpu_lib.new_result(dev)
        r2 = torch.zeros((16, gpu_lib.RESULT_BYTES), dtype=torch.uint8, device=dev)
        sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
        graphs = []
        for st, fn in ((sa, lambda: gpu_lib.register_scan(ctx1, g, scan, g, kf, init_d, p, r1)),
                       (sb, lambda: b.register(binit, r2))):
            with torch.cuda.stream(st):
                fn()
            torch.cuda.synchronize()
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr, stream=st):
                fn()
            graphs.append(gr)
        # alone
        refs = []
        for st, gr, r in ((sa, graphs[0], r1), (sb, graphs[1], r2)):
            with torch.cuda.stream(st):
                gr.replay()
            torch.cuda.synchronize()
            refs.append(r.cpu().numpy().copy())
        # together: the batch first, the single registration behind it on the other stream
        for rnd in range(5):
            r1.zero_()
            r2.zero_()
            torch.cuda.synchronize()
            print(f"round {rnd}", flush=True)
            with torch.cuda.stream(sb):
                graphs[1].replay()
            with torch.cuda.stream(sa):
                graphs[0].replay()
            torch.cuda.synchronize()
            assert np.array_equal(r1.cpu().numpy(), refs[0]), rnd
            assert np.array_equal(r2.cpu().numpy(), refs[1]), rnd
        b.close()
    finally:
        torch.cuda.synchronize()
        ctx1.close()
        ctx2.close()
