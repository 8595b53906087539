"""The largest panoramas the library accepts, on the GPU: 4096 rows x 16384
columns (2^26 pixels, the context limit), a noise-free box room rendered in
FP64.  The oracle cannot run at this size in a test, so the checks are
properties that hold at any size: surfel normals equal the rendered faces'
exact normals away from edges, every valid pixel corresponds to itself at the
identity (bit-exact indices at the largest pixel index), and a registration
recovers a known motion.  Sized to stay within a few seconds on the GPU and a
few GB of host memory."""
import math

import numpy as np
import pytest

import synth
from synth import lidar_geom, rot_x, rot_z, se3

pytestmark = pytest.mark.gpu

ROWS, COLS = 4096, 16384


@pytest.fixture(scope="module")
def big(gpu_lib):
    import torch
    g = lidar_geom(ROWS, COLS)
    scene = synth.room_scene(0, sensor_positions=[[0.0, 0.0, 1.5], [0.05, 0.03, 1.5]], n_boxes=3)
    T_kf = se3(np.eye(3), [0.0, 0.0, 1.5])
    T_gt = se3(rot_z(math.radians(1.0)) @ rot_x(math.radians(0.5)), [0.05, 0.03, 0.0])
    kf, kf_n = synth.render(scene, g, T_kf, want_normals=True)
    scan = synth.render(scene, g, T_kf @ T_gt)
    ctx = gpu_lib.Context(0, max_pixels=ROWS * COLS)
    kf_s = gpu_lib.panorama_normals(ctx, g, torch.from_numpy(kf).cuda())
    scan_s = gpu_lib.panorama_normals(ctx, g, torch.from_numpy(scan).cuda())
    torch.cuda.synchronize()
    yield dict(g=g, ctx=ctx, kf=kf, kf_n=kf_n, kf_s=kf_s, scan_s=scan_s, T_gt=T_gt)
    ctx.close()


def test_normals_at_the_largest_size(big):
    s = big["kf_s"][::7, ::13].cpu().numpy()      # a strided sample of the image
    n_true = big["kf_n"][::7, ::13]
    valid = big["kf"][::7, ::13] > 0
    ok = valid & (np.abs(s[..., :3]).sum(-1) > 0)
    assert ok.sum() > 0.95 * valid.sum()
    err = np.linalg.norm(s[..., :3][ok] - n_true[ok], axis=-1)
    print(f"normals: {ok.sum()} sampled, median error {np.median(err):.2e}, 99th pct {np.percentile(err, 99):.2e}")
    # FP32 ranges at 0.02 deg pixel spacing: neighbour differences carry ~1e-5 relative noise
    assert np.median(err) < 5e-5 and np.percentile(err, 95) < 1e-3


def test_identity_correspondences_at_the_largest_size(gpu_lib, big):
    import torch
    g = big["g"]
    idx, inl = gpu_lib.correspondences(big["ctx"], g, big["kf_s"], g, big["kf_s"], np.eye(4))
    torch.cuda.synchronize()
    own = torch.arange(ROWS * COLS, dtype=torch.int32, device="cuda").view(ROWS, COLS)
    surf = big["kf_s"]
    has = (surf[..., 3] > 0) & (surf[..., :3].abs().sum(-1) > 0)
    assert bool(((idx == own) | ~has).all())
    assert bool((idx[~has] == -1).all())
    assert bool((inl.bool() == has).all())
    assert int(idx.max()) == int(own[has].max())


def test_registration_at_the_largest_size(gpu_lib, big):
    g = big["g"]
    p = gpu_lib.IcpParams(levels=4, iters=(5, 5, 5, 5), stop_update_norm=1e-9)
    res = gpu_lib.read_result(gpu_lib.register_scan(big["ctx"], g, big["scan_s"], g, big["kf_s"], np.eye(4), p))
    rot, tr = synth.pose_error(res["T"], big["T_gt"])
    print(f"4096x16384 registration: {rot:.2e} rad {tr:.2e} m, status {res['status']}, "
          f"inlier ratio {res['inlier_ratio']:.3f}")
    assert res["status"] in (gpu_lib.STATUS_CONVERGED, gpu_lib.STATUS_MAX_ITERS)
    assert rot < 1e-5 and tr < 1e-4
