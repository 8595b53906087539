"""The registration entry point that allocates nothing
(ups_register_scan_noalloc: static device scratch, no context) against
ups_register_scan on the same inputs, through the C ABI: two calls in a row,
the second on smaller panoramas with fewer pyramid levels, then the first
again (the static scratch keeps the previous call's contents, which must not
leak into the next).  Poses within 1e-5 rad / 1e-5 m, same status and
iteration count, inlier counts within the counted correspondence mismatches
(the two paths compute their ray tables on the host and on the GPU)."""
import numpy as np
import pytest

import synth
from synth import workloads as W

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _np(t):
    return t.detach().cpu().numpy()


def test_noalloc_matches_context_entry_point(gpu_lib):
    import torch
    ctx = gpu_lib.Context(0, max_pixels=128 * 2048)
    big = W.batch_pair(3, size=(128, 2048), max_angle=np.radians(6), max_trans=0.5)
    small = W.config0()
    cases = [("128x2048, 3 levels", big, gpu_lib.IcpParams(levels=3, iters=(10, 10, 10))),
             ("64x512, 1 level", small, gpu_lib.IcpParams()),
             ("128x2048 again", big, gpu_lib.IcpParams(levels=3, iters=(10, 10, 10)))]
    for name, c, params in cases:
        g = c["geom"]
        print(f"[noalloc] {name}", flush=True)
        kf = gpu_lib.panorama_normals(ctx, g, _t(c["kf"]))
        scan = gpu_lib.panorama_normals(ctx, g, _t(c["scan"]))
        ref_t = gpu_lib.register_scan(ctx, g, scan, g, kf, np.eye(4), params)
        res_t = gpu_lib.register_scan_noalloc(g, scan, g, kf, np.eye(4), params)
        torch.cuda.synchronize()
        ref, res = gpu_lib.read_result(ref_t), gpu_lib.read_result(res_t)
        rot, tr = synth.pose_error(res["T"], ref["T"])
        bitwise = bool(np.array_equal(_np(res_t), _np(ref_t)))
        print(f"[noalloc] {name}: {rot:.2e} rad {tr:.2e} m from ups_register_scan, bitwise equal: {bitwise}",
              flush=True)
        assert rot < 1e-5 and tr < 1e-5, (name, rot, tr)
        assert res["status"] == ref["status"] and res["iters_run"] == ref["iters_run"]
        idx_r, inl_r = gpu_lib.correspondences(ctx, g, scan, g, kf, gpu_lib.result_pose(ref_t))
        idx_n, inl_n = gpu_lib.correspondences(ctx, g, scan, g, kf, gpu_lib.result_pose(res_t))
        mism = int(((idx_r != idx_n) | (inl_r != inl_n)).sum().item())
        assert abs(res["inliers"] - ref["inliers"]) <= mism and res["valid"] == ref["valid"]
        rot_gt, tr_gt = synth.pose_error(res["T"], c["T_gt"])
        assert rot_gt < 2e-3 and tr_gt < 2e-2, (name, rot_gt, tr_gt)
    ctx.close()
