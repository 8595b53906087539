"""The sensor-scale registration on identical inputs, and where the two
pipelines part.

Workload: the 128x1024 outdoor scene (Perlin ground, 200 cylinders, 4
facades), a keyframe fused from 10 scans along a 5 m path, the 11th scan
displaced by up to 5 deg / 0.5 m and started at the 10th scan's pose, 3
pyramid levels x 10 Gauss-Newton iterations (Section III-B), then the scan
fused into the keyframe (Section III-C).

test_config1_identical_inputs gives both implementations the oracle's scan
surfels and the oracle-fused keyframe rounded to FP32: the pose must agree to
1e-5 rad / 1e-5 m, the quality block within the counted correspondence
mismatches, the fused keyframe within the counted count mismatches.

test_config1_pipeline_stages replaces the oracle's inputs by the GPU's one
stage at a time (scan normals; keyframe-scan normals; keyframe fusion), up to
the whole GPU pipeline, and requires each registered pose within 1e-5 rad /
1e-5 m of the oracle pipeline's.
"""
import numpy as np
import pytest

import oracle as O
import synth
from parity_checks import (assert_fusion_close, assert_quality_close, fusion_ambiguous, pose_displacement_bound,
                           quality_mismatches)
from synth import workloads as W

pytestmark = pytest.mark.gpu

P = dict(levels=3, iters=(10, 10, 10))


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def c1():
    return W.config1()


@pytest.fixture(scope="module")
def orc(c1):
    """The oracle pipeline: FP64 normals of every scan, FP64 fusion of the 10
    keyframe scans, FP64 registration of the 11th scan."""
    g = c1["geom"]
    kf_surf = [O.panorama_normals(g, d) for d in c1["kf_scans"]]
    kf = np.zeros((g.rows, g.cols, 4))
    cnt = np.zeros((g.rows, g.cols), np.uint16)
    for s, T in zip(kf_surf, c1["T_kf_scans"]):
        kf, cnt = O.fuse(g, s, g, kf, cnt, T)
    scan = O.panorama_normals(g, c1["scan"])
    reg = O.register(g, scan, g, kf, c1["T_init"], O.IcpParams(**P))
    return dict(kf_surf=kf_surf, kf=kf, cnt=cnt, scan=scan, reg=reg)


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0, max_pixels=128 * 1024)
    yield c
    c.close()


def test_config1_identical_inputs(gpu_lib, ctx, c1, orc):
    g = c1["geom"]
    kf = orc["kf"].astype(np.float32)
    scan = orc["scan"].astype(np.float32)
    cnt = orc["cnt"]
    res = gpu_lib.read_result(gpu_lib.register_scan(ctx, g, _t(scan), g, _t(kf), c1["T_init"],
                                                    gpu_lib.IcpParams(**P)))
    ref = O.register(g, scan, g, kf, c1["T_init"], O.IcpParams(**P))
    rot, tr = synth.pose_error(res["T"], ref["T"])
    rot_gt, tr_gt = synth.pose_error(ref["T"], c1["T_gt"])
    print(f"128x1024 outdoor, identical inputs: GPU vs oracle {rot:.2e} rad {tr:.2e} m "
          f"(oracle vs truth {rot_gt:.2e} rad {tr_gt:.2e} m); truncated cost {res['trunc_cost']:.6f} / "
          f"{ref['trunc_cost']:.6f}", flush=True)
    assert res["status"] == ref["status"] == 0
    assert res["iters_run"] == ref["iters_run"] == 30
    assert rot < 1e-5 and tr < 1e-5, (rot, tr)
    mism = quality_mismatches(gpu_lib, ctx, g, scan, kf, res["T"], ref["T"])
    rr = O.residuals(g, scan, g, kf, ref["T"])
    dr = pose_displacement_bound(res["T"], ref["T"], float(scan[..., 3].max()))
    assert_quality_close(res, ref, mism, 0.5, dr, float(np.abs(rr["r"][rr["inlier"]]).sum()))

    # then the scan is fused into the keyframe, each side at its own pose
    kf_d, cnt_d = _t(kf), _t(cnt.view(np.int16))
    gpu_lib.fuse_scan(ctx, g, _t(scan), g, kf_d, cnt_d, res["T"])
    ko, co = O.fuse(g, scan, g, kf, cnt, ref["T"])
    kg, cg = _np(kf_d), _np(cnt_d).view(np.uint16)
    amb = fusion_ambiguous(g, scan.astype(np.float64), g, kf.astype(np.float64), cnt, ref["T"])
    n_diff, n_amb, n_bad = assert_fusion_close(kg, cg, ko, co, amb)
    print(f"fusion: {n_diff} keyframe pixels differ, {n_amb} at a projection or gate boundary, "
          f"{n_bad} unexplained; {int((co > cnt).sum())} counts raised", flush=True)
    assert n_bad == 0 and n_diff <= 2e-3 * cg.size
    # pixels seen by all 10 keyframe scans stay at the saturated count
    assert (co > cnt).sum() > 0.1 * cg.size


def test_config1_pipeline_stages(gpu_lib, ctx, c1, orc):
    """Each stage of the GPU pipeline substituted for the oracle's alone; the
    registration itself is the GPU's in every row (identical inputs put it
    within 1e-5 of the oracle's, above)."""
    import torch
    g = c1["geom"]
    dev = torch.device("cuda:0")
    gpu_scan = gpu_lib.panorama_normals(ctx, g, _t(c1["scan"]))
    gpu_kf_surf = [gpu_lib.panorama_normals(ctx, g, _t(d)) for d in c1["kf_scans"]]

    def gpu_fusion(surfels):
        kf_d = torch.zeros((g.rows, g.cols, 4), dtype=torch.float32, device=dev)
        cnt_d = torch.zeros((g.rows, g.cols), dtype=torch.int16, device=dev)
        for s, T in zip(surfels, c1["T_kf_scans"]):
            gpu_lib.fuse_scan(ctx, g, s, g, kf_d, cnt_d, T)
        return kf_d

    def orc_fusion(surfels):
        kf = np.zeros((g.rows, g.cols, 4))
        cnt = np.zeros((g.rows, g.cols), np.uint16)
        for s, T in zip(surfels, c1["T_kf_scans"]):
            kf, cnt = O.fuse(g, s, g, kf, cnt, T)
        return _t(kf.astype(np.float32))

    o_scan = _t(orc["scan"].astype(np.float32))
    o_kf = _t(orc["kf"].astype(np.float32))
    gpu_kf_surf_np = [_np(s).astype(np.float64) for s in gpu_kf_surf]
    o_kf_surf32 = [_t(s.astype(np.float32)) for s in orc["kf_surf"]]
    rows = [
        ("oracle inputs", o_scan, o_kf),
        ("GPU scan normals", gpu_scan, o_kf),
        ("GPU keyframe-scan normals, oracle fusion", o_scan, orc_fusion(gpu_kf_surf_np)),
        ("oracle keyframe-scan normals, GPU fusion", o_scan, gpu_fusion(o_kf_surf32)),
        ("GPU keyframe (normals + fusion)", o_scan, gpu_fusion(gpu_kf_surf)),
        ("GPU pipeline", gpu_scan, gpu_fusion(gpu_kf_surf)),
    ]
    T_ref = orc["reg"]["T"]
    errs = {}
    for name, s_d, k_d in rows:
        r = gpu_lib.read_result(gpu_lib.register_scan(ctx, g, s_d, g, k_d, c1["T_init"], gpu_lib.IcpParams(**P)))
        rot, tr = synth.pose_error(r["T"], T_ref)
        errs[name] = (rot, tr)
        print(f"  {name:45s}: {rot:.2e} rad {tr:.2e} m from the oracle pipeline", flush=True)
    # FP32 normals and FP32 fusion keep the pipeline's pose within the
    # registration's own 1e-5 bar
    for name, (rot, tr) in errs.items():
        assert rot < 1e-5 and tr < 1e-5, (name, rot, tr)
