"""The symmetries the proposal's training data relies on (CPU): rolling a
panorama by k columns is the rotation of its frame by 2 pi k / cols about z,
and the targets of rolled / mirrored pairs transform as the poses do."""
import math

import numpy as np

import synth
from paper_2101_00585_amd import proposal as P


def test_roll_is_a_rotation_about_z():
    scene = synth.room_scene(3, sensor_positions=[[0.0, 0.0, 1.5]])
    g = synth.lidar_geom(32, 256)
    T = synth.se3(synth.rot_z(0.3) @ synth.rot_x(0.02), [0.4, -0.2, 1.5])
    d0 = synth.render(scene, g, T, dtype=np.float64)
    for k in (1, 17, 200):
        D = 2 * math.pi * k / 256
        d1 = synth.render(scene, g, T @ synth.se3(synth.rot_z(D), [0, 0, 0]), dtype=np.float64)
        rolled = d0[:, (np.arange(256) + k) % 256]
        ok = (d1 > 0) & (rolled > 0)
        assert ok.mean() > 0.95
        assert np.abs(d1[ok] - rolled[ok]).max() < 1e-6


def test_target_transforms_match_the_poses():
    rng = np.random.Generator(np.random.PCG64(4))
    S = np.diag([1.0, -1.0, 1.0, 1.0])
    for _ in range(20):
        w = rng.normal(size=3) * 0.3
        T = synth.se3(synth.rot_z(w[2]) @ synth.rot_y(w[1]) @ synth.rot_x(w[0]), rng.normal(size=3))
        y = P.pose_to_target(T)[None]
        k = int(rng.integers(256))
        Rz = synth.se3(synth.rot_z(2 * math.pi * k / 256), [0, 0, 0])
        np.testing.assert_allclose(P.roll_targets(y, [k])[0], P.pose_to_target(Rz.T @ T @ Rz), atol=1e-12)
        np.testing.assert_allclose(P.mirror_targets(y, [True])[0], P.pose_to_target(S @ T @ S), atol=1e-12)


def test_scan_roll_targets_match_the_pose():
    rng = np.random.Generator(np.random.PCG64(7))
    for _ in range(20):
        w = rng.normal(size=3) * 0.3
        T = synth.se3(synth.rot_z(w[2]) @ synth.rot_y(w[1]) @ synth.rot_x(w[0]), rng.normal(size=3))
        k2 = int(rng.integers(-48, 49))
        Rz = synth.se3(synth.rot_z(2 * math.pi * k2 / 256), [0, 0, 0])
        got = P.scan_roll_targets(P.pose_to_target(T)[None], [k2])[0]
        np.testing.assert_allclose(got, P.pose_to_target(T @ Rz), atol=1e-12)


def test_augment_inputs_and_targets_agree_with_numpy():
    import torch
    rng = np.random.Generator(np.random.PCG64(5))
    x = rng.normal(size=(6, 4, 256, 2)).astype(np.float32)
    k = rng.integers(0, 256, size=6)
    flip = np.array([0, 1, 0, 1, 1, 0], bool)
    k2 = rng.integers(-48, 49, size=6)
    got = P.augment_inputs(torch.from_numpy(x), torch.from_numpy(k), torch.from_numpy(flip),
                           torch.from_numpy(k2)).numpy()
    j = np.arange(256)
    for b in range(6):
        ref = x[b].copy()
        ref[:, :, 1] = ref[:, (j + k2[b]) % 256, 1]
        ref = ref[:, (j + k[b]) % 256]
        if flip[b]:
            ref = ref[:, (256 - j) % 256]
        np.testing.assert_array_equal(got[b], ref)
    y = rng.normal(size=(6, 6)) * 0.5
    ref = P.mirror_targets(P.roll_targets(P.scan_roll_targets(y, k2), k), flip)
    got = P._augment_targets_torch(torch.from_numpy(y), torch.from_numpy(k), torch.from_numpy(flip),
                                   torch.from_numpy(k2)).numpy()
    np.testing.assert_allclose(got, ref, atol=1e-10)


def test_log_so3_round_trip():
    rng = np.random.Generator(np.random.PCG64(6))
    for _ in range(20):
        w = rng.normal(size=3)
        w *= rng.uniform(0, 3.0) / np.linalg.norm(w)  # angles below pi
        th = np.linalg.norm(w)
        K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        R = np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * K @ K
        np.testing.assert_allclose(P.log_so3(R), w, atol=1e-10)
