"""The proposal network's HIP kernels (BF16 MFMA convolutions, FP32 head,
loss, Adam, input and pose maps) against the FP64 oracle in oracle/cnn.py.

The oracle is fed bfloat16-rounded copies of every operand the GPU stores in
bfloat16 (inputs, conv weights, masked output gradients), so only the
accumulation differs: FP32 on the matrix cores against FP64."""
import numpy as np
import pytest

from oracle import cnn as C

pytestmark = pytest.mark.gpu


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _bf(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).cuda()


def _f32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _np(t):
    import torch
    return t.detach().to(torch.float64).cpu().numpy()


# network layers plus shapes with ragged tiles, odd channel counts and stride 1;
# between them every operand-gather path of the forward pass (four channels
# per load, channel pairs, single channels) with 16- and 32-wide K slices
SHAPES = [(2, h, w, cin, cout, s) for (h, w, cin, cout, s) in C.shapes()[0]] + [
    (3, 6, 12, 3, 8, 1), (1, 5, 14, 6, 12, 2), (5, 4, 64, 16, 68, 2), (2, 4, 8, 5, 8, 1), (1, 3, 10, 1, 4, 2)]


def _layer_case(shape, seed):
    n, h, w, cin, cout, s = shape
    r = _rng(seed)
    x = C.bf16_round(np.abs(r.normal(size=(n, h, w, cin))) * (r.uniform(size=(n, h, w, cin)) > 0.2))
    W = C.bf16_round(r.normal(size=(9 * cin, cout)) * np.sqrt(2.0 / (9 * cin)))
    b = r.normal(size=cout).astype(np.float32).astype(np.float64) * 0.1
    return x, W, b


def _close_bf16(g, ref, what):
    """GPU bf16 outputs equal the rounded FP64 result up to one bf16 step where
    the FP32 and FP64 sums straddle a rounding boundary."""
    tol = 2.0 ** -7 * np.maximum(np.abs(ref), np.abs(g)) + 1e-6
    bad = np.abs(g - ref) > tol
    assert not bad.any(), (what, int(bad.sum()), float(np.abs(g - ref).max()))
    assert np.mean(g == ref) > 0.98, (what, float(np.mean(g == ref)))


@pytest.mark.parametrize("shape", SHAPES, ids=[f"n{s[0]}_{s[1]}x{s[2]}_{s[3]}to{s[4]}_s{s[5]}" for s in SHAPES])
def test_conv_forward(gpu_lib, shape):
    n, h, w, cin, cout, s = shape
    x, W, b = _layer_case(shape, 100 + h + cin)
    y = gpu_lib.conv3x3_forward(_bf(x), _bf(W.T), _f32(b), cout, s)
    ref = C.bf16_round(C.relu(C.conv_forward(x, W, b, s)))
    assert tuple(y.shape) == ref.shape
    _close_bf16(_np(y), ref, "forward")


@pytest.mark.parametrize("shape", SHAPES, ids=[f"n{s[0]}_{s[1]}x{s[2]}_{s[3]}to{s[4]}_s{s[5]}" for s in SHAPES])
def test_conv_backward(gpu_lib, shape):
    n, h, w, cin, cout, s = shape
    x, W, b = _layer_case(shape, 200 + h + cin)
    r = _rng(300 + cout)
    # y from the oracle (rounded as stored), dy rounded as the GPU rounds the masked gradient
    y = C.bf16_round(C.relu(C.conv_forward(x, W, b, s)))
    dy = C.bf16_round(r.normal(size=y.shape))
    dx_ref, dW_ref, db_ref = C.conv_backward(x, y, dy, W, s)
    dx = gpu_lib.conv3x3_backward_data(_bf(y), _f32(dy), _bf(W), h, w, cin, s)
    dW, db = gpu_lib.conv3x3_backward_weight(_bf(x), _bf(y), _f32(dy), s)
    for got, ref, what in ((_np(dx), dx_ref, "dx"), (_np(dW), dW_ref, "dW"), (_np(db), db_ref, "db")):
        scale = np.abs(ref).max() + 1e-30
        err = np.abs(got - ref).max() / scale
        assert err < 2e-5, (what, err)


def test_conv_empty_batch(gpu_lib):
    import torch
    x = torch.zeros((0, 8, 16, 4), dtype=torch.bfloat16, device="cuda")
    W = _bf(np.ones((36, 8)))
    y = gpu_lib.conv3x3_forward(x, _bf(np.ones((8, 36))), _f32(np.zeros(8)), 8, 2)
    assert tuple(y.shape) == (0, 4, 8, 8)
    dw, db = gpu_lib.conv3x3_backward_weight(x, y, torch.zeros((0, 4, 8, 8), dtype=torch.float32, device="cuda"), 2)
    assert float(dw.abs().sum()) == 0.0 and float(db.abs().sum()) == 0.0
    del W


def test_conv_rejects_bad_shapes(gpu_lib):
    x = _bf(np.zeros((1, 8, 16, 4)))
    with pytest.raises(gpu_lib.UpsError):
        gpu_lib.conv3x3_forward(x, _bf(np.zeros((6, 36))), _f32(np.zeros(6)), 6, 2)  # cout not a multiple of 4
    with pytest.raises(gpu_lib.UpsError):
        gpu_lib.conv3x3_forward(x, _bf(np.zeros((8, 36))), _f32(np.zeros(8)), 8, 3)  # stride 3


def _params(seed):
    r = _rng(seed)
    parts = []
    for cin, cout, _ in C.LAYERS:
        parts += [r.normal(size=9 * cin * cout) * np.sqrt(2.0 / (9 * cin)), r.normal(size=cout) * 0.05]
    parts += [r.normal(size=6 * C.FEAT) * np.sqrt(1.0 / C.FEAT), r.normal(size=6) * 0.1]
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def _inputs(seed, n):
    r = _rng(seed)
    x = r.uniform(0.02, 1.0, size=(n, 32, 256, 2))
    x[r.uniform(size=x.shape) < 0.25] = 0.0
    return C.bf16_round(x)


@pytest.fixture(scope="module")
def prop(gpu_lib):
    ctx = gpu_lib.Context(0, max_pixels=1 << 16)
    p = gpu_lib.Proposal(ctx, 16)
    yield p
    p.close()
    ctx.close()


def test_network_forward(gpu_lib, prop):
    p = _params(1)
    x = _inputs(2, 5)
    prop.set_params(p)
    y = _np(prop.forward(5, _bf(x)))
    ref = C.forward(p, x, bf16=True)
    assert np.abs(y - ref).max() <= 1e-2 * (np.abs(ref).max() + 1.0), (y, ref)


def test_network_gradients(gpu_lib, prop):
    import torch
    p = _params(3)
    x = _inputs(4, 6)
    target = _rng(5).normal(size=(6, 6))
    prop.set_params(p)
    loss = prop.train_step(_bf(x), _f32(target), lr=0.0)
    torch.cuda.synchronize()
    g = prop.get_grads().astype(np.float64)
    L, gref = C.gradients(p, x, target, bf16=True)
    assert abs(float(loss.item()) - L) <= 1e-3 * abs(L)
    # parameters unchanged at lr = 0
    assert np.array_equal(prop.get_params(), p.astype(np.float32))
    sizes = np.cumsum([0] + C.param_sizes())
    for k in range(len(sizes) - 1):
        a, b = g[sizes[k]:sizes[k + 1]], gref[sizes[k]:sizes[k + 1]]
        rel = np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-30)
        assert rel < 2e-2, (k, rel)


def test_adam_steps(gpu_lib, prop):
    """Conv weights zero: every activation is zero, only the FC bias has a
    gradient (the mean output error), so the GPU's Adam steps can be replayed
    exactly by the oracle's."""
    import torch
    r = _rng(6)
    p = np.zeros(C.NUM_PARAMS)
    p[-6 * C.FEAT - 6:-6] = r.normal(size=6 * C.FEAT) * 0.01
    p[-6:] = r.normal(size=6)
    p = p.astype(np.float32).astype(np.float64)
    x = _inputs(7, 4)
    target = r.normal(size=(4, 6)).astype(np.float32).astype(np.float64)
    prop.set_params(p)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    pr = p.copy()
    for t in range(1, 4):
        prop.train_step(_bf(x), _f32(target), lr=0.01)
        _, g = C.gradients(pr, x, target, bf16=True)
        pr, m, v = C.adam_step(pr, g, m, v, t, 0.01)
    torch.cuda.synchronize()
    got = prop.get_params().astype(np.float64)
    np.testing.assert_allclose(got, pr, rtol=1e-5, atol=1e-7)
    assert np.array_equal(got[:-6], p[:-6].astype(np.float32))


def test_training_reduces_loss(gpu_lib, prop):
    import torch
    p = _params(8) * 0.5
    x = _inputs(9, 16)
    target = _rng(10).normal(size=(16, 6)) * 0.5
    prop.set_params(p)
    xs, ts = _bf(x), _f32(target)
    losses = []
    for _ in range(60):
        losses.append(float(prop.train_step(xs, ts, lr=1e-3).item()))
    torch.cuda.synchronize()
    assert losses[-1] < 0.2 * losses[0], losses[::10]


def test_input_from_depth_and_surfels(gpu_lib, prop):
    import torch
    import synth
    r = _rng(11)
    depth = r.uniform(0.5, 60.0, size=(64, 512)).astype(np.float32)
    depth[r.uniform(size=depth.shape) < 0.1] = 0.0
    depth2 = r.uniform(0.5, 40.0, size=(128, 1024)).astype(np.float32)
    d1, d2 = _f32(depth), _f32(depth2)
    surf = torch.zeros((128, 1024, 4), dtype=torch.float32, device="cuda")
    surf[..., 3] = d2
    g1, g2 = synth.lidar_geom(64, 512), synth.lidar_geom(128, 1024)
    prop.plan_input([d1, surf], [d2, d1], [g1, g2], [g2, g1])
    x = torch.empty((2, 32, 256, 2), dtype=torch.bfloat16, device="cuda")
    prop.input(x)
    got = _np(x)
    np.testing.assert_array_equal(got[0], C.network_input(depth, depth2))
    np.testing.assert_array_equal(got[1], C.network_input(depth2, depth))


def test_poses_from_outputs(gpu_lib, prop):
    r = _rng(12)
    y = r.normal(size=(7, 6)).astype(np.float32)
    y[0] = 0.0
    P = _np(prop.poses(_f32(y)))
    for k in range(7):
        T = C.proposal_pose(y[k].astype(np.float64))
        np.testing.assert_allclose(P[k, :9].reshape(3, 3), T[:3, :3], atol=1e-14)
        np.testing.assert_allclose(P[k, 9:], T[:3, 3], atol=1e-14)


def test_parameter_file_round_trip(gpu_lib, prop, tmp_path):
    """save / load through the C ABI: the same parameters come back in a new
    network object; other files are rejected."""
    path = str(tmp_path / "params.bin")
    ref = prop.get_params()
    prop.save(path)
    raw = open(path, "rb").read()
    assert raw[:8] == b"UPSPRM01" and int.from_bytes(raw[8:16], "little") == ref.size
    assert len(raw) == 16 + 4 * ref.size
    other = gpu_lib.Proposal(prop.ctx, 4)
    try:
        other.load(path)
        assert np.array_equal(other.get_params(), ref)
        bad = tmp_path / "bad.bin"
        bad.write_bytes(raw[:-4])              # truncated
        with pytest.raises(gpu_lib.UpsError):
            other.load(str(bad))
        bad.write_bytes(b"XXXXXXXX" + raw[8:])  # wrong magic
        with pytest.raises(gpu_lib.UpsError):
            other.load(str(bad))
        bad.write_bytes(raw + b"\0")           # trailing bytes
        with pytest.raises(gpu_lib.UpsError):
            other.load(str(bad))
        assert np.array_equal(other.get_params(), ref)
    finally:
        other.close()
