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


EPS32 = 2.0 ** -24


def _bf16_flip_band(z, err):
    """Elements whose bfloat16-rounded ReLU output may differ between the
    pre-activation z and a value within err of it: |z| <= err (zero or not),
    or z > err within err of a bf16 rounding boundary."""
    b = C.bf16_round(z)
    e = np.floor(np.log2(np.maximum(np.abs(b), 1e-38)))
    half_ulp = 2.0 ** (e - 8)
    return (np.abs(z) <= err) | ((z > err) & (half_ulp - np.abs(z - b) <= err))


def test_network_forward_layer_by_layer(gpu_lib, prop):
    """The network object's forward pass, layer by layer on identical inputs:
    the oracle's convolution of the GPU's stored bfloat16 input of each layer
    (FP64) rounded to bfloat16 equals the GPU's stored output, except where
    the FP32 accumulation (at most K 2^-24 sum |x w| for K terms) can move the
    value across a bfloat16 rounding boundary, and there it is one bfloat16
    step away; the FP32 head equals the oracle's on the GPU's features within
    its accumulation bound."""
    p = _params(1)
    x = _inputs(2, 5)
    prop.set_params(p)
    y = _np(prop.forward(5, _bf(x)))
    convs, (Wfc, bfc) = C.unflatten(p)
    a = x
    for k, ((W, b), (cin, cout, s)) in enumerate(zip(convs, C.LAYERS)):
        got, _ = prop.activations(k + 1, 5)
        Wb = C.bf16_round(W)
        z = C.conv_forward(a, Wb, b, s)
        bound = 9 * cin * EPS32 * (C.conv_forward(np.abs(a), np.abs(Wb), np.abs(b), s) + 1e-30)
        ref = C.bf16_round(C.relu(z))
        band = _bf16_flip_band(z, bound)
        diff = got != ref
        print(f"layer {k + 1}: {diff.sum()} of {diff.size} outputs differ, {band.sum()} in the rounding band")
        assert not (diff & ~band).any(), (k, int((diff & ~band).sum()))
        assert (np.abs(got - ref)[diff] <= 2.0 ** (np.floor(np.log2(np.maximum(np.abs(ref[diff]), 1e-38))) - 7)
                + bound[diff]).all()
        assert band.mean() < 0.5  # at least half the outputs are held bit-exact
        a = got
    f = a.reshape(a.shape[0], -1)
    y_ref = C.fc_forward(f, Wfc, bfc)
    bound = C.FEAT * EPS32 * (np.abs(f) @ np.abs(Wfc).T + np.abs(bfc)) + 1e-30
    assert (np.abs(y - y_ref) <= bound).all(), np.abs(y - y_ref).max()


def _within(got, ref, floor, rel=1e-4):
    return np.abs(got - ref) <= rel * np.abs(ref) + floor


def test_network_gradients_layer_by_layer(gpu_lib, prop):
    """One training step (lr = 0) checked stage by stage on identical
    inputs: the loss, the head's gradients and the feature gradient from the
    GPU's output and features; each convolution's weight and bias gradients
    and its input gradient from the GPU's stored input, output and output
    gradient of that layer.  Both backward passes take the masked output
    gradient as a bfloat16 matrix-core operand, so the oracle is fed the same
    bfloat16 values and only accumulation differs.  Element-wise: within 1e-4
    relative plus the FP32 accumulation bound n 2^-24 sum |terms| of the
    element's own n terms."""
    import torch
    p = _params(3)
    x = _inputs(4, 6)
    target = _rng(5).normal(size=(6, 6))
    prop.set_params(p)
    y = _np(prop.forward(6, _bf(x))).astype(np.float64)
    loss = prop.train_step(_bf(x), _f32(target), lr=0.0)
    torch.cuda.synchronize()
    g = prop.get_grads().astype(np.float64)
    assert np.array_equal(prop.get_params(), p.astype(np.float32))
    convs, (Wfc, bfc) = C.unflatten(p)
    gconvs, (gWfc, gbfc) = C.unflatten(g)
    acts = [x] + [prop.activations(k, 6)[0] for k in range(1, 6)]
    dacts = [None] + [prop.activations(k, 6)[1] for k in range(1, 6)]
    L = C.loss(y, target)
    assert abs(float(loss.item()) - L) <= 1e-5 * abs(L)
    # head
    dout = C.loss_grad(y, target)
    f = acts[5].reshape(6, -1)
    df, dW, db = C.fc_backward(f, Wfc, dout)
    adf, adW, adb = C.fc_backward(np.abs(f), np.abs(Wfc), np.abs(dout))
    assert _within(gWfc, dW, 6 * EPS32 * adW + 1e-30).all()
    assert _within(gbfc, db, 6 * EPS32 * adb + 1e-30).all()
    assert _within(dacts[5].reshape(6, -1), df, 6 * EPS32 * adf + 1e-30).all()
    # convolutions, last to first
    checked = 0
    for k in range(4, -1, -1):
        cin, cout, s = C.LAYERS[k]
        Wb = C.bf16_round(convs[k][0])
        xk, yk, dyk = acts[k], acts[k + 1], C.bf16_round(dacts[k + 1])
        dx, dW, db = C.conv_backward(xk, yk, dyk, Wb, s)
        adx, adW, adb = C.conv_backward(np.abs(xk), yk, np.abs(dyk), np.abs(Wb), s)
        m = yk.shape[0] * yk.shape[1] * yk.shape[2]  # terms of a weight-gradient element
        ok_w = _within(gconvs[k][0], dW, m * EPS32 * adW + 1e-30)
        ok_b = _within(gconvs[k][1], db, m * EPS32 * adb + 1e-30)
        print(f"layer {k + 1}: weight gradient max rel err "
              f"{(np.abs(gconvs[k][0] - dW) / (np.abs(dW) + 1e-30)).max():.2e}")
        assert ok_w.all() and ok_b.all(), (k, int((~ok_w).sum()), int((~ok_b).sum()))
        if k > 0:
            ok_x = _within(dacts[k], dx, 9 * cout * EPS32 * adx + 1e-30)
            assert ok_x.all(), (k, int((~ok_x).sum()))
        checked += dW.size
    assert checked == sum(9 * ci * co for ci, co, _ in C.LAYERS)


def test_checkpoint_resumes_training_exactly(gpu_lib, prop, tmp_path):
    """Two Adam steps, a checkpoint, a third step; a new network loaded from
    the checkpoint takes the third step to bitwise the same parameters, while
    one loaded from the parameter file alone (moments reset) does not."""
    import torch
    p = _params(13) * 0.5
    xa, xb = _bf(_inputs(14, 8)), _bf(_inputs(15, 8))
    ta, tb = _f32(_rng(16).normal(size=(8, 6))), _f32(_rng(17).normal(size=(8, 6)))
    prop.set_params(p)
    prop.train_step(xa, ta, lr=1e-3)
    prop.train_step(xb, tb, lr=1e-3)
    ckpt, params_file = str(tmp_path / "state.ckpt"), str(tmp_path / "params.bin")
    prop.save_checkpoint(ckpt)
    prop.save(params_file)
    prop.train_step(xa, ta, lr=1e-3)
    torch.cuda.synchronize()
    want = prop.get_params()
    raw = open(ckpt, "rb").read()
    assert raw[:8] == b"UPSCKP01" and int.from_bytes(raw[16:24], "little") == 2
    for loader, same in (("load_checkpoint", True), ("load", False)):
        other = gpu_lib.Proposal(prop.ctx, 8)
        try:
            getattr(other, loader)(ckpt if same else params_file)
            other.train_step(xa, ta, lr=1e-3)
            torch.cuda.synchronize()
            assert np.array_equal(other.get_params(), want) == same, loader
        finally:
            other.close()
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(raw[:-4])
    with pytest.raises(gpu_lib.UpsError):
        prop.load_checkpoint(str(bad))
    with pytest.raises(gpu_lib.UpsError):
        prop.load_checkpoint(params_file)


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


def test_training_loop_resumes_exactly(gpu_lib, prop, tmp_path):
    """The training loop interrupted after 3 of 6 steps and resumed from its
    checkpoint (parameters, Adam moments, step count, the batch generator's
    state) ends with bitwise the parameters of the uninterrupted run."""
    import torch
    from paper_2101_00585_amd import proposal as P
    x = _bf(_inputs(20, 12))
    y = _rng(21).normal(size=(12, 6)) * 0.3
    p0 = _params(22) * 0.5
    ck = str(tmp_path / "loop.ckpt")
    prop.set_params(p0)
    P.train(prop, x, y, steps=6, batch=4, lr=1e-3, seed=7)
    torch.cuda.synchronize()
    want = prop.get_params()
    prop.set_params(p0)
    P.train(prop, x, y, steps=6, batch=4, lr=1e-3, seed=7, checkpoint=ck, checkpoint_every=3, until=3)
    other = gpu_lib.Proposal(prop.ctx, 8)
    try:
        other.set_params(np.zeros_like(p0))
        P.train(other, x, y, steps=6, batch=4, lr=1e-3, seed=99, checkpoint=ck, resume=True)
        torch.cuda.synchronize()
        assert np.array_equal(other.get_params(), want)
    finally:
        other.close()
