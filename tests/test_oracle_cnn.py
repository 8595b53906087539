"""Pins of the FP64 proposal-network oracle (oracle/cnn.py) against library
routines (torch autograd and convolution, scipy rotations), central finite
differences and closed forms."""
import math

import numpy as np
import pytest

from oracle import cnn as C


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _torch():
    import torch
    return torch


def test_bf16_round_known_values_and_torch():
    one = 1.0
    # ties go to the even mantissa: 1 + 2^-8 -> 1, 1 + 3 2^-8 -> 1 + 2^-6
    assert C.bf16_round(np.array([one + 2 ** -8]))[0] == 1.0
    assert C.bf16_round(np.array([one + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6
    assert C.bf16_round(np.array([one + 2 ** -8 + 2 ** -20]))[0] == 1.0 + 2 ** -7
    assert C.bf16_round(np.array([-2.5]))[0] == -2.5
    torch = _torch()
    x = _rng(1).normal(size=4096).astype(np.float32) * 10.0 ** _rng(2).uniform(-6, 6, size=4096).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(C.bf16_round(x), ref)
    assert np.array_equal(C.bf16_bits(x), torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy()
                          .astype(np.uint16))


def _torch_conv(x, W, b, s):
    """The same convolution from torch: circular padding of the width, zero
    padding of the height, NCHW conv2d with weights [cout][cin][3][3]."""
    torch = _torch()
    F = torch.nn.functional
    n, h, w, cin = x.shape
    cout = W.shape[1]
    xt = x.permute(0, 3, 1, 2)
    xt = F.pad(xt, (1, 1, 0, 0), mode="circular")
    Wt = W.reshape(3, 3, cin, cout).permute(3, 2, 0, 1)
    z = F.conv2d(xt, Wt, b, stride=s, padding=(1, 0))
    return z.permute(0, 2, 3, 1)


@pytest.mark.parametrize("h,w,cin,cout,s", [(8, 16, 2, 4, 2), (6, 12, 3, 5, 1), (7, 10, 4, 3, 2), (4, 8, 8, 8, 1)])
def test_conv_forward_backward_against_torch(h, w, cin, cout, s):
    torch = _torch()
    r = _rng(h * 100 + w)
    x = r.normal(size=(2, h, w, cin))
    W = r.normal(size=(9 * cin, cout))
    b = r.normal(size=cout)
    z = C.conv_forward(x, W, b, s)
    xt = torch.tensor(x, requires_grad=True)
    Wt = torch.tensor(W, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    zt = _torch_conv(xt, Wt, bt, s)
    assert zt.shape == z.shape
    np.testing.assert_allclose(z, zt.detach().numpy(), rtol=1e-12, atol=1e-12)
    y = C.relu(z)
    dy = r.normal(size=y.shape)
    dx, dW, db = C.conv_backward(x, y, dy, W, s)
    (torch.relu(zt) * torch.tensor(dy)).sum().backward()
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dW, Wt.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_conv_brute_force_tiny():
    """One output written out from the definition, with a wrapped column and
    a zero row."""
    r = _rng(5)
    x = r.normal(size=(1, 4, 6, 2))
    W = r.normal(size=(18, 3))
    b = r.normal(size=3)
    z = C.conv_forward(x, W, b, 2)
    oy, ox, co = 0, 0, 2
    acc = b[co]
    for ky in range(3):
        for kx in range(3):
            iy, ix = 2 * oy + ky - 1, (2 * ox + kx - 1) % 6
            if 0 <= iy < 4:
                for ci in range(2):
                    acc += x[0, iy, ix, ci] * W[(3 * ky + kx) * 2 + ci, co]
    assert abs(z[0, oy, ox, co] - acc) < 1e-13


def test_shapes_and_parameter_count():
    sh, feat = C.shapes()
    assert [s[:2] for s in sh] == [(32, 256), (16, 128), (8, 64), (4, 32), (2, 16)]
    assert feat == 4096
    assert C.NUM_PARAMS == sum(9 * a * b + b for a, b, _ in C.LAYERS) + 6 * 4096 + 6 == 357_382


def _params(seed, scale=1.0):
    r = _rng(seed)
    parts = []
    for cin, cout, _ in C.LAYERS:
        parts += [r.normal(size=9 * cin * cout) * math.sqrt(2.0 / (9 * cin)) * scale, r.normal(size=cout) * 0.1]
    parts += [r.normal(size=6 * C.FEAT) * math.sqrt(1.0 / C.FEAT), r.normal(size=6) * 0.1]
    return np.concatenate(parts)


def _inputs(seed, n=2):
    r = _rng(seed)
    x = r.uniform(0.0, 1.0, size=(n, 32, 256, 2))
    x[r.uniform(size=x.shape) < 0.2] = 0.0
    return x


def test_network_gradient_against_finite_differences():
    p = _params(7)
    x = _inputs(8)
    target = _rng(9).normal(size=(2, 6))
    L, g = C.gradients(p, x, target)
    r = _rng(10)
    sizes = np.cumsum([0] + C.param_sizes())
    picks = [int(r.integers(sizes[k], sizes[k + 1])) for k in range(len(sizes) - 1)]
    h = 1e-6
    for i in picks:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (C.loss(C.forward(pp, x), target) - C.loss(C.forward(pm, x), target)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3), (i, fd, g[i])


def test_network_against_torch_autograd():
    torch = _torch()
    p = _params(11)
    x = _inputs(12, n=3)
    target = _rng(13).normal(size=(3, 6))
    L, g = C.gradients(p, x, target)
    convs, (Wfc, bfc) = C.unflatten(p)
    ts = [torch.tensor(a, requires_grad=True) for W, b in convs for a in (W, b)]
    tfc = [torch.tensor(Wfc, requires_grad=True), torch.tensor(bfc, requires_grad=True)]
    a = torch.tensor(x)
    for k, (_, _, s) in enumerate(C.LAYERS):
        a = torch.relu(_torch_conv(a, ts[2 * k], ts[2 * k + 1], s))
    y = a.reshape(3, -1) @ tfc[0].T + tfc[1]
    Lt = ((y - torch.tensor(target)) ** 2).sum() / (2 * 3)
    Lt.backward()
    assert abs(L - Lt.item()) < 1e-12 * max(1.0, abs(L))
    gt = np.concatenate([t.grad.numpy().ravel() for t in ts + tfc])
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-12)


def test_adam_first_step_closed_form_and_torch():
    torch = _torch()
    r = _rng(14)
    p0 = r.normal(size=50)
    lr = 1e-3
    gs = [r.normal(size=50) for _ in range(3)]
    # step 1: m^ = g, v^ = g^2, so the update is lr g / (|g| + eps)
    p1, m, v = C.adam_step(p0, gs[0], np.zeros(50), np.zeros(50), 1, lr)
    np.testing.assert_allclose(p1, p0 - lr * gs[0] / (np.abs(gs[0]) + 1e-8), rtol=0, atol=1e-15)
    pt = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(gs, start=1):
        p, m, v = C.adam_step(p, g, m, v, t, lr)
        pt.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=0, atol=1e-14)


def test_pose_maps():
    from scipy.spatial.transform import Rotation
    r = _rng(15)
    for _ in range(20):
        w = r.normal(size=3) * r.uniform(0, 1.5)
        np.testing.assert_allclose(C.exp_so3(w), Rotation.from_rotvec(w).as_matrix(), atol=1e-14)
        y = np.concatenate([w / C.S_OMEGA, r.normal(size=3)])
        np.testing.assert_allclose(C.pose_target(C.proposal_pose(y)), y, atol=1e-12)
    assert np.array_equal(C.pose_target(np.eye(4)), np.zeros(6))


def test_network_input_values_and_subsampling():
    rng = np.full((64, 512), 2.0, dtype=np.float32)
    rng[0, 0] = 0.0
    rng[2, 4] = 60.0
    rng[4, 2] = np.inf
    rng[6, 8] = 4.0
    rng[1, 1] = 0.0  # not sampled (odd row / column)
    x = C.network_input(rng, rng)
    assert x.shape == (32, 256, 2)
    assert x[0, 0, 0] == 0.0 and x[1, 2, 1] == 0.0 and x[2, 1, 0] == 0.0
    assert x[3, 4, 1] == 0.25 and x[5, 5, 0] == 0.5
    assert np.count_nonzero(x == 0.5) == 2 * 32 * 256 - 2 * 4
