"""FP64 oracle of the learned pose proposal.  TEST INFRASTRUCTURE ONLY: the
product library never imports it; only the tests, the smoke check and the
benchmark's CPU-baseline leg do.

The paper finds loop-closure starting poses by a grid search over candidate
transforms (Section III-C); this project adds a small convolutional network
that proposes the starting pose of a registration from the two panoramas
instead, with plain identity-started ICP kept as the fallback.  Nothing of the
network is in the paper, so every definition below is the project's own and
is pinned against library routines (scipy, torch autograd), finite
differences and closed forms in tests/test_oracle_cnn.py.

Network.  Input: a pair of 32x256 inverse-range images (keyframe, scan),
NHWC [n][32][256][2], 0 where there is no return.  Five 3x3 convolutions
with ReLU; width (azimuth) is circular, height (elevation) is zero-padded;
(cin, cout, stride) = (2,32,2) (32,64,2) (64,96,2) (96,128,2) (128,128,1);
then a fully connected layer 4096 -> 6 giving y, with the proposed increment
omega = S_OMEGA y[0:3] (rotation vector, rad) and t = S_T y[3:6] (m) of the
scan -> keyframe pose (R = Exp(omega), t).

Conv weights are [9 cin][cout] with row (3 ky + kx) cin + ci; the FC weight
is [6][4096] over the NHWC flattening (y, x, c) of the last activation.
Parameters are flattened layer by layer: conv W, conv b, ..., FC W, FC b.

BF16 storage: the GPU keeps the input, the conv weights and every conv
activation in bfloat16 and accumulates in FP32.  With bf16=True the oracle
rounds the same tensors to bfloat16 (round to nearest even) at the same
points, so that only the accumulation differs.
"""
from __future__ import annotations

import numpy as np

ROWS, COLS = 32, 256
LAYERS = ((2, 32, 2), (32, 64, 2), (64, 96, 2), (96, 128, 2), (128, 128, 1))
OUT = 6
S_OMEGA, S_T = 0.25, 1.0


def out_hw(h, w, s):
    """Output size of a 3x3 convolution with one pixel of padding and stride s."""
    return (h - 1) // s + 1, (w - 1) // s + 1


def shapes():
    """[(h, w, cin, cout, stride)] of the five convolutions, FEAT, OUT."""
    out, h, w = [], ROWS, COLS
    for cin, cout, s in LAYERS:
        out.append((h, w, cin, cout, s))
        h, w = out_hw(h, w, s)
    return out, h * w * LAYERS[-1][1]


FEAT = shapes()[1]


def param_sizes():
    sz = []
    for cin, cout, _ in LAYERS:
        sz += [9 * cin * cout, cout]
    sz += [OUT * FEAT, OUT]
    return sz


NUM_PARAMS = int(sum(param_sizes()))


def unflatten(p):
    """Flat parameter vector -> ([(W, b)] of the convolutions, (Wfc, bfc))."""
    p = np.asarray(p, dtype=np.float64)
    assert p.size == NUM_PARAMS
    convs, o = [], 0
    for cin, cout, _ in LAYERS:
        W = p[o:o + 9 * cin * cout].reshape(9 * cin, cout)
        o += 9 * cin * cout
        b = p[o:o + cout]
        o += cout
        convs.append((W, b))
    Wfc = p[o:o + OUT * FEAT].reshape(OUT, FEAT)
    o += OUT * FEAT
    bfc = p[o:o + OUT]
    return convs, (Wfc, bfc)


def flatten(convs, fc):
    parts = []
    for W, b in convs:
        parts += [np.ravel(W), np.ravel(b)]
    parts += [np.ravel(fc[0]), np.ravel(fc[1])]
    return np.concatenate(parts)


# ---------------------------------------------------------------- bfloat16

def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even) through float32: keep the
    upper 16 bits of the float32 pattern after adding half an ulp of bf16
    (0x7FFF plus the lowest kept bit, which breaks ties towards even)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (u.astype(np.uint32) << 16).view(np.float32)
    return out.astype(np.float64).reshape(np.shape(x))


def bf16_bits(x):
    """The bfloat16 bit patterns (uint16) of bf16_round(x)."""
    r = np.ascontiguousarray(bf16_round(x).astype(np.float32))
    return (r.view(np.uint32) >> 16).astype(np.uint16)


# ------------------------------------------------------------ convolution

def _padded(x):
    """[n][h][w][c] -> [n][h+2][w+2][c]: zero rows above and below, the
    last / first column wrapped around on the left / right."""
    x = np.asarray(x, dtype=np.float64)
    xw = np.concatenate([x[:, :, -1:], x, x[:, :, :1]], axis=2)
    z = np.zeros_like(xw[:, :1])
    return np.concatenate([z, xw, z], axis=1)


def _tap_slices(ho, wo, s, ky, kx):
    return (slice(None), slice(ky, ky + s * (ho - 1) + 1, s), slice(kx, kx + s * (wo - 1) + 1, s))


def conv_forward(x, W, b, s):
    """Pre-activation z[n][ho][wo][cout] = b + sum over taps (ky, kx) and ci
    of x[n][s oy + ky - 1][(s ox + kx - 1) mod w][ci] W[(3 ky + kx) cin + ci]."""
    n, h, w, cin = x.shape
    ho, wo = out_hw(h, w, s)
    xp = _padded(x)
    z = np.zeros((n, ho, wo, W.shape[1])) + b
    for ky in range(3):
        for kx in range(3):
            t = 3 * ky + kx
            z += xp[_tap_slices(ho, wo, s, ky, kx)] @ W[t * cin:(t + 1) * cin]
    return z


def relu(z):
    return np.maximum(z, 0.0)


def conv_backward(x, y, dy, W, s):
    """Gradients of a ReLU convolution given its input x, its output y
    (after ReLU) and dL/dy.  Returns (dx, dW, db); g = dy where y > 0."""
    n, h, w, cin = x.shape
    ho, wo = y.shape[1:3]
    g = np.where(np.asarray(y) > 0, dy, 0.0)
    xp = _padded(x)
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    g2 = g.reshape(-1, g.shape[-1])
    for ky in range(3):
        for kx in range(3):
            t = 3 * ky + kx
            sl = _tap_slices(ho, wo, s, ky, kx)
            dW[t * cin:(t + 1) * cin] = xp[sl].reshape(-1, cin).T @ g2
            dxp[sl] += g @ W[t * cin:(t + 1) * cin].T
    db = g2.sum(axis=0)
    dx = dxp[:, 1:h + 1, 1:w + 1].copy()
    dx[:, :, w - 1] += dxp[:, 1:h + 1, 0]
    dx[:, :, 0] += dxp[:, 1:h + 1, w + 1]
    return dx, dW, db


# --------------------------------------------------------- head and loss

def fc_forward(f, Wfc, bfc):
    return f @ Wfc.T + bfc


def loss(y, target):
    """L = sum over samples and outputs of (y - target)^2 / (2 n)."""
    d = np.asarray(y) - np.asarray(target)
    return float((d * d).sum() / (2 * d.shape[0]))


def loss_grad(y, target):
    return (np.asarray(y) - np.asarray(target)) / y.shape[0]


def fc_backward(f, Wfc, dout):
    """(df, dWfc, dbfc) of y = f Wfc^T + bfc."""
    return dout @ Wfc, dout.T @ f, dout.sum(axis=0)


# ---------------------------------------------------------------- network

def forward(params, x, bf16=False, keep=False):
    """Network output y[n][6] for inputs x[n][32][256][2]; with keep=True also
    the list of activations [x, y1, ..., y5]."""
    convs, (Wfc, bfc) = unflatten(params)
    a = bf16_round(x) if bf16 else np.asarray(x, dtype=np.float64)
    acts = [a]
    for (W, b), (_, _, s) in zip(convs, LAYERS):
        a = relu(conv_forward(a, bf16_round(W) if bf16 else W, b, s))
        if bf16:
            a = bf16_round(a)
        acts.append(a)
    y = fc_forward(a.reshape(a.shape[0], -1), Wfc, bfc)
    return (y, acts) if keep else y


def gradients(params, x, target, bf16=False):
    """(loss, flat gradient) by backpropagation through forward()."""
    convs, (Wfc, bfc) = unflatten(params)
    y, acts = forward(params, x, bf16=bf16, keep=True)
    dout = loss_grad(y, target)
    f = acts[-1].reshape(acts[-1].shape[0], -1)
    df, dWfc, dbfc = fc_backward(f, Wfc, dout)
    d = df.reshape(acts[-1].shape)
    grads = [None] * len(LAYERS)
    for k in range(len(LAYERS) - 1, -1, -1):
        W = bf16_round(convs[k][0]) if bf16 else convs[k][0]
        dx, dW, db = conv_backward(acts[k], acts[k + 1], d, W, LAYERS[k][2])
        grads[k] = (dW, db)
        d = dx
    return loss(y, target), flatten(grads, (dWfc, dbfc))


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One step of Adam (Kingma and Ba, 2015) at step number t >= 1.
    Returns the new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------ input and output

def inverse_range(r, r_min=0.0, r_max=50.0):
    """Network input value of a range: 1/r in FP32 for a valid range, else 0,
    rounded to bfloat16 as the GPU stores it."""
    r = np.asarray(r, dtype=np.float32)
    ok = np.isfinite(r) & (r > r_min) & (r <= r_max)
    inv = np.where(ok, np.float32(1.0) / np.where(ok, r, np.float32(1.0)), np.float32(0.0)).astype(np.float32)
    return bf16_round(inv)


def network_input(kf_range, scan_range, r_min=0.0, r_max=50.0):
    """[32][256][2] input from two range images whose sizes are integer
    multiples of 32x256: pixel (y, x) takes pixel (y rows/32, x cols/256)."""
    out = np.zeros((ROWS, COLS, 2))
    for c, r in enumerate((kf_range, scan_range)):
        r = np.asarray(r)
        fy, fx = r.shape[0] // ROWS, r.shape[1] // COLS
        assert fy * ROWS == r.shape[0] and fx * COLS == r.shape[1]
        out[:, :, c] = inverse_range(r[::fy, ::fx], r_min, r_max)
    return out


def exp_so3(w):
    """Rodrigues' formula (series below 1e-8 rad)."""
    w = np.asarray(w, dtype=np.float64)
    th = float(np.linalg.norm(w))
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-8:
        return np.eye(3) + K + K @ K / 2
    return np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * K @ K


def proposal_pose(y):
    """4x4 scan -> keyframe pose proposed by the output y[6]."""
    T = np.eye(4)
    T[:3, :3] = exp_so3(S_OMEGA * np.asarray(y[:3], dtype=np.float64))
    T[:3, 3] = S_T * np.asarray(y[3:6], dtype=np.float64)
    return T


def log_so3(R):
    """Rotation vector of R (angle below pi): the skew part of R is
    sin(th) times the unit axis, the trace gives cos(th)."""
    R = np.asarray(R, dtype=np.float64)
    v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]]) / 2
    sn = float(np.linalg.norm(v))
    th = float(np.arctan2(sn, (np.trace(R) - 1) / 2))
    return v if sn < 1e-12 else v * (th / sn)


def pose_target(T):
    """Inverse of proposal_pose: y[6] = (log R / S_OMEGA, t / S_T)."""
    return np.concatenate([log_so3(np.asarray(T)[:3, :3]) / S_OMEGA, np.asarray(T)[:3, 3] / S_T])
