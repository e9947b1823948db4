"""FP64 reference of the learned initial guess network (test infrastructure only).

A plain convolutional network: layer l maps C_l channels to C_{l+1} with a 3x3
kernel, zero padding and a bias; ReLU follows every layer but the last.  The
loss is the mean squared error over all output values.  Gradients are the
textbook back-propagation formulas written out directly (no autodiff); the
tests check them against central finite differences.

Shapes: activations (C, H, W); weights (C_out, C_in, 3, 3); bias (C_out,).
Convolution here is the cross-correlation used by neural networks, with a
dilation d (taps d cells apart; d = 1 is the plain 3x3 stencil):
    y[co, i, j] = b[co] + sum_{ci, di, dj} w[co, ci, di, dj] x[ci, i + (di - 1) d, j + (dj - 1) d].
"""
from __future__ import annotations

import numpy as np


def _pad(x: np.ndarray, d: int) -> np.ndarray:
    c, H, W = x.shape
    xp = np.zeros((c, H + 2 * d, W + 2 * d))
    xp[:, d:d + H, d:d + W] = x
    return xp


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray | None = None, d: int = 1) -> np.ndarray:
    cin, H, W = x.shape
    cout = w.shape[0]
    xp = _pad(x, d)
    y = np.zeros((cout, H, W)) if b is None else np.repeat(np.asarray(b, float)[:, None, None], H * W).reshape(cout, H, W).copy()
    for di in range(3):
        for dj in range(3):
            patch = xp[:, di * d:di * d + H, dj * d:dj * d + W]      # x[ci, i + (di-1)d, j + (dj-1)d]
            y += np.tensordot(w[:, :, di, dj], patch, axes=([1], [0]))
    return y


def conv3x3_weight_grad(x: np.ndarray, dy: np.ndarray, d: int = 1) -> np.ndarray:
    """dL/dw[co, ci, di, dj] = sum_{i,j} dy[co, i, j] x[ci, i + (di-1) d, j + (dj-1) d]."""
    cin, H, W = x.shape
    xp = _pad(x, d)
    g = np.zeros((dy.shape[0], cin, 3, 3))
    for di in range(3):
        for dj in range(3):
            patch = xp[:, di * d:di * d + H, dj * d:dj * d + W]
            g[:, :, di, dj] = np.tensordot(dy, patch, axes=([1, 2], [1, 2]))
    return g


def conv3x3_input_grad(dy: np.ndarray, w: np.ndarray, d: int = 1) -> np.ndarray:
    """dL/dx[ci, i, j] = sum_{co, di, dj} dy[co, i - (di-1) d, j - (dj-1) d] w[co, ci, di, dj]."""
    cout, H, W = dy.shape
    dyp = _pad(dy, d)
    dx = np.zeros((w.shape[1], H, W))
    for di in range(3):
        for dj in range(3):
            # x[i, j] meets dy[i - (di-1) d, j - (dj-1) d]
            patch = dyp[:, (2 - di) * d:(2 - di) * d + H, (2 - dj) * d:(2 - dj) * d + W]
            dx += np.tensordot(w[:, :, di, dj], patch, axes=([0], [0]))
    return dx


def init_params(channels, seed: int = 0):
    """He-style random weights (normal, std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        w = rng.standard_normal((cout, cin, 3, 3)) * np.sqrt(2.0 / (9 * cin))
        params.append((w, np.zeros(cout)))
    return params


def forward(params, x: np.ndarray, dil=None):
    """Returns the list of layer inputs (post-activation) and the output;
    dil[l] is the dilation of layer l (default 1)."""
    dil = dil or [1] * len(params)
    acts = [x]
    h = x
    for l, (w, b) in enumerate(params):
        z = conv3x3(h, w, b, dil[l])
        h = np.maximum(z, 0.0) if l < len(params) - 1 else z
        acts.append(h)
    return acts


def mse(out: np.ndarray, target: np.ndarray) -> float:
    return float(np.mean((out - target) ** 2))


def backward(params, acts, target, dil=None):
    """Gradients of the mean squared error for one sample.

    Returns (loss, [(dw, db) per layer], dx of the input)."""
    dil = dil or [1] * len(params)
    out = acts[-1]
    loss = mse(out, target)
    dz = 2.0 * (out - target) / out.size
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        w, _ = params[l]
        x = acts[l]
        grads[l] = (conv3x3_weight_grad(x, dz, dil[l]), dz.sum(axis=(1, 2)))
        dx = conv3x3_input_grad(dz, w, dil[l])
        if l > 0:
            dz = dx * (acts[l] > 0.0)        # ReLU of the previous layer
    return loss, grads, dx


def loss_and_grads_batch(params, xs, targets, dil=None):
    """Mean loss over a batch and the gradients of that mean."""
    tot = 0.0
    acc = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    for x, t in zip(xs, targets):
        loss, g, _ = backward(params, forward(params, x, dil), t, dil)
        tot += loss
        acc = [(aw + gw, ab + gb) for (aw, ab), (gw, gb) in zip(acc, g)]
    n = len(xs)
    return tot / n, [(aw / n, ab / n) for aw, ab in acc]


def adam_step(params, grads, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015); state = (t, m, v)."""
    t, m, v = state
    t += 1
    new, m2, v2 = [], [], []
    for (w, b), (gw, gb), (mw, mb), (vw, vb) in zip(params, grads, m, v):
        out = []
        for p, g, mm, vv in ((w, gw, mw, vw), (b, gb, mb, vb)):
            mm = beta1 * mm + (1 - beta1) * g
            vv = beta2 * vv + (1 - beta2) * g * g
            mh = mm / (1 - beta1 ** t)
            vh = vv / (1 - beta2 ** t)
            out.append((p - lr * mh / (np.sqrt(vh) + eps), mm, vv))
        new.append((out[0][0], out[1][0]))
        m2.append((out[0][1], out[1][1]))
        v2.append((out[0][2], out[1][2]))
    return new, (t, m2, v2)


def adam_init(params):
    z = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    return (0, z, [(a.copy(), c.copy()) for a, c in z])


def make_sample(x_prev: np.ndarray, r0: np.ndarray, x_next: np.ndarray | None, H: int, W: int,
                unit: float = 1.0):
    """Network input and target for one system of the sequence.

    r0 = b - A x_prev is the residual of the previous solution; the correction
    d = x_next - x_prev solves A d = r0.  With s = max |r0| and sx = max
    |x_prev|: input channels (r0 / s, x_prev / sx), target ((x_next - x_prev)
    unit) / s, on the H x W grid (x index fastest); a zero scale gives a zero
    channel.  Returns (input (2, H, W), target (1, H, W) or None, s)."""
    r0 = np.asarray(r0, np.float64)
    xp = np.asarray(x_prev, np.float64)
    s = float(np.max(np.abs(r0))) if r0.size else 0.0
    sx = float(np.max(np.abs(xp))) if xp.size else 0.0
    c0 = r0 / s if s > 0.0 else np.zeros_like(r0)
    c1 = xp / sx if sx > 0.0 else np.zeros_like(xp)
    inp = np.stack([c0, c1]).reshape(2, H, W)
    if x_next is None:
        tgt = None
    elif s > 0.0:
        tgt = (((np.asarray(x_next) - xp) * unit) / s).reshape(1, H, W)
    else:
        tgt = np.zeros((1, H, W))
    return inp, tgt, s


def apply_guess(x_prev: np.ndarray, out: np.ndarray, s: float, unit: float = 1.0) -> np.ndarray:
    """Initial guess from the network output: x_prev + (s / unit) out."""
    return np.asarray(x_prev) + (s / unit) * np.asarray(out, np.float64).reshape(-1)
