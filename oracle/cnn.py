"""FP64 reference of the learned initial guess network (test infrastructure only).

A plain convolutional network: layer l maps C_l channels to C_{l+1} with a 3x3
kernel, zero padding and a bias; ReLU follows every layer but the last.  The
loss is the mean squared error over all output values.  Gradients are the
textbook back-propagation formulas written out directly (no autodiff); the
tests check them against central finite differences.

Shapes: activations (C, H, W); weights (C_out, C_in, 3, 3); bias (C_out,).
Convolution here is the cross-correlation used by neural networks:
    y[co, i, j] = b[co] + sum_{ci, di, dj} w[co, ci, di, dj] x[ci, i + di - 1, j + dj - 1].
"""
from __future__ import annotations

import numpy as np


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    cin, H, W = x.shape
    cout = w.shape[0]
    xp = np.zeros((cin, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((cout, H, W)) if b is None else np.repeat(np.asarray(b, float)[:, None, None], H * W).reshape(cout, H, W).copy()
    for di in range(3):
        for dj in range(3):
            patch = xp[:, di:di + H, dj:dj + W]                 # (cin, H, W)
            y += np.tensordot(w[:, :, di, dj], patch, axes=([1], [0]))
    return y


def conv3x3_weight_grad(x: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """dL/dw[co, ci, di, dj] = sum_{i,j} dy[co, i, j] x[ci, i + di - 1, j + dj - 1]."""
    cin, H, W = x.shape
    xp = np.zeros((cin, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    g = np.zeros((dy.shape[0], cin, 3, 3))
    for di in range(3):
        for dj in range(3):
            patch = xp[:, di:di + H, dj:dj + W]
            g[:, :, di, dj] = np.tensordot(dy, patch, axes=([1, 2], [1, 2]))
    return g


def conv3x3_input_grad(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """dL/dx[ci, i, j] = sum_{co, di, dj} dy[co, i - di + 1, j - dj + 1] w[co, ci, di, dj]."""
    cout, H, W = dy.shape
    dyp = np.zeros((cout, H + 2, W + 2))
    dyp[:, 1:-1, 1:-1] = dy
    dx = np.zeros((w.shape[1], H, W))
    for di in range(3):
        for dj in range(3):
            # x[i, j] meets dy[i - di + 1, j - dj + 1]
            patch = dyp[:, 2 - di:2 - di + H, 2 - dj:2 - dj + W]
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


def forward(params, x: np.ndarray):
    """Returns the list of layer inputs (post-activation) and the output."""
    acts = [x]
    h = x
    for l, (w, b) in enumerate(params):
        z = conv3x3(h, w, b)
        h = np.maximum(z, 0.0) if l < len(params) - 1 else z
        acts.append(h)
    return acts


def mse(out: np.ndarray, target: np.ndarray) -> float:
    return float(np.mean((out - target) ** 2))


def backward(params, acts, target):
    """Gradients of the mean squared error for one sample.

    Returns (loss, [(dw, db) per layer], dx of the input)."""
    out = acts[-1]
    loss = mse(out, target)
    dz = 2.0 * (out - target) / out.size
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        w, _ = params[l]
        x = acts[l]
        grads[l] = (conv3x3_weight_grad(x, dz), dz.sum(axis=(1, 2)))
        dx = conv3x3_input_grad(dz, w)
        if l > 0:
            dz = dx * (acts[l] > 0.0)        # ReLU of the previous layer
    return loss, grads, dx


def loss_and_grads_batch(params, xs, targets):
    """Mean loss over a batch and the gradients of that mean."""
    tot = 0.0
    acc = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    for x, t in zip(xs, targets):
        loss, g, _ = backward(params, forward(params, x), t)
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


def make_sample(x_prev: np.ndarray, b: np.ndarray, x_next: np.ndarray | None, H: int, W: int):
    """Network input and target for one system of the sequence.

    With s = max |b|: input channels (x_prev / s, b / s), target
    (x_next - x_prev) / s, all on the H x W grid (x index fastest).  Returns
    (input (2, H, W), target (1, H, W) or None, s)."""
    s = float(np.max(np.abs(b))) if b.size else 0.0
    if s == 0.0:
        z = np.zeros((1, H, W))
        return np.zeros((2, H, W)), (None if x_next is None else z), 0.0
    inp = np.stack([np.asarray(x_prev) / s, np.asarray(b) / s]).reshape(2, H, W)
    tgt = None if x_next is None else ((np.asarray(x_next) - np.asarray(x_prev)) / s).reshape(1, H, W)
    return inp, tgt, s


def apply_guess(x_prev: np.ndarray, out: np.ndarray, s: float) -> np.ndarray:
    """Initial guess from the network output: x_prev + s * out."""
    return np.asarray(x_prev) + s * np.asarray(out).reshape(-1)
