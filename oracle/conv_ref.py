"""CPU reference of the learned corrector -- TEST INFRASTRUCTURE ONLY.

Double-precision numpy versions of the pieces the GPU computes for the coarse-grid
corrector: the 4x4 block-mean downsampling of fine fields, the 3x3 convolution with
circular padding (cross-correlation, as in common deep-learning convention), ReLU,
the mean-squared-error loss, the analytic backward pass, and the Adam update
(Kingma & Ba, "Adam: A Method for Stochastic Optimization", ICLR 2015,
Algorithm 1).  Only tests and benchmarks import this module; it shares no code
with the GPU path.

Layouts: activations are [batch, channels, H, W]; weights are
[c_out, c_in, 3, 3]; biases [c_out].  Each function states what it computes in
plain loops or a direct sum over the nine taps (the channel contractions of each
tap go through numpy's einsum with BLAS, in double precision).

Parity: conv3x3 / its backward are pinned by a pure-Python loop on tiny inputs,
by central finite differences of the loss, by the delta-input identity and by
circular-shift equivariance (tests/test_conv_oracle.py).
"""
from __future__ import annotations

import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]  # tap t = (dy+1)*3 + (dx+1)


def block_mean(a: np.ndarray, f: int = 4) -> np.ndarray:
    """Mean over non-overlapping f x f blocks of the last two axes."""
    *lead, h, w = a.shape
    assert h % f == 0 and w % f == 0
    return a.reshape(*lead, h // f, f, w // f, f).mean(axis=(-3, -1))


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[n,o,i,j] = b[o] + sum_{c,dy,dx} w[o,c,dy+1,dx+1] x[n,c,(i+dy) mod H,(j+dx) mod W]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    y = np.zeros((x.shape[0], w.shape[0], x.shape[2], x.shape[3]))
    for dy, dx in TAPS:
        xs = np.roll(x, shift=(-dy, -dx), axis=(2, 3))  # xs[..., i, j] = x[..., i+dy, j+dx]
        y += np.einsum("oc,ncij->noij", w[:, :, dy + 1, dx + 1], xs, optimize=True)
    return y + np.asarray(b, np.float64)[None, :, None, None]


def conv3x3_backward(x, w, dy_out):
    """Gradients (dx, dw, db) of sum(dy_out * conv3x3(x, w, b)) with respect to x, w, b."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    g = np.asarray(dy_out, np.float64)
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for dy, dxx in TAPS:
        xs = np.roll(x, shift=(-dy, -dxx), axis=(2, 3))
        dw[:, :, dy + 1, dxx + 1] = np.einsum("noij,ncij->oc", g, xs, optimize=True)
        # y[i] uses x[i+dy]: the gradient flows back to x[i+dy] = shift g by +dy
        dx += np.roll(np.einsum("oc,noij->ncij", w[:, :, dy + 1, dxx + 1], g, optimize=True), shift=(dy, dxx),
                      axis=(2, 3))
    db = g.sum(axis=(0, 2, 3))
    return dx, dw, db


def relu(x):
    return np.maximum(x, 0.0)


def forward(params, x):
    """4-layer corrector: conv -> ReLU -> conv -> ReLU -> conv -> ReLU -> conv.
    params: list of (w, b).  Returns the output and the list of layer inputs."""
    acts = [np.asarray(x, np.float64)]
    h = acts[0]
    for k, (w, b) in enumerate(params):
        h = conv3x3(h, w, b)
        if k < len(params) - 1:
            h = relu(h)
            acts.append(h)
    return h, acts


def mse(out, target):
    return float(np.mean((np.asarray(out, np.float64) - target) ** 2))


def loss_and_grads(params, x, target):
    """MSE loss and its gradients with respect to every (w, b)."""
    out, acts = forward(params, x)
    g = 2.0 * (out - target) / out.size
    grads = [None] * len(params)
    for k in range(len(params) - 1, -1, -1):
        w, _ = params[k]
        dx, dw, db = conv3x3_backward(acts[k], w, g)
        grads[k] = (dw, db)
        if k > 0:
            g = dx * (acts[k] > 0)
    return mse(out, target), grads


def adam_step(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def to_bf16(a):
    """Round float values to bfloat16 (round to nearest, ties to even) and back."""
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out).astype(np.float64)
