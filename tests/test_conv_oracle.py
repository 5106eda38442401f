"""Pins of the corrector's CPU reference (oracle/conv_ref.py) against definitions
written as plain loops, finite differences, exact identities, a library rounding
routine and the Adam paper's first-step closed form."""
import numpy as np
import pytest

from oracle import conv_ref


def loop_conv(x, w, b):
    """Direct six-fold loop of the circular 3x3 cross-correlation."""
    n, c, h, wd = x.shape
    o = w.shape[0]
    y = np.zeros((n, o, h, wd))
    for a in range(n):
        for q in range(o):
            for i in range(h):
                for j in range(wd):
                    s = b[q]
                    for p in range(c):
                        for u in range(3):
                            for v in range(3):
                                s += w[q, p, u, v] * x[a, p, (i + u - 1) % h, (j + v - 1) % wd]
                    y[a, q, i, j] = s
    return y


def test_conv_forward_matches_loops():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 4, 5))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    assert np.allclose(conv_ref.conv3x3(x, w, b), loop_conv(x, w, b), rtol=0, atol=1e-12)


def test_conv_delta_input_reproduces_kernel():
    """A unit impulse at (i0, j0) in channel 0 gives y[o, i0-dy, j0-dx] = w[o, 0, dy+1, dx+1]."""
    rng = np.random.default_rng(1)
    w = rng.standard_normal((2, 1, 3, 3))
    x = np.zeros((1, 1, 7, 6))
    x[0, 0, 3, 2] = 1.0
    y = conv_ref.conv3x3(x, w, np.zeros(2))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            assert np.allclose(y[0, :, 3 - dy, 2 - dx], w[:, 0, dy + 1, dx + 1])
    assert np.count_nonzero(np.abs(y) > 0) == 2 * 9


def test_conv_circular_shift_equivariance():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 2, 8, 9))
    w = rng.standard_normal((3, 2, 3, 3))
    b = rng.standard_normal(3)
    y = conv_ref.conv3x3(x, w, b)
    ys = conv_ref.conv3x3(np.roll(x, (2, -3), axis=(2, 3)), w, b)
    assert np.allclose(ys, np.roll(y, (2, -3), axis=(2, 3)))


def test_conv_backward_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 3, 6, 5))
    w = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    g = rng.standard_normal((1, 2, 6, 5))
    f = lambda x_, w_, b_: float(np.sum(g * conv_ref.conv3x3(x_, w_, b_)))
    dx, dw, db = conv_ref.conv3x3_backward(x, w, g)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (0, 2, 5, 4), (0, 1, 3, 2), (0, 0, 5, 0)]:
        e = np.zeros_like(x)
        e[idx] = h
        num = (f(x + e, w, b) - f(x - e, w, b)) / (2 * h)
        assert abs(num - dx[idx]) <= 1e-7 * max(1.0, abs(num))
    for idx in [(0, 0, 0, 0), (1, 2, 2, 1), (1, 1, 0, 2)]:
        e = np.zeros_like(w)
        e[idx] = h
        num = (f(x, w + e, b) - f(x, w - e, b)) / (2 * h)
        assert abs(num - dw[idx]) <= 1e-7 * max(1.0, abs(num))
    for o in range(2):
        e = np.zeros_like(b)
        e[o] = h
        num = (f(x, w, b + e) - f(x, w, b - e)) / (2 * h)
        assert abs(num - db[o]) <= 1e-7 * max(1.0, abs(num))


def test_network_gradients_finite_differences():
    """The 4-layer corrector (ReLU between layers) on 1x4x8x8: analytic gradients of
    the MSE loss against central differences."""
    rng = np.random.default_rng(4)
    chans = [4, 5, 5, 5, 3]
    params = [(0.4 * rng.standard_normal((chans[k + 1], chans[k], 3, 3)), 0.1 * rng.standard_normal(chans[k + 1]))
              for k in range(4)]
    x = rng.standard_normal((1, 4, 8, 8))
    t = rng.standard_normal((1, 3, 8, 8))
    loss, grads = conv_ref.loss_and_grads(params, x, t)
    h = 1e-4  # central differences: truncation O(h^2) ~ 1e-11 here, rounding ~ 1e-12

    def loss_with(k, which, idx, delta):
        p = [(w.copy(), b.copy()) for w, b in params]
        arr = p[k][0] if which == 0 else p[k][1]
        arr[idx] += delta
        return conv_ref.mse(conv_ref.forward(p, x)[0], t)

    for k in range(4):
        for idx in [(0, 0, 1, 1), (chans[k + 1] - 1, chans[k] - 1, 0, 2)]:
            num = (loss_with(k, 0, idx, h) - loss_with(k, 0, idx, -h)) / (2 * h)
            assert abs(num - grads[k][0][idx]) <= 1e-7 * max(1e-3, abs(num)), (k, idx)
        num = (loss_with(k, 1, (0,), h) - loss_with(k, 1, (0,), -h)) / (2 * h)
        assert abs(num - grads[k][1][0]) <= 1e-7 * max(1e-3, abs(num))


def test_adam_first_step_and_recursion():
    """At t = 1 the bias corrections give mhat = g, vhat = g^2, so the step is
    lr * g / (|g| + eps) (Kingma & Ba, Algorithm 1); later steps follow the moment
    recursions."""
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = conv_ref.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    g2 = np.array([0.1, 0.1, 0.1])
    th2, m2, v2 = conv_ref.adam_step(th, g2, m, v, 2, lr=0.01)
    m_ref = 0.9 * 0.1 * g + 0.1 * g2
    v_ref = 0.999 * 0.001 * g * g + 0.001 * g2 * g2
    assert np.allclose(m2, m_ref) and np.allclose(v2, v_ref)
    assert np.allclose(th2, th - 0.01 * (m_ref / (1 - 0.81)) / (np.sqrt(v_ref / (1 - 0.999 ** 2)) + 1e-8))


def test_block_mean():
    rng = np.random.default_rng(5)
    a = rng.standard_normal((2, 8, 12))
    m = conv_ref.block_mean(a, 4)
    assert m.shape == (2, 2, 3)
    assert np.isclose(m.sum() * 16, a.sum())
    assert np.isclose(m[1, 1, 2], a[1, 4:8, 8:12].mean())
    assert np.allclose(conv_ref.block_mean(np.full((4, 4), 3.5)), 3.5)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(6)
    vals = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(-5, 5, 1000),
                           [1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -1 - 2.0 ** -8, 0.0, 65504.0]])
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(conv_ref.to_bf16(vals), ref)
    assert conv_ref.to_bf16([1 + 2.0 ** -8])[0] == 1.0  # tie to even
    assert conv_ref.to_bf16([1 + 3 * 2.0 ** -8])[0] == 1 + 2.0 ** -6
