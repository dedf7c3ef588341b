"""Pins of the FP64 reference network of the learned warm start (oracle/convnet.py).

The convolution is pinned to torch's own 3D convolution (an independent library
implementation), the hand-written gradients to central finite differences of the
forward pass, the coefficient map to closed-form trigonometric samples, and Adam's
first step to its closed form.
"""
import math

import numpy as np
import pytest
import torch

from oracle import convnet, spectral


def _layer(rng, cin, cout, k, stride, pad, relu):
    w = rng.standard_normal((cout, cin, k, k, k)) / math.sqrt(cin * k ** 3)
    b = 0.1 * rng.standard_normal(cout)
    return convnet.Layer(w, b, stride, pad, relu)


@pytest.mark.parametrize("k,stride,pad,relu,shape", [
    (3, 1, 1, True, (2, 3, 5, 6, 7)),
    (3, 2, 1, True, (1, 2, 8, 7, 6)),
    (1, 1, 0, False, (2, 4, 3, 3, 3)),
    (3, 2, 1, False, (1, 3, 5, 5, 5)),
])
def test_conv3d_matches_library_convolution(k, stride, pad, relu, shape):
    rng = np.random.default_rng(3)
    L = _layer(rng, shape[1], 5, k, stride, pad, relu)
    x = rng.standard_normal(shape)
    y = convnet.conv3d(x, L)
    ref = torch.nn.functional.conv3d(torch.from_numpy(x), torch.from_numpy(L.w), torch.from_numpy(L.b),
                                     stride=stride, padding=pad)
    if relu:
        ref = torch.relu(ref)
    assert y.shape == tuple(ref.shape)
    np.testing.assert_allclose(y, ref.numpy(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv3d_backward_matches_finite_differences(stride):
    rng = np.random.default_rng(5)
    L = _layer(rng, 2, 3, 3, stride, 1, False)  # linear layer: differences are exact up to rounding
    x = rng.standard_normal((2, 2, 5, 4, 6))
    y = convnet.conv3d(x, L)
    dy = rng.standard_normal(y.shape)
    dx, dw, db = convnet.conv3d_backward(x, y, dy, L)
    f = lambda xx, LL: float((convnet.conv3d(xx, LL) * dy).sum())
    h = 1e-6
    for idx in [(0, 0, 0, 0, 0), (1, 1, 2, 3, 5), (0, 1, 4, 1, 2), (1, 0, 3, 3, 0)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (f(x + e, L) - f(x - e, L)) / (2 * h)
        assert abs(fd - dx[idx]) <= 1e-7 * max(1.0, abs(fd))
    for idx in [(0, 0, 0, 0, 0), (2, 1, 1, 2, 0), (1, 0, 2, 2, 2)]:
        w2 = L.w.copy()
        w2[idx] += h
        w1 = L.w.copy()
        w1[idx] -= h
        fd = (f(x, convnet.Layer(w2, L.b, stride, 1, False)) - f(x, convnet.Layer(w1, L.b, stride, 1, False))) / (2 * h)
        assert abs(fd - dw[idx]) <= 1e-7 * max(1.0, abs(fd))
    np.testing.assert_allclose(db, dy.sum(axis=(0, 2, 3, 4)), rtol=1e-12)


def test_relu_gradient_masks_inactive_outputs():
    rng = np.random.default_rng(6)
    L = _layer(rng, 2, 3, 3, 1, 1, True)
    x = rng.standard_normal((1, 2, 4, 4, 4))
    y = convnet.conv3d(x, L)
    dy = np.ones_like(y)
    _, _, db = convnet.conv3d_backward(x, y, dy, L)
    np.testing.assert_allclose(db, (y > 0).sum(axis=(0, 2, 3, 4)))


def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    channels, out_c = [3, 4], 3
    shapes = []
    cin = 2
    for i, c in enumerate(channels):
        shapes.append(c * cin * 27 + c)
        cin = c
    shapes.append(out_c * cin + out_c)
    params = 0.5 * rng.standard_normal(sum(shapes))
    layers = convnet.make_layers(params, channels, out_c)
    x = rng.standard_normal((2, 2, 8, 8, 8))
    acts = convnet.forward(x, layers)
    assert acts[-1].shape == (2, 3, 4, 4, 4)
    dout = rng.standard_normal(acts[-1].shape)
    g = convnet.backward(acts, dout, layers)
    f = lambda p: float((convnet.forward(x, convnet.make_layers(p, channels, out_c))[-1] * dout).sum())
    h = 1e-6
    for i in rng.choice(params.size, 12, replace=False):
        e = np.zeros_like(params)
        e[i] = h
        fd = (f(params + e) - f(params - e)) / (2 * h)
        # ReLU kinks are measure-zero; a sampled parameter next to one would need a smaller step
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(fd)), (i, fd, g[i])


def test_samples_to_block_closed_forms():
    s = 8
    X = np.meshgrid(*[np.arange(s) / s] * 3, indexing="ij")
    f = np.zeros((1, 3, s, s, s))
    f[0, 0] = math.sqrt(2) * np.cos(2 * np.pi * X[0])                                   # slot (1,0,0)
    f[0, 1] = 2.0 * math.sqrt(2) * np.sin(2 * np.pi * 3 * X[2]) + 0.5                     # slots (0,0,6), (0,0,0)
    f[0, 2] = 2 * np.sin(2 * np.pi * 2 * X[1]) * np.cos(2 * np.pi * X[2]) + np.cos(np.pi * s * X[0])  # + Nyquist
    blk = convnet.samples_to_block(f, s)
    exp = np.zeros_like(blk)
    exp[0, 0, 1, 0, 0] = 1.0
    exp[0, 1, 0, 0, 6] = 2.0
    exp[0, 1, 0, 0, 0] = 0.5
    exp[0, 2, 0, 4, 1] = 1.0  # sqrt2 sin(4 pi y) sqrt2 cos(2 pi z); the Nyquist term is not in the band
    np.testing.assert_allclose(blk, exp, atol=1e-13)


def test_vnorm_loss_value_and_gradient():
    rng = np.random.default_rng(9)
    s, K, alpha, sx = 8, (12, 10, 14), 0.0025, 2
    target = rng.standard_normal((2, 3) + K)
    # the symbol on the real slots: slot a holds frequency (a + 1) // 2, the last slot is a pad
    fr = [np.array([(a + 1) // 2 for a in range(Kj)], dtype=np.float64) for Kj in K]
    F = np.meshgrid(*fr, indexing="ij")
    Lw = (1.0 + alpha * (2 * np.pi) ** 2 * (F[0] ** 2 + F[1] ** 2 + F[2] ** 2)) ** sx
    pad = np.ones(K)
    for j, Kj in enumerate(K):
        sl = [slice(None)] * 3
        sl[j] = Kj - 1
        pad[tuple(sl)] = 0.0
    target = target * pad
    loss0, _ = convnet.vnorm_loss(np.zeros((2, 3, s, s, s)), target, alpha, sx)
    assert abs(loss0 - float((Lw * target ** 2).sum() / 2)) <= 1e-10 * loss0
    samples = rng.standard_normal((2, 3, s, s, s))
    loss, g = convnet.vnorm_loss(samples, target, alpha, sx)
    h = 1e-5
    for idx in [(0, 0, 0, 0, 0), (1, 2, 3, 4, 5), (0, 1, 7, 7, 7), (1, 0, 2, 6, 1)]:
        e = np.zeros_like(samples)
        e[idx] = h
        fd = (convnet.vnorm_loss(samples + e, target, alpha, sx)[0]
              - convnet.vnorm_loss(samples - e, target, alpha, sx)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, g[idx])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(11)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr = 1e-3
    p1, m, v = convnet.adam(p, g, np.zeros(50), np.zeros(50), 1, lr)
    # bias-corrected moments equal g and g^2 after one step
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_stride_schedule_for_an_output_grid():
    """The default schedule (stride 2 but the last level) is the one a requested output grid of
    in_size / 2^(levels - 1) gives; other output grids stop halving once reached, and one that halving
    cannot reach is refused.  A network with the 32^3 schedule maps 64^3 inputs to 32^3 samples."""
    ch = [16, 32, 64, 128]
    assert convnet.strides(ch) == [2, 2, 2, 1]
    assert convnet.strides(ch, 64, 8) == [2, 2, 2, 1]
    assert convnet.strides(ch, 64, 16) == [2, 2, 1, 1]
    assert convnet.strides(ch, 64, 32) == [2, 1, 1, 1]
    assert convnet.strides(ch, 64, 64) == [1, 1, 1, 1]
    with pytest.raises(ValueError):
        convnet.strides(ch, 64, 24)
    rng = np.random.default_rng(8)
    channels, out_c = [3, 4, 2], 3
    n, cin = 0, 2
    for c in channels:
        n += c * cin * 27 + c
        cin = c
    n += out_c * cin + out_c
    layers = convnet.make_layers(rng.standard_normal(n), channels, out_c, in_size=8, out_size=4)
    assert [L.stride for L in layers] == [2, 1, 1, 1]
    assert convnet.forward(rng.standard_normal((1, 2, 8, 8, 8)), layers)[-1].shape == (1, 3, 4, 4, 4)
