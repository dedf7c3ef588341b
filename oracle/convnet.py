"""Learned warm start: FP64 reference of the small convolutional network.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The warm start and the low-rank preconditioner are the learned additions to
the Gauss-Newton-Krylov solver (Section 2.3.1 gives the solver they feed: the
PCG system of the reduced Hessian and its initial guess).  The network is an
encoder of 3^3 convolutions (zero padding 1, ReLU; stride 2 on every level but
the last, or, for a requested output grid, stride 2 while the grid is larger than
it and 1 afterwards) on the two-channel image pair, followed by a 1^3 head
without activation.  Its output holds grid samples of the three velocity components on
a coarse s^3 grid of the unit torus; their band-limited projection onto the K=s
real basis (the exact s-point DFT without the unpaired Nyquist frequency) gives
the low-frequency block of the velocity's band-limited coefficients.  The
training loss is the squared V-norm of the coefficient error,
    loss = (1/B) sum_b sum_a L~(a) (v_pred - v*)_a^2,
with L~ = (Id - alpha Laplacian)^s diagonal on the band (Section 2.1).

Every routine here is the plain definition: a convolution is the sum over its
taps of channel contractions (a library matrix product per tap), and the
gradients are those of that sum written out by the chain rule.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from . import spectral


@dataclass
class Layer:
    w: np.ndarray  # [Cout][Cin][k][k][k]
    b: np.ndarray  # [Cout]
    stride: int
    pad: int
    relu: bool


def _out_size(n, k, stride, pad):
    return (n + 2 * pad - k) // stride + 1


def _tap_slice(t, stride, n_out):
    return slice(t, t + stride * (n_out - 1) + 1, stride)


def conv3d(x, layer: Layer):
    """y[b,o,z,y,x] = act(bias[o] + sum_{c,tap} w[o,c,tap] x_pad[b,c,stride*(z,y,x) + tap])."""
    x = np.asarray(x, dtype=np.float64)
    w = layer.w.astype(np.float64)
    B, C, D, H, W = x.shape
    k = w.shape[-1]
    p, s = layer.pad, layer.stride
    Do, Ho, Wo = (_out_size(n, k, s, p) for n in (D, H, W))
    xp = np.pad(x, ((0, 0), (0, 0), (p, p), (p, p), (p, p)))
    y = np.zeros((B, w.shape[0], Do, Ho, Wo))
    for tz in range(k):
        for ty in range(k):
            for tx in range(k):
                patch = xp[:, :, _tap_slice(tz, s, Do), _tap_slice(ty, s, Ho), _tap_slice(tx, s, Wo)]
                y += np.einsum("oc,bczyx->bozyx", w[:, :, tz, ty, tx], patch)
    y += layer.b.astype(np.float64)[None, :, None, None, None]
    if layer.relu:
        y = np.maximum(y, 0.0)
    return y


def conv3d_backward(x, y, dy, layer: Layer):
    """Gradients of conv3d at input x with output y for the upstream gradient dy.

    g = dy * act'(y); dbias = sum g; dw[o,c,tap] = sum g[b,o,.] x_pad[b,c,.+tap];
    dx_pad[b,c,.+tap] += sum_o w[o,c,tap] g[b,o,.].  Returns (dx, dw, db).
    """
    x = np.asarray(x, dtype=np.float64)
    w = layer.w.astype(np.float64)
    g = np.asarray(dy, dtype=np.float64)
    if layer.relu:
        g = g * (y > 0)
    B, C, D, H, W = x.shape
    k = w.shape[-1]
    p, s = layer.pad, layer.stride
    Do, Ho, Wo = g.shape[2:]
    xp = np.pad(x, ((0, 0), (0, 0), (p, p), (p, p), (p, p)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for tz in range(k):
        for ty in range(k):
            for tx in range(k):
                sl = (slice(None), slice(None), _tap_slice(tz, s, Do), _tap_slice(ty, s, Ho), _tap_slice(tx, s, Wo))
                dw[:, :, tz, ty, tx] = np.einsum("bozyx,bczyx->oc", g, xp[sl])
                dxp[sl] += np.einsum("oc,bozyx->bczyx", w[:, :, tz, ty, tx], g)
    dx = dxp[:, :, p:p + D, p:p + H, p:p + W]
    db = g.sum(axis=(0, 2, 3, 4))
    return dx, dw, db


def strides(channels: Sequence[int], in_size: int = 0, out_size: int = 0) -> List[int]:
    """Stride of each 3^3 level: 2 on every level but the last; with out_size, 2 while the grid
    (in_size on the first level) is larger than out_size, then 1."""
    if not out_size:
        return [2 if i < len(channels) - 1 else 1 for i in range(len(channels))]
    out, n = [], in_size
    for _ in channels:
        st = 2 if n > out_size else 1
        out.append(st)
        n = _out_size(n, 3, st, 1)
    if n != out_size:
        raise ValueError("output grid not reachable by halving the input grid")
    return out


def make_layers(params: np.ndarray, channels: Sequence[int], out_channels: int, in_size: int = 0,
                out_size: int = 0) -> List[Layer]:
    """Unpack a flat parameter vector (per layer: weights [Cout][Cin][k^3], then biases)."""
    layers, cin, o = [], 2, 0
    specs = [(c, 3, st, 1, True) for c, st in zip(channels, strides(channels, in_size, out_size))]
    specs.append((out_channels, 1, 1, 0, False))
    for cout, k, stride, pad, relu in specs:
        nw = cout * cin * k ** 3
        w = params[o:o + nw].reshape(cout, cin, k, k, k).astype(np.float64)
        b = params[o + nw:o + nw + cout].astype(np.float64)
        o += nw + cout
        layers.append(Layer(w, b, stride, pad, relu))
        cin = cout
    if o != params.size:
        raise ValueError("parameter vector does not match the architecture")
    return layers


def forward(x, layers: List[Layer]):
    """Activations of every layer (the last is the network output)."""
    acts = [np.asarray(x, dtype=np.float64)]
    for L in layers:
        acts.append(conv3d(acts[-1], L))
    return acts


def backward(acts, dout, layers: List[Layer]) -> np.ndarray:
    """Flat parameter gradient for the upstream gradient dout of the output."""
    grads = []
    g = np.asarray(dout, dtype=np.float64)
    for i in range(len(layers) - 1, -1, -1):
        dx, dw, db = conv3d_backward(acts[i], acts[i + 1], g, layers[i])
        grads.append(np.concatenate([dw.ravel(), db.ravel()]))
        g = dx
    return np.concatenate(grads[::-1])


def samples_to_block(samples, s: int):
    """Coarse grid samples [B][3][s][s][s] -> coefficients of the K=s band [B][3][s][s][s].

    This is the band-limited projection of Section 2.2 on the s^3 grid; with K = s
    the last slot of every axis is the zero pad, so the block holds the
    frequencies |k| <= s/2 - 1 per axis.
    """
    samples = np.asarray(samples, dtype=np.float64)
    return spectral.project(samples, (s, s, s)).numpy()


def embed_block(block, K):
    """Place a low coefficient block [B][3][s]^3 into a zero band [B][3][K0][K1][K2].

    A real-basis slot a < s holds the same function for every band size, so the
    block maps slot by slot.
    """
    block = np.asarray(block, dtype=np.float64)
    B, C, s = block.shape[0], block.shape[1], block.shape[2]
    out = np.zeros((B, C) + tuple(K))
    out[:, :, :s, :s, :s] = block
    return out


def vnorm_loss(samples, target_bl, alpha: float, s_exp: int):
    """Mean squared V-norm error of the predicted velocity over the batch, and its
    gradient with respect to the coarse samples.

    target_bl: [B][3][K0][K1][K2].  The prediction is zero outside the low block,
    so the target's energy there enters the loss as a constant.
    """
    samples = np.asarray(samples, dtype=np.float64)
    target = np.asarray(target_bl, dtype=np.float64)
    B, s = samples.shape[0], samples.shape[-1]
    K = target.shape[-3:]
    pred = embed_block(samples_to_block(samples, s), K)
    # L~ is diagonal on the real basis (cos and sin slots of one frequency share its symbol)
    Lw = spectral.apply_L(np.ones(K), 3, alpha, s_exp).numpy()
    diff = pred - target
    loss = float((Lw * diff * diff).sum() / B)
    dcoef = (2.0 / B) * Lw * diff
    # gradient through the projection: pi is linear, pi^T = iota / prod(s) on the s^3 grid
    dblock = dcoef[:, :, :s, :s, :s]
    dsamples = spectral.include(dblock, (s, s, s)).numpy() / float(s ** 3)
    return loss, dsamples


def adam(params, grads, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; returns new (params, m, v)."""
    m = beta1 * m + (1 - beta1) * grads
    v = beta2 * v + (1 - beta2) * grads * grads
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
