"""Periodic cubic B-spline interpolation with exact prefiltering.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper integrates with cubic interpolation at off-grid points (Section 3.1)
and implements it as a cubic interpolator with prefiltering after Ruijters et al.
(Section 4.2).  Boundary conditions are not stated; they are taken periodic, as
the spectral operators are.

* Prefilter: the interpolating coefficients c of samples f satisfy
  sum_m c[i - m] beta3(m) = f[i]; on the periodic grid this is a circulant
  system, solved here by division in Fourier space by
  prod_j (2 + cos(omega_j)) / 3, the DFT of the sampled kernel (1/6, 4/6, 1/6).
* Evaluation: q(p) = sum over the 4^d nodes around p of
  prod_j beta3(p_j - n_j) c[n mod N], with beta3 the centred cubic B-spline
  written out from its piecewise definition; the gradient uses beta3'.

Points are given in grid-index units (node i sits at i).
"""
from __future__ import annotations

import itertools
import math

import torch

from .spectral import DT, CT, as_t


def beta3(x: torch.Tensor) -> torch.Tensor:
    """Centred cubic B-spline: 2/3 - x^2 + |x|^3/2 on |x|<1, (2-|x|)^3/6 on 1<=|x|<2, 0 beyond."""
    ax = x.abs()
    inner = 2.0 / 3.0 - ax ** 2 + 0.5 * ax ** 3
    outer = (2.0 - ax) ** 3 / 6.0
    return torch.where(ax < 1.0, inner, torch.where(ax < 2.0, outer, torch.zeros_like(ax)))


def dbeta3(x: torch.Tensor) -> torch.Tensor:
    """Derivative of beta3."""
    ax = x.abs()
    sg = torch.sign(x)
    inner = -2.0 * x + 1.5 * x * ax
    outer = -0.5 * sg * (2.0 - ax) ** 2
    return torch.where(ax < 1.0, inner, torch.where(ax < 2.0, outer, torch.zeros_like(ax)))


def prefilter(f, d: int) -> torch.Tensor:
    """Interpolating cubic B-spline coefficients of periodic samples f [..., N] (exact, FFT division)."""
    f = as_t(f)
    N = f.shape[-d:]
    F = torch.fft.fftn(f.to(CT), dim=tuple(range(-d, 0)))
    for j, n in enumerate(N):
        om = 2 * math.pi * torch.arange(n, dtype=DT) / n
        shape = [1] * d
        shape[j] = n
        F = F / ((2.0 + torch.cos(om)) / 3.0).reshape(shape).to(CT)
    return torch.fft.ifftn(F, dim=tuple(range(-d, 0))).real.contiguous()


def evaluate(coef, pts, grad: bool = False):
    """Evaluate the spline with coefficients coef [*N] at points pts [d, *S] (grid units).

    Returns the values [*S], and with grad=True also the derivatives with
    respect to the grid coordinates [d, *S].
    """
    coef = as_t(coef)
    pts = as_t(pts)
    d = pts.shape[0]
    N = coef.shape[-d:]
    flat = coef.reshape(-1)
    strides = [math.prod(N[j + 1:]) for j in range(d)]
    base = torch.floor(pts)
    t = pts - base
    base = base.to(torch.int64)
    idx, w, dw = [], [], []
    for j in range(d):
        idx.append([((base[j] + a) % N[j]) * strides[j] for a in (-1, 0, 1, 2)])
        w.append([beta3(t[j] - a) for a in (-1, 0, 1, 2)])
        if grad:
            dw.append([dbeta3(t[j] - a) for a in (-1, 0, 1, 2)])
    val = torch.zeros(pts.shape[1:], dtype=DT)
    gr = [torch.zeros(pts.shape[1:], dtype=DT) for _ in range(d)] if grad else None
    for taps in itertools.product(range(4), repeat=d):
        lin = sum(idx[j][taps[j]] for j in range(d))
        cv = flat[lin]
        wt = w[0][taps[0]]
        for j in range(1, d):
            wt = wt * w[j][taps[j]]
        val = val + wt * cv
        if grad:
            for g in range(d):
                wg = dw[g][taps[g]] if g == 0 else w[0][taps[0]]
                for j in range(1, d):
                    wg = wg * (dw[j][taps[j]] if j == g else w[j][taps[j]])
                gr[g] = gr[g] + wg * cv
    if grad:
        return val, torch.stack(gr, 0)
    return val


def grid_index(N) -> torch.Tensor:
    """Node coordinates in grid units, [d, *N]."""
    return torch.stack(torch.meshgrid(*[torch.arange(n, dtype=DT) for n in N], indexing="ij"), 0)


def interp_samples(f, disp, d: int) -> torch.Tensor:
    """P(f) o X: spline interpolant of the samples f [*N] at X = x + disp (disp [d, *N], grid units)."""
    f = as_t(f)
    N = f.shape[-d:]
    return evaluate(prefilter(f, d), grid_index(N) + disp)
