"""Pins of the oracle's band-limited operators (Section 2.2) against independent computations.

Each check compares against something other than the oracle's own FFT route:
brute-force sums over the real basis functions, finite differences on a fine
grid, or the product of fields evaluated on a finer grid.
"""
import itertools
import math

import numpy as np
import pytest
import torch

from oracle import spectral as sp
from paper_2006_06823_amd import synthetic as syn


def basis_1d(a, K, x):
    """Real orthonormal basis function of slot a on the unit torus, written out."""
    if a == K - 1:
        return np.zeros_like(x)
    if a == 0:
        return np.ones_like(x)
    k = (a + 1) // 2
    if a % 2 == 1:
        return math.sqrt(2.0) * np.cos(2 * math.pi * k * x)
    return math.sqrt(2.0) * np.sin(2 * math.pi * k * x)


def brute_include(c, N):
    K = c.shape
    X = syn.grid_coords(N)
    f = np.zeros(N)
    for a in itertools.product(*[range(k) for k in K]):
        b = np.ones(N)
        for j in range(len(N)):
            b = b * basis_1d(a[j], K[j], X[j])
        f += c[a] * b
    return f


def brute_project(f, K):
    N = f.shape
    X = syn.grid_coords(N)
    c = np.zeros(K)
    for a in itertools.product(*[range(k) for k in K]):
        b = np.ones(N)
        for j in range(len(N)):
            b = b * basis_1d(a[j], K[j], X[j])
        c[a] = (f * b).mean()
    return c


@pytest.mark.parametrize("N,K", [((8, 6), (4, 4)), ((7, 9), (6, 4)), ((6, 5, 4), (4, 4, 2))])
def test_include_project_match_direct_sums(N, K):
    """P1: iota / pi equal the direct sums over the real basis (brute force)."""
    rng = np.random.default_rng(1)
    c = syn.random_bl_coefficients(1, K, 3)[0]
    f = rng.standard_normal(N)
    assert np.allclose(sp.include(c, N).numpy(), brute_include(c, N), atol=1e-13)
    assert np.allclose(sp.project(f, K).numpy(), brute_project(f, K), atol=1e-13)


@pytest.mark.parametrize("N,K", [((32, 20), (16, 8)), ((12, 10, 14), (8, 6, 8))])
def test_parseval_idempotence(N, K):
    """P2: Parseval, pi o iota = Id on the band, iota o pi idempotent, pad slot stays zero."""
    rng = np.random.default_rng(2)
    c = torch.tensor(syn.random_bl_coefficients(1, K, 4)[0])
    f = sp.include(c, N)
    assert abs(float((c * c).sum() - (f * f).mean())) < 1e-13
    assert float((sp.project(f, K) - c).abs().max()) < 1e-13
    g = torch.tensor(rng.standard_normal(N))
    pg = sp.include(sp.project(g, K), N)
    assert float((sp.include(sp.project(pg, K), N) - pg).abs().max()) < 1e-13
    pc = sp.project(g, K)
    for j, k in enumerate(K):
        sl = [slice(None)] * len(K)
        sl[j] = k - 1
        assert float(pc[tuple(sl)].abs().max()) == 0.0
    # orthogonality of the residual: <g - iota pi g, iota pi g> = 0
    assert abs(float(((g - pg) * pg).mean())) < 1e-13


def test_derivative_single_mode():
    """P3: the spectral derivative of a single real mode equals the analytic derivative."""
    N, K = (24, 20), (8, 10)
    X = syn.grid_coords(N)
    for a0, a1 in [(3, 0), (4, 5), (1, 8), (6, 7)]:
        c = np.zeros(K)
        c[a0, a1] = 1.0
        k0, k1 = (a0 + 1) // 2, (a1 + 1) // 2
        # d/dx0 of basis_1d(a0)(x0) written analytically
        if a0 == 0:
            d0 = np.zeros_like(X[0])
        elif a0 % 2 == 1:
            d0 = -2 * math.pi * k0 * math.sqrt(2) * np.sin(2 * math.pi * k0 * X[0])
        else:
            d0 = 2 * math.pi * k0 * math.sqrt(2) * np.cos(2 * math.pi * k0 * X[0])
        expect = d0 * basis_1d(a1, K[1], X[1])
        got = sp.include(sp.deriv(c, 0, 2), N).numpy()
        assert np.allclose(got, expect, atol=1e-11 * (1 + k0))


def test_L_matches_finite_difference_operator():
    """P3: L~ = (Id - alpha Lap)^s agrees with the finite-difference operator and converges at O(h^2)."""
    alpha, s = 0.0025, 2
    K = (8, 8)
    c = syn.random_bl_coefficients(1, K, 7)[0]
    errs = []
    for n in (64, 128):
        f = sp.include(c, (n, n)).numpy()
        h = 1.0 / n

        def lap(g):
            return sum((np.roll(g, 1, j) - 2 * g + np.roll(g, -1, j)) / h ** 2 for j in range(2))

        Lf = f.copy()
        for _ in range(s):
            Lf = Lf - alpha * lap(Lf)
        ref = sp.include(sp.apply_L(c, 2, alpha, s), (n, n)).numpy()
        errs.append(np.abs(Lf - ref).max() / np.abs(ref).max())
    assert errs[0] < 1e-2
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_div_grad_is_laplacian_and_L_inverse():
    """P3: div~ grad~ = Lap~ and L~^{-1} L~ = Id."""
    K = (10, 8, 6)
    c = torch.tensor(syn.random_bl_coefficients(1, K, 8)[0])
    assert float((sp.div(sp.grad(c, 3), 3) - sp.laplacian(c, 3)).abs().max()) < 1e-10
    back = sp.apply_L(sp.apply_L(c, 3, 0.0025, 2), 3, 0.0025, 2, inverse=True)
    assert float((back - c).abs().max()) < 1e-13


def test_truncated_convolution_is_alias_free():
    """P4: a star b on the N grid (N > 3h) equals the projection of the product computed on a 4x finer grid."""
    K = (8, 10)
    N = (16, 20)            # N_j > 3 h_j
    a = syn.random_bl_coefficients(1, K, 11)[0]
    b = syn.random_bl_coefficients(1, K, 12)[0]
    fine = tuple(4 * n for n in N)
    ref = sp.project(sp.include(a, fine) * sp.include(b, fine), K)
    got = sp.star(a, b, N, K)
    assert float((got - ref).abs().max()) < 1e-14
