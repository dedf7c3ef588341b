"""Band-limited vector-field space (Section 2.2, 'Parameterization in the space of band-limited vector fields').

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper works with the truncated discrete Fourier domain Omega~ with bounds
K_1..K_d, the inclusion iota: V~ -> V, the projection pi: V -> V~, the
projected operators written with a tilde, the truncated convolution (star) and
the metric <L~ v~, w~>_{l^2}.  It leaves the domain extent, the Fourier
normalisation and the exact band unstated; the readings used here are:

* Domain: the periodic unit torus [0,1)^d, nodes x = i / N_j; the L^2 inner
  product is the grid mean (1/prod N) sum_x.
* Band: per axis the frequencies |k_j| <= h_j = K_j/2 - 1, held in K_j real
  slots: slot 0 the constant, slots 2k-1 / 2k the functions sqrt(2) cos(2 pi k x)
  / sqrt(2) sin(2 pi k x) (k = 1..h_j), and slot K_j - 1 an always-zero pad.  The
  unpaired -K_j/2 frequency is dropped so that iota is real and iota o pi is an
  orthogonal projector.  The d-dimensional basis is the tensor product.
* With this orthonormal basis the paper's complex coefficients are
  c^(k) = (c_cos - i c_sin)/sqrt(2), c^(-k) = conj, per axis; the l^2 metric on
  the real coefficients equals the L^2(Omega) metric of the fields (Parseval).
* Spectral operators act on c^ by their Fourier symbols: d/dx_j -> 2 pi i k_j,
  Laplacian -> -(2 pi)^2 |k|^2, L = (Id - alpha Laplacian)^s (Section 2.1) ->
  (1 + alpha (2 pi)^2 |k|^2)^s.
* Truncated convolution: a star b = pi(iota(a) iota(b)).

Here iota and pi are computed with complex FFTs on the N grid plus cropping or
zero padding; the real/complex basis change is an explicit per-axis matrix.
"""
from __future__ import annotations

import math
from functools import lru_cache

import torch

DT = torch.float64
CT = torch.complex128


def as_t(x):
    """Convert to a float64 CPU tensor (no copy when already one)."""
    if isinstance(x, torch.Tensor):
        return x.to(dtype=DT)
    return torch.as_tensor(x, dtype=DT)


def half_band(K: int) -> int:
    """h = K/2 - 1: largest frequency held by a band of K (even) slots."""
    if K < 2 or K % 2:
        raise ValueError(f"band size must be even and >= 2, got {K}")
    return K // 2 - 1


@lru_cache(maxsize=None)
def _axis_T(K: int) -> torch.Tensor:
    """Complex change of basis for one axis: c^(k) = sum_a T[k + h, a] c_a."""
    h = half_band(K)
    T = torch.zeros(2 * h + 1, K, dtype=CT)
    T[h, 0] = 1.0
    r = 1.0 / math.sqrt(2.0)
    for k in range(1, h + 1):
        T[h + k, 2 * k - 1] = r
        T[h + k, 2 * k] = -1j * r
        T[h - k, 2 * k - 1] = r
        T[h - k, 2 * k] = 1j * r
    return T


def freqs(K: int) -> torch.Tensor:
    h = half_band(K)
    return torch.arange(-h, h + 1, dtype=DT)


def to_complex(c: torch.Tensor, d: int) -> torch.Tensor:
    """Real-basis coefficients [..., K_1..K_d] -> complex Fourier block [..., 2h_1+1, ..]."""
    K = c.shape[-d:]
    out = c.to(CT)
    for j in range(d):
        ax = out.ndim - d + j
        out = torch.movedim(torch.tensordot(out, _axis_T(int(K[j])), dims=([ax], [1])), -1, ax)
    return out


def from_complex(ch: torch.Tensor, K) -> torch.Tensor:
    """Inverse of to_complex (the columns of T are orthonormal); returns the real part."""
    d = len(K)
    out = ch
    for j in range(d):
        ax = out.ndim - d + j
        T = _axis_T(int(K[j]))
        out = torch.movedim(torch.tensordot(out, T.conj(), dims=([ax], [0])), -1, ax)
    return out.real.contiguous()


def _freq_index(K, N):
    idx = []
    for Kj, Nj in zip(K, N):
        h = half_band(int(Kj))
        if 2 * h + 1 > Nj:
            raise ValueError(f"grid {Nj} too small for band {Kj}")
        idx.append(torch.arange(-h, h + 1) % Nj)
    return torch.meshgrid(*idx, indexing="ij")


def include(c, N) -> torch.Tensor:
    """iota: band-limited coefficients [..., K] -> samples on the grid [..., N] (Section 2.2)."""
    c = as_t(c)
    N = tuple(int(n) for n in N)
    d = len(N)
    K = tuple(int(k) for k in c.shape[-d:])
    ch = to_complex(c, d)
    F = torch.zeros(c.shape[:-d] + N, dtype=CT)
    F[(Ellipsis,) + _freq_index(K, N)] = ch
    f = torch.fft.ifftn(F, dim=tuple(range(-d, 0))) * math.prod(N)
    return f.real.contiguous()


def project(f, K) -> torch.Tensor:
    """pi: grid samples [..., N] -> band-limited coefficients [..., K] (Section 2.2).

    pi(f)_a = mean_x f(x) b_a(x): the L^2-orthogonal projection onto the band.
    """
    f = as_t(f)
    K = tuple(int(k) for k in K)
    d = len(K)
    N = tuple(int(n) for n in f.shape[-d:])
    F = torch.fft.fftn(f.to(CT), dim=tuple(range(-d, 0))) / math.prod(N)
    ch = F[(Ellipsis,) + _freq_index(K, N)]
    return from_complex(ch, K)


def _symbol_apply(c, d, sym):
    K = tuple(int(k) for k in c.shape[-d:])
    return from_complex(to_complex(c, d) * sym, K)


def _kgrid(K):
    return torch.meshgrid(*[freqs(int(k)) for k in K], indexing="ij")


def deriv(c, j: int, d: int) -> torch.Tensor:
    """Spectral partial derivative along axis j (unit-torus units) of BL coefficients."""
    c = as_t(c)
    K = c.shape[-d:]
    kj = _kgrid(K)[j]
    return _symbol_apply(c, d, 2j * math.pi * kj)


def grad(c, d: int) -> torch.Tensor:
    """nabla~ of a BL scalar [..K] -> [d, ..K]."""
    return torch.stack([deriv(c, j, d) for j in range(d)], dim=0)


def div(c, d: int) -> torch.Tensor:
    """nabla~ . of a BL vector [d, ..K] -> [..K]."""
    return sum(deriv(c[j], j, d) for j in range(d))


def jac(u, d: int) -> torch.Tensor:
    """D~ of a BL vector: [d, ..K] -> [d (component i), d (derivative j), ..K]."""
    return torch.stack([torch.stack([deriv(u[i], j, d) for j in range(d)], 0) for i in range(d)], 0)


def L_symbol(K, alpha: float, s: int) -> torch.Tensor:
    kk = _kgrid(K)
    k2 = sum(k * k for k in kk)
    return (1.0 + alpha * (2 * math.pi) ** 2 * k2) ** s


def apply_L(c, d: int, alpha: float, s: int, inverse: bool = False) -> torch.Tensor:
    """L~ = (Id - alpha Laplacian~)^s (or its inverse) on BL coefficients (Sections 2.1-2.2)."""
    c = as_t(c)
    sym = L_symbol(c.shape[-d:], alpha, s)
    if inverse:
        sym = 1.0 / sym
    return _symbol_apply(c, d, sym.to(CT))


def laplacian(c, d: int) -> torch.Tensor:
    c = as_t(c)
    kk = _kgrid(c.shape[-d:])
    k2 = sum(k * k for k in kk)
    return _symbol_apply(c, d, (-(2 * math.pi) ** 2 * k2).to(CT))


def star(a, b, N, K) -> torch.Tensor:
    """Truncated convolution a star b = pi(iota(a) iota(b)) (Section 2.2)."""
    return project(include(a, N) * include(b, N), K)


def l2(a, b) -> torch.Tensor:
    """l^2 inner product of coefficient arrays (equals the L^2 grid-mean inner product of the fields)."""
    return (as_t(a) * as_t(b)).sum()
