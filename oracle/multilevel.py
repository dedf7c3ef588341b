"""Two-level spectral preconditioner for the Gauss-Newton PCG.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper preconditions PCG with L~^-1 (Section 2.2, eqs. BLNewton / BLKKT) and names, in its
Discussion, the multi-level preconditioner of the Claire software (Mang et al. 2019) as the step to take
next; it gives no formula.  The reading implemented here is the two-level form of that preconditioner,
built from the band-limited space:
* coarse level: the band Kc_j = 2 floor(K_j / 4) on the grid Nc_j = N_j / 2 (the first Kc_j - 1 slots of an
  axis hold the same basis functions in both bands, so restriction R keeps them and extension E pads zeros),
  with the images restricted by averages over 2^d blocks of voxels, and the same variant, Nt, alpha, s and
  sigma^2;
* M^-1 r = L~^-1 (r - E R r) + E C^-1 R r: the regularisation inverse on the frequencies above the coarse
  band and, on those inside it, the coarse problem's Gauss-Newton Hessian C at the restricted velocity R v,
  inverted approximately by a fixed number of PCG iterations from 0 preconditioned by L~_c^-1;
* an inexact inner solve is not a fixed linear operator, so the outer iteration is flexible CG.
"""
from __future__ import annotations

import torch

from . import spectral as sp
from .gauss_newton import pcg
from .problem import Problem


def coarse_sizes(N, K):
    Nc = tuple(n // 2 for n in N)
    Kc = tuple(2 * (k // 4) for k in K)
    return Nc, Kc


def restrict_image(f, d: int):
    """Mean over 2^d blocks of voxels: [N] -> [N/2]."""
    f = sp.as_t(f)
    shape = []
    for n in f.shape[-d:]:
        shape += [n // 2, 2]
    return f.reshape(shape).mean(dim=tuple(range(1, 2 * d, 2)))


def restrict_band(c, Kc):
    """Keep the slots of the coarse band's frequencies (the pad slot of the coarse band is zero)."""
    c = sp.as_t(c)
    d = len(Kc)
    idx = (Ellipsis,) + tuple(slice(0, k - 1) for k in Kc)
    out = torch.zeros(c.shape[:-d] + tuple(Kc), dtype=sp.DT)
    out[idx] = c[idx]
    return out


def extend_band(c, K):
    c = sp.as_t(c)
    d = len(K)
    Kc = c.shape[-d:]
    idx = (Ellipsis,) + tuple(slice(0, k - 1) for k in Kc)
    out = torch.zeros(c.shape[:-d] + tuple(K), dtype=sp.DT)
    out[idx] = c[idx]
    return out


class TwoLevel:
    flexible = True

    def __init__(self, model_cls, prob: Problem, I0, I1, inner: int):
        d = prob.d
        Nc, Kc = coarse_sizes(prob.N, prob.K)
        self.p = prob
        self.cp = Problem(Nc, Kc, Nt=prob.Nt, alpha=prob.alpha, s=prob.s, sigma2=prob.sigma2)
        self.coarse = model_cls(self.cp, restrict_image(I0, d), restrict_image(I1, d))
        self.inner = inner

    def set_velocity(self, v):
        self.coarse.setup(restrict_band(v, self.cp.K))
        self.coarse.state()

    def __call__(self, r):
        p, cp = self.p, self.cp
        rc = restrict_band(r, cp.K)
        Lc_inv = lambda x: sp.apply_L(x, cp.d, cp.alpha, cp.s, inverse=True)
        xc, _, _, _ = pcg(self.coarse.hess_matvec, rc, Lc_inv, 0.0, self.inner, fixed=True)
        high = r - extend_band(rc, p.K)
        return sp.apply_L(high, p.d, p.alpha, p.s, inverse=True) + extend_band(xc, p.K)
