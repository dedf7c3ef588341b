"""Discretise-then-optimise shadow of the oracle's objective.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper derives its gradient and Hessian in the continuum and then
discretises them (optimise-then-discretise).  Those are not the exact
derivatives of the discrete SL-RK2 objective, so a central finite-difference
check cannot pin them to 1e-6.  This module differentiates the discrete
objective of the oracle's own forward map (characteristics, SL transport,
projections, final warp, eq. BLEnergy) exactly, by reverse-mode automatic
differentiation of the torch CPU float64 forward; the finite-difference pin
binds this gradient, and the optimise-then-discretise gradient is compared
with it under refinement.
"""
from __future__ import annotations

import torch

from . import spectral as sp


def objective(model, v) -> torch.Tensor:
    """Discrete E(v~) as a differentiable torch scalar."""
    model.setup(v)
    model.state()
    return model.objective()[0]


def gradient(model, v):
    """Exact gradient of the discrete objective with respect to the coefficients v~."""
    v = sp.as_t(v).detach().clone().requires_grad_(True)
    E = objective(model, v)
    (g,) = torch.autograd.grad(E, v)
    return g.detach()


def _residual(model, v):
    model.setup(v)
    m1 = model.state()
    return m1 - model.I1


def gn_hessian_matvec(model, v, dv):
    """Exact Gauss-Newton Hessian of the discrete objective: L~ dv + (2/sigma^2) J^T J dv / prod(N)."""
    p = model.p
    v = sp.as_t(v).detach()
    dv = sp.as_t(dv).detach()
    _, Jdv = torch.autograd.functional.jvp(lambda x: _residual(model, x), (v,), (dv,))
    _, JtJdv = torch.autograd.functional.vjp(lambda x: _residual(model, x), (v,), (Jdv,))
    nvox = float(Jdv.numel())
    return sp.apply_L(dv, p.d, p.alpha, p.s) + (2.0 / p.sigma2) * JtJdv[0] / nvox
