"""Gauss-Newton-Krylov driver, metrics and Jacobian determinant.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Section 2.2 (eqs. BLNewton and BLKKT): v~ <- v~ + eps dv~ with dv~ from
preconditioned conjugate gradients on H dv~ = -g, preconditioner L~^{-1}, and
Section 4.3 (at most 10 Gauss-Newton iterations and 5 PCG iterations).  The
paper does not give the update length rule, the PCG tolerance or the stopping
test; the readings used here are:
* PCG in the l^2 coefficient inner product from dv~ = 0, stopped when
  ||r|| <= eta_k ||g|| with eta_k = min(0.5, sqrt(||g_k|| / ||g_0||)), at the
  iteration cap, or on non-positive curvature p^T H p <= 0 (truncated CG; on
  the first iteration the preconditioned steepest-descent direction is taken);
* eps by Armijo backtracking from 1, halving at most 10 times, accepting when
  E(v~ + eps dv~) <= E(v~) + 1e-4 eps <g, dv~>;
* stop when ||g||_inf <= tol ||g_ref||_inf (the relative gradient of Section 5.1.1),
  with ||g||_inf the maximum over grid nodes and components of |iota(g)|; with
  fixed iterations every cap is run to the end (PCG still stops on negative
  curvature).
Metrics (Section 5.1.1): MSE_rel = ||m(1) - I1||^2 / ||I0 - I1||^2 and the
relative gradient.  The Jacobian determinant is det(I - D iota(u~(1))) of
phi(1) = id - iota(u~(1)), with the displacement from the deformation state
equation (Sections 2.3.2-2.3.3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import torch

from . import spectral as sp
from . import semilag
from .problem import Problem


def grad_inf(g, prob: Problem) -> float:
    return float(sp.include(g, prob.N).abs().max())


def pcg(matvec, b, precond, tol: float, maxit: int, fixed: bool = False, flexible: bool = False, dot=None):
    """Preconditioned CG from 0 for A x = b.  Returns (x, iterations, flag, rnorm).

    flag: 0 converged/cap, 3 non-positive curvature.  flexible: the direction update
    beta = r_new . (z_new - z_old) / r_old . z_old (flexible CG, for a preconditioner that is itself an
    iteration); it equals the PCG update when the preconditioner is a fixed SPD operator.  dot: the inner
    product (default: the l^2 product of the coefficients).
    """
    ip = dot if dot is not None else sp.l2
    x = torch.zeros_like(b)
    r = b.clone()
    z = precond(r)
    p = z.clone()
    rz = float(ip(r, z))
    it = 0
    flag = 0
    for it in range(maxit):
        rn = math.sqrt(float(ip(r, r)))
        if not fixed and rn <= tol:
            return x, it, flag, rn
        Ap = matvec(p)
        pAp = float(ip(p, Ap))
        if pAp <= 0.0:
            flag = 3
            if it == 0:
                x = p.clone()
            return x, it, flag, rn
        a = rz / pAp
        x = x + a * p
        r = r - a * Ap
        z_old = z
        z = precond(r)
        rz_new = float(ip(r, z))
        num = rz_new - float(ip(r, z_old)) if flexible else rz_new
        p = z + (num / rz) * p
        rz = rz_new
    return x, maxit, flag, math.sqrt(float(ip(r, r)))


@dataclass
class GNReport:
    gn_iters: int = 0
    pcg_iters_total: int = 0
    backtracks: int = 0
    E0: float = 0.0
    E: float = 0.0
    mse_rel: float = 0.0
    grad_inf_rel: float = 0.0
    status: int = 0
    history: List[dict] = field(default_factory=list)

    @property
    def decisions(self):
        """Per GN iteration: (PCG iterations, 1 if PCG stopped on non-positive curvature, Armijo backtracks
        before the accepted step or -1 when none was accepted): the discrete branches of the driver."""
        return [(h["pcg"], 1 if h["flag"] == 3 else 0, h["backtracks"] if h["accepted"] else -1)
                for h in self.history]


def gauss_newton(model, v0, max_gn=10, max_pcg=5, grad_rtol=1e-3, grad_ref_inf=0.0,
                 fixed_iters=False, precond=None):
    """Gauss-Newton-Krylov on the BL energy.  model: a variant instance.  precond: r -> M^-1 r; one with a
    set_velocity(v) method is re-linearised at every GN iteration, one with flexible = True runs flexible CG."""
    p = model.p
    if precond is None:
        precond = lambda r: sp.apply_L(r, p.d, p.alpha, p.s, inverse=True)
    flexible = bool(getattr(precond, "flexible", False))
    ip = getattr(model, "inner", sp.l2)   # a non-stationary model's node-field inner product
    v = sp.as_t(v0).clone()
    model.setup(v)
    model.state()
    E = float(model.objective()[0])
    rep = GNReport(E0=E)
    model.adjoint()
    g = model.gradient()
    ginf = grad_inf(g, p)
    ref = grad_ref_inf if grad_ref_inf > 0 else ginf
    gnorm0 = math.sqrt(float(ip(g, g)))
    for k in range(max_gn):
        if not fixed_iters and ginf <= grad_rtol * ref:
            break
        gnorm = math.sqrt(float(ip(g, g)))
        eta = min(0.5, math.sqrt(gnorm / gnorm0)) if gnorm0 > 0 else 0.5
        if hasattr(precond, "set_velocity"):
            precond.set_velocity(v)
        dv, its, flag, _ = pcg(model.hess_matvec, -g, precond, eta * gnorm, max_pcg, fixed_iters, flexible, ip)
        rep.pcg_iters_total += its
        gd = float(ip(g, dv))
        eps = 1.0
        accepted = False
        bt0 = rep.backtracks
        for bt in range(11):
            vt = v + eps * dv
            model.setup(vt)
            model.state()
            Et = float(model.objective()[0])
            if Et <= E + 1e-4 * eps * gd:
                accepted = True
                break
            rep.backtracks += 1
            eps *= 0.5
        rep.history.append(dict(iter=k, E=E, grad_inf=ginf, pcg=its, flag=flag, eps=eps if accepted else 0.0,
                                accepted=accepted, backtracks=rep.backtracks - bt0))
        if not accepted:
            model.setup(v)
            model.state()
            rep.status = 2
            break
        v, E = vt, Et
        model.adjoint()
        g = model.gradient()
        ginf = grad_inf(g, p)
        rep.gn_iters = k + 1
    rep.E = E
    rep.grad_inf_rel = ginf / ref if ref > 0 else 0.0
    m1 = model.m[-1] if hasattr(model, "m") else model.m1
    rep.mse_rel = float(((m1 - model.I1) ** 2).sum() / ((model.I0 - model.I1) ** 2).sum())
    return v, rep


def displacement_state(prob: Problem, v):
    """u~(1) from the deformation state equation (Table 1 row 3) at velocity v~."""
    v = sp.as_t(v)
    vgrid = sp.include(v, prob.N)
    Xb = semilag.characteristics(vgrid, prob.dt, -1)
    u = torch.zeros((prob.d,) + prob.K, dtype=sp.DT)
    for _ in range(prob.Nt):
        q = sp.include(u + 0.5 * prob.dt * v, prob.N)
        u = sp.project(semilag.interp_at(q, Xb), prob.K) + 0.5 * prob.dt * v
    return u


def jacobian_det(prob: Problem, u):
    """det(I - D iota(u~)) on the grid, [*N] (spectral derivatives, FP64)."""
    d = prob.d
    Du = sp.include(sp.jac(sp.as_t(u), d), prob.N)          # [d, d, *N]
    A = torch.eye(d, dtype=sp.DT).reshape((d, d) + (1,) * d) - Du
    A = A.reshape(d, d, -1).permute(2, 0, 1)
    return torch.linalg.det(A).reshape(prob.N)
