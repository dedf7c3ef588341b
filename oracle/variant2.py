"""BL PDE-LDDMM based on the state equation (Section 2.3.2), with SL-RK2.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The gradient and the Gauss-Newton Hessian-vector product have the form of the
original variant (Section 2.3.1):
    L~ v~ + int lambda~ star nabla~ m~ dt,   L~ dv~ + int dlambda~ star nabla~ m~ dt,
with m~ = pi(m), lambda~ = pi(lambda), but the spatial state and adjoint come
from transformations instead of transport solves:
    m(t) = I0 o phi(t),  lambda(t) = J(t) lambda(1) o psi(t),
    phi(t) = id - iota(u~(t)),  psi(t) = id - iota(nu~(t)),  J(t) = 1 - iota(U~(t)),
where u~ solves the truncated displacement state equation forward from
u~(0) = 0 and nu~, U~ solve the backward equations of eq. BLDefState from
nu~(1) = 0, U~(1) = 0.  psi(t) carries a point at time t to time 1 and J(t)
is its Jacobian determinant, so lambda(t) solves the adjoint equation
(eq. BLAdjoint) with final value lambda(1) = -(2/sigma^2)(m(1) - I1).

Readings where the paper is silent or ambiguous:
* the right-hand side of the nu~ equation is printed as -nu~_t; it is read as
  -v~_t (the equation of a map that is constant along the characteristics,
  as the u~ equation above it);
* SL forms: u~ as Table 1 row 3; nu~ and U~ are integrated backward in time
  along the mirrored characteristics, -D~_t nu~ = -v~ (a source independent of
  the unknown: the trapezoid rule) and -D~_t U~ = -div~ v~ + U~ star div~ v~
  (Heun, with the stage placement of the other band-limited adjoints);
* the incremental state is du~ (eq. BLIncDefState) and the linearised image
  at t = 1 is dm(1) = -(nabla P(I0)) o phi(1) . iota(du~(1)) (the sign of
  phi = id - iota(u~));
* the incremental adjoint of the Gauss-Newton Hessian is
  dlambda(t) = J(t) dlambda(1) o psi(t), dlambda(1) = -(2/sigma^2) dm(1): the
  solution of the adjoint equation from the incremental final value, as in
  the original variant whose incremental adjoint equation carries no dv~
  term.  The paper prints J(t) nabla lambda(1) o psi(t) . iota(dnu~(t)), the
  term of the full linearisation of lambda(t) that scales with the image
  residual and that a Gauss-Newton Hessian drops; dnu~ is therefore not
  needed;
* m(t) and lambda(t) are grid fields evaluated at every time node (cubic
  B-spline interpolation of the prefiltered I0 and lambda(1));
* trapezoid time integrals, data term and projection placement as in
  oracle/variant1.py.
"""
from __future__ import annotations

import torch

from . import bspline, semilag
from . import spectral as sp
from .problem import Problem, velocity_grid_units


class Variant2:
    def __init__(self, prob: Problem, I0, I1):
        self.p = prob
        self.I0 = sp.as_t(I0)
        self.I1 = sp.as_t(I1)
        self.cI0 = bspline.prefilter(self.I0, prob.d)

    def setup(self, v):
        p = self.p
        self.v = sp.as_t(v)
        self.vgrid = sp.include(self.v, p.N)
        self.Xb = semilag.characteristics(self.vgrid, p.dt, -1)
        self.Xf = semilag.characteristics(self.vgrid, p.dt, +1)
        self.divv = sp.include(sp.div(self.v, p.d), p.N)
        for stale in ("nu", "U", "J", "lam"):
            self.__dict__.pop(stale, None)

    def _warp(self, coef, disp_bl, grad=False):
        """P(f) o (id - iota(w~)) for prefiltered samples coef and a band-limited displacement w~."""
        p = self.p
        pts = bspline.grid_index(p.N) - velocity_grid_units(sp.include(disp_bl, p.N), p.N)
        return bspline.evaluate(coef, pts, grad=grad)

    # -- forward map phi: d_t u~ + D~u~ star v~ = v~, u~(0) = 0 (Table 1 row 3) --
    def state(self):
        p = self.p
        u = [torch.zeros((p.d,) + p.K, dtype=sp.DT)]
        for n in range(p.Nt):
            q = sp.include(u[n] + 0.5 * p.dt * self.v, p.N)
            u.append(sp.project(semilag.interp_at(q, self.Xb), p.K) + 0.5 * p.dt * self.v)
        self.u = u
        # m(t_n) = I0 o phi(t_n) at every node; g1 = (nabla P(I0)) o phi(1)
        self.m = [self._warp(self.cI0, un) for un in u[:-1]]
        m1, gidx = self._warp(self.cI0, u[-1], grad=True)
        self.m.append(m1)
        scale = torch.tensor([float(n) for n in p.N], dtype=sp.DT).reshape((-1,) + (1,) * p.d)
        self.g1 = gidx * scale
        self.mt = [sp.project(mn, p.K) for mn in self.m]
        self.G = [sp.include(sp.grad(mt, p.d), p.N) for mt in self.mt]
        self.m1 = m1
        return m1

    def objective(self):
        """eq. BLEnergy: returns (E, regulariser, data term)."""
        p = self.p
        reg = 0.5 * sp.l2(sp.apply_L(self.v, p.d, p.alpha, p.s), self.v)
        data = ((self.m1 - self.I1) ** 2).mean() / p.sigma2
        return reg + data, reg, data

    # -- inverse map psi and its Jacobian: the backward equations of eq. BLDefState --
    def inverse_state(self):
        p = self.p
        nu = [None] * (p.Nt + 1)
        U = [None] * (p.Nt + 1)
        nu[p.Nt] = torch.zeros((p.d,) + p.K, dtype=sp.DT)
        U[p.Nt] = torch.zeros(p.K, dtype=sp.DT)
        divt = sp.div(self.v, p.d)
        for n in range(p.Nt - 1, -1, -1):
            # -D~_t nu~ = -v~: trapezoid rule along the mirrored characteristic
            q = sp.include(nu[n + 1] - 0.5 * p.dt * self.v, p.N)
            nu[n] = sp.project(semilag.interp_at(q, self.Xf), p.K) - 0.5 * p.dt * self.v
            # -D~_t U~ = -div~ v~ + U~ star div~ v~: Heun
            e = sp.include(U[n + 1], p.N)
            fl = -divt + sp.project(e * self.divv, p.K)                 # stage-1 source, exact star
            a = semilag.interp_at(e, self.Xf)
            b = semilag.interp_at(sp.include(fl, p.N), self.Xf)
            ustar = a + p.dt * b                                        # predictor (grid)
            U[n] = sp.project(a + 0.5 * p.dt * (b + (-self.divv + ustar * self.divv)), p.K)
        self.nu, self.U = nu, U
        self.J = [1.0 - sp.include(Un, p.N) for Un in U]
        return nu, U

    def _pull_back(self, final):
        """J(t_n) f o psi(t_n) at every node for a grid field f given at t = 1."""
        c = bspline.prefilter(final, self.p.d)
        return [Jn * self._warp(c, nun) for Jn, nun in zip(self.J, self.nu)]

    # -- adjoint: lambda(t) = J(t) lambda(1) o psi(t) --------------------------
    def adjoint(self):
        p = self.p
        if not hasattr(self, "J"):
            self.inverse_state()
        self.lam = self._pull_back(-(2.0 / p.sigma2) * (self.m1 - self.I1))
        return self.lam

    def gradient(self):
        """L~ v~ + int_0^1 lambda~ star nabla~ m~ dt."""
        p = self.p
        g = sp.apply_L(self.v, p.d, p.alpha, p.s)
        for n, w in enumerate(p.trapezoid_weights()):
            lg = sp.include(sp.project(self.lam[n], p.K), p.N)
            g = g + w * sp.project(lg.unsqueeze(0) * self.G[n], p.K)
        return g

    # -- incremental state (eq. BLIncDefState; Table 1 row 7) -------------------
    def inc_state(self, dv):
        p = self.p
        dvg = sp.include(sp.as_t(dv), p.N)
        Du = [sp.include(sp.jac(un, p.d), p.N) for un in self.u]
        s = [dvg - (Du[n] * dvg.unsqueeze(0)).sum(1) for n in range(p.Nt + 1)]
        f = [sp.project(sn, p.K) for sn in s]
        du = [torch.zeros((p.d,) + p.K, dtype=sp.DT)]
        for n in range(p.Nt):
            q = sp.include(du[n] + 0.5 * p.dt * f[n], p.N)
            du.append(sp.project(semilag.interp_at(q, self.Xb) + 0.5 * p.dt * s[n + 1], p.K))
        return du

    def hess_matvec(self, dv):
        """Gauss-Newton H dv~ = L~ dv~ + int_0^1 dlambda~ star nabla~ m~ dt."""
        p = self.p
        dv = sp.as_t(dv)
        if not hasattr(self, "J"):
            self.inverse_state()
        du = self.inc_state(dv)
        dm1 = -(self.g1 * sp.include(du[-1], p.N)).sum(0)
        dl = self._pull_back(-(2.0 / p.sigma2) * dm1)
        h = sp.apply_L(dv, p.d, p.alpha, p.s)
        for n, w in enumerate(p.trapezoid_weights()):
            e = sp.include(sp.project(dl[n], p.K), p.N)
            h = h + w * sp.project(e.unsqueeze(0) * self.G[n], p.K)
        self.last_inc = (du, dl)
        return h

    def displacement_state(self):
        return self.u[-1]
