"""BL PDE-LDDMM based on the deformation state equation, with SL-RK2.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Section 2.3.3: state u~ (truncated displacement state equation
d_t u~ + D~u~ star v~ = v~, u~(0) = 0), adjoint rho~ (eq. BLDefAdjoint),
incremental state du~ and incremental adjoint drho~ (eq. BLIncDefAdjoint), with
phi(1) = id - iota(u~(1)) (Section 2.3.2) and m(1) = I0 o phi(1).  SL forms:
Table 1 rows 3, 4, 7 and 8.

Readings where the paper is silent or ambiguous:
* gradient  L~v~ + int (rho~ - (Du)^T rho~) dt, i.e. the term printed
  'D~u~ star rho~' is read as the band-limited projection of
  sum_i rho_i nabla u_i (the Lagrangian-consistent form);
* Hessian  L~dv~ + int (drho~ - (Du)^T drho~) dt: the Gauss-Newton form, which
  drops the term (D du)^T rho that is proportional to the image residual;
* the gradient of m(1) in the final conditions of rho~ and drho~ is taken as
  g1 = (nabla P(I0)) o phi(1), the exact derivative of m(1) with respect to the
  displacement; the linearised image is dm(1) = -g1 . iota(du~(1));
* trapezoid time integrals, data term and projection placement as in
  oracle/variant1.py.
"""
from __future__ import annotations

import torch

from . import bspline, semilag
from . import spectral as sp
from .problem import Problem, velocity_grid_units


class Variant3:
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

    # -- state (Table 1 row 3: D~_t u~ = v~) ------------------------------------
    def state(self):
        p = self.p
        u = [torch.zeros((p.d,) + p.K, dtype=sp.DT)]
        for n in range(p.Nt):
            # source independent of the unknown: trapezoid rule along the characteristic
            q = sp.include(u[n] + 0.5 * p.dt * self.v, p.N)
            u.append(sp.project(semilag.interp_at(q, self.Xb), p.K) + 0.5 * p.dt * self.v)
        self.u = u
        # Du_n = iota(D~ u~_n): [d (i), d (j), *N] with entry d_j u_i
        self.Du = [sp.include(sp.jac(un, p.d), p.N) for un in u]
        self.final_warp()
        return self.m1

    def final_warp(self):
        """m(1) = P(I0) o phi(1), g1 = (nabla P(I0)) o phi(1), phi(1) = x - iota(u~(1))."""
        p = self.p
        ug = velocity_grid_units(sp.include(self.u[-1], p.N), p.N)
        pts = bspline.grid_index(p.N) - ug
        m1, gidx = bspline.evaluate(self.cI0, pts, grad=True)
        scale = torch.tensor([float(n) for n in p.N], dtype=sp.DT).reshape((-1,) + (1,) * p.d)
        self.m1 = m1
        self.g1 = gidx * scale   # derivative with respect to unit-torus coordinates

    def objective(self):
        p = self.p
        reg = 0.5 * sp.l2(sp.apply_L(self.v, p.d, p.alpha, p.s), self.v)
        data = ((self.m1 - self.I1) ** 2).mean() / p.sigma2
        return reg + data, reg, data

    # -- adjoint (Table 1 row 4: -D~_t rho~ = rho~ star div~ v~) ------------------
    def bl_adjoint_sweep(self, final):
        """Backward Heun sweep of a band-limited vector adjoint with source (.) star div~ v~."""
        p = self.p
        out = [None] * (p.Nt + 1)
        out[p.Nt] = final
        for n in range(p.Nt - 1, -1, -1):
            e = sp.include(out[n + 1], p.N)
            fl = sp.project(e * self.divv, p.K)
            a = semilag.interp_at(e, self.Xf)
            b = semilag.interp_at(sp.include(fl, p.N), self.Xf)
            ustar = a + p.dt * b
            out[n] = sp.project(a + 0.5 * p.dt * (b + ustar * self.divv), p.K)
        return out

    def adjoint(self):
        p = self.p
        final = sp.project(-(2.0 / p.sigma2) * (self.m1 - self.I1) * self.g1, p.K)
        self.rho = self.bl_adjoint_sweep(final)
        return self.rho

    @staticmethod
    def _DuT(Du, r):
        """(Du)^T r: component j = sum_i r_i d_j u_i."""
        return (Du * r.unsqueeze(1)).sum(0)

    @staticmethod
    def _Du(Du, w):
        """(Du) w: component i = sum_j d_j u_i w_j."""
        return (Du * w.unsqueeze(0)).sum(1)

    def gradient(self):
        p = self.p
        g = sp.apply_L(self.v, p.d, p.alpha, p.s)
        for n, w in enumerate(p.trapezoid_weights()):
            r = sp.include(self.rho[n], p.N)
            g = g + w * (self.rho[n] - sp.project(self._DuT(self.Du[n], r), p.K))
        return g

    # -- incremental state (Table 1 row 7: D~_t du~ = dv~ - D~u~ star dv~) ------
    def inc_state(self, dv):
        p = self.p
        dvg = sp.include(sp.as_t(dv), p.N)
        s = [dvg - self._Du(self.Du[n], dvg) for n in range(p.Nt + 1)]
        f = [sp.project(sn, p.K) for sn in s]
        du = [torch.zeros((p.d,) + p.K, dtype=sp.DT)]
        for n in range(p.Nt):
            q = sp.include(du[n] + 0.5 * p.dt * f[n], p.N)
            du.append(sp.project(semilag.interp_at(q, self.Xb) + 0.5 * p.dt * s[n + 1], p.K))
        return du

    def coupling(self, du_final):
        """drho~(1) = pi(-(2/sigma^2) dm(1) g1), dm(1) = -g1 . iota(du~(1))."""
        p = self.p
        dm1 = -(self.g1 * sp.include(du_final, p.N)).sum(0)
        return sp.project(-(2.0 / p.sigma2) * dm1 * self.g1, p.K)

    def hess_matvec(self, dv):
        p = self.p
        dv = sp.as_t(dv)
        du = self.inc_state(dv)
        dr = self.bl_adjoint_sweep(self.coupling(du[-1]))
        h = sp.apply_L(dv, p.d, p.alpha, p.s)
        for n, w in enumerate(p.trapezoid_weights()):
            e = sp.include(dr[n], p.N)
            h = h + w * (dr[n] - sp.project(self._DuT(self.Du[n], e), p.K))
        self.last_inc = (du, dr)
        return h

    def displacement_state(self):
        return self.u[-1]
