"""Non-stationary velocities (Section 1.3; the NSt rows of Tables 3 and 4) for the image-transport and the
deformation-state variants, with SL-RK2.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The velocity is a band-limited field at every time node, v~_n = v~(t_n), n = 0..Nt.  The energy is eq.
LS-LDDMM / BLEnergy with the regulariser's time integral by the trapezoid rule over the nodes, and the
gradient and Gauss-Newton Hessian-vector product are fields of the nodes, the integrands of the stationary
forms taken node by node:
    image transport     (grad)_n = L~ v~_n + lambda~_n star grad~ m~_n,   (H dv)_n = L~ dv~_n + dlambda~_n star grad~ m~_n
    deformation state   (grad)_n = L~ v~_n + rho~_n - (D~u~_n)^T rho~_n,  (H dv)_n = L~ dv~_n + drho~_n - (D~u~_n)^T drho~_n.
They are gradients with respect to the L^2(0, 1) inner product of the node fields, sum_n w_n <a_n, b_n> with the
trapezoid weights w_n, which the Gauss-Newton driver uses as its inner product (`inner`).

Readings where the paper is silent:
* characteristics of a step t_n -> t_{n+1}: the scheme of Section 3.1 with the velocity at the arrival time at
  the arrival node and the velocity at the departure time at the predicted departure point,
  X* = x - dt v_{n+1}(x), X = x - dt/2 (v_{n+1}(x) + v_n(X*)) (mirrored for the backward-in-time equations:
  arrival t_n, departure t_{n+1}, +dt);
* sources along the characteristic at the departure node's time (stage 1) and the arrival node's time
  (stage 2): the deformation state's trapezoid dt/2 (v_n o X + v_{n+1}), the adjoints' div v at t_{n+1} in
  stage 1 and at t_n in stage 2, the incremental sources s_n built from dv_n;
* everything else as in oracle/variant1.py and oracle/variant3.py.
"""
from __future__ import annotations

import torch

from . import bspline, semilag
from . import spectral as sp
from .problem import velocity_grid_units
from .variant1 import Variant1
from .variant3 import Variant3


def characteristics_ns(v_arr, v_dep, dt: float, direction: int) -> torch.Tensor:
    """Departure displacements (grid units) for a step whose arrival velocity samples are v_arr and whose
    departure velocity samples are v_dep (both [d, *N])."""
    d = v_arr.shape[0]
    N = v_arr.shape[1:]
    va = velocity_grid_units(v_arr, N)
    vd = velocity_grid_units(v_dep, N)
    xs = bspline.grid_index(N) + direction * dt * va
    vstar = torch.stack([bspline.evaluate(bspline.prefilter(vd[j], d), xs) for j in range(d)], 0)
    return direction * 0.5 * dt * (va + vstar)


class _NonStationary:
    """Per-step characteristics, per-node divergence, trapezoid-weighted regulariser and inner product."""

    def setup(self, v):
        p = self.p
        self.v = sp.as_t(v)                                   # [Nt+1, d, *K]
        assert self.v.shape[0] == p.Nt + 1
        self.vgrid = [sp.include(vn, p.N) for vn in self.v]
        self.Xb = [characteristics_ns(self.vgrid[n + 1], self.vgrid[n], p.dt, -1) for n in range(p.Nt)]
        self.Xf = [characteristics_ns(self.vgrid[n], self.vgrid[n + 1], p.dt, +1) for n in range(p.Nt)]
        self.divv = [sp.include(sp.div(vn, p.d), p.N) for vn in self.v]

    def _reg(self, v):
        p = self.p
        return sum(w * 0.5 * sp.l2(sp.apply_L(vn, p.d, p.alpha, p.s), vn)
                   for w, vn in zip(p.trapezoid_weights(), v))

    def inner(self, a, b):
        """sum_n w_n <a_n, b_n>: the inner product of node fields."""
        return sum(w * sp.l2(an, bn) for w, an, bn in zip(self.p.trapezoid_weights(), a, b))

    def _L(self, v):
        p = self.p
        return torch.stack([sp.apply_L(vn, p.d, p.alpha, p.s) for vn in v], 0)

    def _heun_back(self, e_next, n):
        """One backward band-limited Heun step t_{n+1} -> t_n of -D~_t x = x star div~ v~ (grid sample of
        x_{n+1} in, band-limited x_n out)."""
        p = self.p
        fl = sp.project(e_next * self.divv[n + 1], p.K)
        a = semilag.interp_at(e_next, self.Xf[n])
        b = semilag.interp_at(sp.include(fl, p.N), self.Xf[n])
        ustar = a + p.dt * b
        return sp.project(a + 0.5 * p.dt * (b + ustar * self.divv[n]), p.K)

    def bl_adjoint_sweep(self, final):
        p = self.p
        out = [None] * (p.Nt + 1)
        out[p.Nt] = final
        for n in range(p.Nt - 1, -1, -1):
            out[n] = self._heun_back(sp.include(out[n + 1], p.N), n)
        return out


class NSVariant1(_NonStationary, Variant1):
    def state(self):
        p = self.p
        m = [self.I0]
        for n in range(p.Nt):
            m.append(semilag.interp_at(m[-1], self.Xb[n]))
        self.m = m
        self.mt = [sp.project(mn, p.K) for mn in m]
        self.G = [sp.include(sp.grad(mt, p.d), p.N) for mt in self.mt]
        return m[-1]

    def objective(self):
        p = self.p
        reg = self._reg(self.v)
        data = ((self.m[-1] - self.I1) ** 2).mean() / p.sigma2
        return reg + data, reg, data

    def adjoint(self):
        p = self.p
        lam = [None] * (p.Nt + 1)
        lam[p.Nt] = -(2.0 / p.sigma2) * (self.m[-1] - self.I1)
        for n in range(p.Nt - 1, -1, -1):
            a = semilag.interp_at(lam[n + 1], self.Xf[n])
            b = semilag.interp_at(lam[n + 1] * self.divv[n + 1], self.Xf[n])
            ustar = a + p.dt * b
            lam[n] = a + 0.5 * p.dt * (b + ustar * self.divv[n])
        self.lam = lam
        return lam

    def gradient(self):
        p = self.p
        terms = [sp.project(sp.include(sp.project(self.lam[n], p.K), p.N).unsqueeze(0) * self.G[n], p.K)
                 for n in range(p.Nt + 1)]
        return self._L(self.v) + torch.stack(terms, 0)

    def inc_state(self, dv):
        p = self.p
        dv = sp.as_t(dv)
        s = [-(self.G[n] * sp.include(dv[n], p.N)).sum(0) for n in range(p.Nt + 1)]
        f = [sp.project(sn, p.K) for sn in s]
        dm = [torch.zeros(p.K, dtype=sp.DT)]
        for n in range(p.Nt):
            q = sp.include(dm[n] + 0.5 * p.dt * f[n], p.N)
            dm.append(sp.project(semilag.interp_at(q, self.Xb[n]) + 0.5 * p.dt * s[n + 1], p.K))
        return dm

    def hess_matvec(self, dv):
        p = self.p
        dv = sp.as_t(dv)
        dm = self.inc_state(dv)
        dl = self.inc_adjoint(dm[-1])
        terms = [sp.project(sp.include(dl[n], p.N).unsqueeze(0) * self.G[n], p.K) for n in range(p.Nt + 1)]
        self.last_inc = (dm, dl)
        return self._L(dv) + torch.stack(terms, 0)


class NSVariant3(_NonStationary, Variant3):
    def state(self):
        p = self.p
        u = [torch.zeros((p.d,) + p.K, dtype=sp.DT)]
        for n in range(p.Nt):
            q = sp.include(u[n] + 0.5 * p.dt * self.v[n], p.N)
            u.append(sp.project(semilag.interp_at(q, self.Xb[n]), p.K) + 0.5 * p.dt * self.v[n + 1])
        self.u = u
        self.Du = [sp.include(sp.jac(un, p.d), p.N) for un in u]
        self.final_warp()
        return self.m1

    def objective(self):
        p = self.p
        reg = self._reg(self.v)
        data = ((self.m1 - self.I1) ** 2).mean() / p.sigma2
        return reg + data, reg, data

    def gradient(self):
        p = self.p
        terms = []
        for n in range(p.Nt + 1):
            r = sp.include(self.rho[n], p.N)
            terms.append(self.rho[n] - sp.project(self._DuT(self.Du[n], r), p.K))
        return self._L(self.v) + torch.stack(terms, 0)

    def inc_state(self, dv):
        p = self.p
        dv = sp.as_t(dv)
        s = []
        for n in range(p.Nt + 1):
            dvg = sp.include(dv[n], p.N)
            s.append(dvg - self._Du(self.Du[n], dvg))
        f = [sp.project(sn, p.K) for sn in s]
        du = [torch.zeros((p.d,) + p.K, dtype=sp.DT)]
        for n in range(p.Nt):
            q = sp.include(du[n] + 0.5 * p.dt * f[n], p.N)
            du.append(sp.project(semilag.interp_at(q, self.Xb[n]) + 0.5 * p.dt * s[n + 1], p.K))
        return du

    def hess_matvec(self, dv):
        p = self.p
        dv = sp.as_t(dv)
        du = self.inc_state(dv)
        dr = self.bl_adjoint_sweep(self.coupling(du[-1]))
        terms = []
        for n in range(p.Nt + 1):
            e = sp.include(dr[n], p.N)
            terms.append(dr[n] - sp.project(self._DuT(self.Du[n], e), p.K))
        self.last_inc = (du, dr)
        return self._L(dv) + torch.stack(terms, 0)

    def displacement_state(self):
        return self.u[-1]
