"""BL PDE-LDDMM based on the deformation state equation, integrated in time by an explicit Runge-Kutta
scheme on the Eulerian grid: the RK comparator of the paper's evaluation (Section 4.3 parameter
configuration, RK rows of Tables 3 and 4) beside its SL-RK2 scheme.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The equations of Section 2.3.3 in their original form, every truncated product exact and every
derivative spectral (Section 2.2):
    d_t u~    = v~ - D~u~ star v~                    forward from u~(0) = 0
    d_t rho~  = -div~(rho~ star v~)                  backward from rho~(1)  (eq. BLDefAdjoint)
    d_t du~   = dv~ - D~du~ star v~ - D~u~ star dv~   forward from du~(0) = 0
    d_t drho~ = -div~(drho~ star v~)                 backward from drho~(1) (eq. BLIncDefAdjoint)
where (D~u~ star v~)_i = sum_j d~_j u~_i star v~_j and div~(rho~ star v~)_i = sum_j d~_j (rho~_i star v~_j).

Readings where the paper is silent:
* the scheme is the classical four-stage Runge-Kutta method: the paper names no order, and the time
  steps it needs for stability (nt = 25 to 50) fit a scheme whose stability region holds a stretch of
  the imaginary axis (the spectrum of a transport operator), which a two-stage scheme's does not;
* the incremental state's coefficient D~u~ at the half step t_n + dt/2 is the mean of the two nodes'
  values (the state is kept at the nodes only); the other equations have coefficients that do not
  change in time;
* objective, final warp, final conditions, t = 1 coupling and the trapezoid time integrals of the
  gradient and Hessian terms are those of oracle/variant3.py.
"""
from __future__ import annotations

import torch

from . import spectral as sp
from .variant3 import Variant3


class Variant3RK(Variant3):
    def setup(self, v):
        p = self.p
        self.v = sp.as_t(v)
        self.vgrid = sp.include(self.v, p.N)
        self.divv = sp.include(sp.div(self.v, p.d), p.N)

    # -- right-hand sides ---------------------------------------------------------------
    def _Du_star(self, u, wgrid):
        """(D~u~ star w)_i = pi(sum_j iota(d~_j u~_i) w_j) for grid samples w of a BL vector."""
        p = self.p
        Dg = sp.include(sp.jac(u, p.d), p.N)                       # [i][j][N]
        return sp.project((Dg * wgrid.unsqueeze(0)).sum(1), p.K)

    def _rhs_state(self, u):
        return self.v - self._Du_star(u, self.vgrid)

    def _rhs_adjoint(self, r):
        """-div~(r~ star v~), component i = -sum_j d~_j pi(iota(r~_i) iota(v~_j))."""
        p = self.p
        rg = sp.include(r, p.N)
        out = []
        for i in range(p.d):
            prod = sp.project(rg[i].unsqueeze(0) * self.vgrid, p.K)  # [j][K]
            out.append(-sp.div(prod, p.d))
        return torch.stack(out, 0)

    @staticmethod
    def _rk4(y, f, h):
        """One classical RK4 step of y' = f(y) with step h (h < 0 integrates backward)."""
        k1 = f(y)
        k2 = f(y + 0.5 * h * k1)
        k3 = f(y + 0.5 * h * k2)
        k4 = f(y + h * k3)
        return y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)

    # -- state ------------------------------------------------------------------------
    def state(self):
        p = self.p
        u = [torch.zeros((p.d,) + p.K, dtype=sp.DT)]
        for _ in range(p.Nt):
            u.append(self._rk4(u[-1], self._rhs_state, p.dt))
        self.u = u
        self.Du = [sp.include(sp.jac(un, p.d), p.N) for un in u]
        self.final_warp()
        return self.m1

    # -- adjoint sweeps (the same operator for rho~ and drho~) --------------------------
    def bl_adjoint_sweep(self, final):
        p = self.p
        out = [None] * (p.Nt + 1)
        out[p.Nt] = final
        for n in range(p.Nt - 1, -1, -1):
            out[n] = self._rk4(out[n + 1], self._rhs_adjoint, -p.dt)
        return out

    # -- incremental state ----------------------------------------------------------------
    def inc_state(self, dv):
        p = self.p
        dv = sp.as_t(dv)
        dvg = sp.include(dv, p.N)
        du = [torch.zeros((p.d,) + p.K, dtype=sp.DT)]
        for n in range(p.Nt):
            u0, u1 = self.u[n], self.u[n + 1]
            uh = 0.5 * (u0 + u1)
            rhs = lambda y, uc: dv - self._Du_star(y, self.vgrid) - self._Du_star(uc, dvg)
            y = du[-1]
            h = p.dt
            k1 = rhs(y, u0)
            k2 = rhs(y + 0.5 * h * k1, uh)
            k3 = rhs(y + 0.5 * h * k2, uh)
            k4 = rhs(y + h * k3, u1)
            du.append(y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4))
        return du
