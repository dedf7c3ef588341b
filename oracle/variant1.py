"""Original BL PDE-LDDMM (image-transport state) with SL-RK2.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Section 2.3.1 ('Original BL PDE-constrained LDDMM'): gradient
L~ v~ + lambda~ star nabla~ m~, Gauss-Newton Hessian-vector product
L~ dv~ + dlambda~ star nabla~ m~, with m~ = pi(m), lambda~ = pi(lambda), the
spatial state m (eq. BLState) and adjoint lambda (eq. BLAdjoint), and the
band-limited incremental state dm~ (eq. BLIncState) and incremental adjoint
dlambda~ (eq. BLIncAdjoint) with initial conditions m(0) = I0,
lambda(1) = -(2/sigma^2)(m(1) - I1), dm~(0) = 0, dlambda~(1) = -(2/sigma^2) dm~(1).
The SL forms are Table 1 rows 1, 2, 5 and 6 (row 6 is read with dlambda~ on the
right-hand side, as in eq. BLIncAdjoint).  The energy is eq. BLEnergy.

Readings where the paper is silent:
* stationary velocity: the time integrals of the gradient and Hessian terms use
  the trapezoid rule over the Nt+1 time nodes; the regulariser is 1/2 <L~v~, v~>;
* the data term is (1/sigma^2) times the grid mean of (m(1) - I1)^2;
* m and lambda are full-grid fields and are never projected during their
  solves; each band-limited unknown (dm~, dlambda~) is projected once per step:
  in a Heun step the stage-1 source is the exact truncated product of the
  band-limited snapshot, the predictor stays a grid field and the stage-2
  source is formed on the grid and projected together with the step result.
"""
from __future__ import annotations

import torch

from . import spectral as sp
from . import semilag
from .problem import Problem


class Variant1:
    def __init__(self, prob: Problem, I0, I1):
        self.p = prob
        self.I0 = sp.as_t(I0)
        self.I1 = sp.as_t(I1)

    # -- per-velocity set-up (Section 3.1 characteristics) --------------------
    def setup(self, v):
        p = self.p
        self.v = sp.as_t(v)
        self.vgrid = sp.include(self.v, p.N)
        self.Xb = semilag.characteristics(self.vgrid, p.dt, -1)
        self.Xf = semilag.characteristics(self.vgrid, p.dt, +1)
        self.divv = sp.include(sp.div(self.v, p.d), p.N)

    # -- state (Table 1 row 1: D_t m = 0) ---------------------------------------
    def state(self):
        p = self.p
        m = [self.I0]
        for _ in range(p.Nt):
            m.append(semilag.interp_at(m[-1], self.Xb))
        self.m = m
        # projected state and its band-limited gradient, nabla~ m~ at every node
        self.mt = [sp.project(mn, p.K) for mn in m]
        self.G = [sp.include(sp.grad(mt, p.d), p.N) for mt in self.mt]
        return m[-1]

    def objective(self):
        """eq. BLEnergy: returns (E, regulariser, data term)."""
        p = self.p
        reg = 0.5 * sp.l2(sp.apply_L(self.v, p.d, p.alpha, p.s), self.v)
        data = ((self.m[-1] - self.I1) ** 2).mean() / p.sigma2
        return reg + data, reg, data

    # -- adjoint (Table 1 row 2: -D_t lambda = lambda div v) --------------------
    def adjoint(self):
        p = self.p
        lam = [None] * (p.Nt + 1)
        lam[p.Nt] = -(2.0 / p.sigma2) * (self.m[-1] - self.I1)
        f = lambda g: g * self.divv
        for n in range(p.Nt - 1, -1, -1):
            lam[n] = semilag.heun_step(lam[n + 1], f, self.Xf, p.dt)
        self.lam = lam
        return lam

    def gradient(self):
        """L~ v~ + int_0^1 lambda~ star nabla~ m~ dt (Section 2.3.1)."""
        p = self.p
        g = sp.apply_L(self.v, p.d, p.alpha, p.s)
        for n, w in enumerate(p.trapezoid_weights()):
            lg = sp.include(sp.project(self.lam[n], p.K), p.N)
            g = g + w * sp.project(lg.unsqueeze(0) * self.G[n], p.K)
        return g

    # -- incremental state (Table 1 row 5: D~_t dm~ = -nabla~ m~ star dv~) ------
    def inc_state(self, dv):
        p = self.p
        dvg = sp.include(sp.as_t(dv), p.N)
        s = [-(self.G[n] * dvg).sum(0) for n in range(p.Nt + 1)]      # grid sources
        f = [sp.project(sn, p.K) for sn in s]                            # their projections
        dm = [torch.zeros(p.K, dtype=sp.DT)]
        for n in range(p.Nt):
            # the source does not depend on the unknown: Heun reduces to the trapezoid rule
            q = sp.include(dm[n] + 0.5 * p.dt * f[n], p.N)
            dm.append(sp.project(semilag.interp_at(q, self.Xb) + 0.5 * p.dt * s[n + 1], p.K))
        return dm

    # -- incremental adjoint (Table 1 row 6: -D_t dlambda~ = dlambda~ star div~ v~) --
    def bl_adjoint_sweep(self, final):
        """Backward Heun sweep of a band-limited adjoint with source (.) star div~ v~."""
        p = self.p
        out = [None] * (p.Nt + 1)
        out[p.Nt] = final
        for n in range(p.Nt - 1, -1, -1):
            e = sp.include(out[n + 1], p.N)
            fl = sp.project(e * self.divv, p.K)                      # stage-1 source, exact star
            a = semilag.interp_at(e, self.Xf)
            b = semilag.interp_at(sp.include(fl, p.N), self.Xf)
            ustar = a + p.dt * b                                     # predictor (grid)
            out[n] = sp.project(a + 0.5 * p.dt * (b + ustar * self.divv), p.K)
        return out

    def inc_adjoint(self, dm_final):
        return self.bl_adjoint_sweep(-(2.0 / self.p.sigma2) * dm_final)

    def hess_matvec(self, dv):
        """Gauss-Newton H dv~ = L~ dv~ + int_0^1 dlambda~ star nabla~ m~ dt (Section 2.3.1)."""
        p = self.p
        dv = sp.as_t(dv)
        dm = self.inc_state(dv)
        dl = self.inc_adjoint(dm[-1])
        h = sp.apply_L(dv, p.d, p.alpha, p.s)
        for n, w in enumerate(p.trapezoid_weights()):
            e = sp.include(dl[n], p.N)
            h = h + w * sp.project(e.unsqueeze(0) * self.G[n], p.K)
        self.last_inc = (dm, dl)
        return h
