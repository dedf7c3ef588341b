"""Pins of the oracle's explicit Runge-Kutta comparator (deformation-state equations of Section 2.3.3 in
Eulerian form, classical RK4 in time).

* zero velocity: u~ = 0 and the adjoint is constant in time;
* constant velocity: u~(t_n) = t_n c exactly; every Fourier mode of the adjoint is multiplied per backward
  step by the RK4 stability polynomial R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 at z = 2 pi i k.c dt, and the
  incremental state obeys the RK4 recursion of y' = lam y + b, y <- R(lam dt) y + dt phi(lam dt) b with
  phi(z) = (R(z) - 1) / z, lam = -2 pi i k.c: closed forms of the scheme itself;
* the state converges at fourth order in dt;
* the optimise-then-discretise gradient and Hessian approach the exact derivatives of the discrete
  objective as dt -> 0.
"""
import math

import numpy as np
import torch

from oracle import dto, spectral as sp
from oracle.eulerian_rk import Variant3RK
from oracle.problem import Problem
from paper_2006_06823_amd import synthetic as syn
from test_oracle_transport import constant_velocity

torch.set_num_threads(min(8, torch.get_num_threads()))


def R(z):
    return 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24


def _kdotc(K, c):
    ks = torch.meshgrid(*[sp.freqs(int(k)) for k in K], indexing="ij")
    return sum(ks[j] * c[j] for j in range(len(K)))


def test_rk_zero_velocity_identity():
    prob = Problem((16, 12), (8, 8), Nt=5)
    I0, I1 = syn.blob_pair_2d(16, 0, 1.0)
    I0, I1 = I0[:, :12], I1[:, :12]
    m = Variant3RK(prob, I0, I1)
    m.setup(np.zeros((2, 8, 8)))
    m.state()
    assert all(float(u.abs().max()) == 0.0 for u in m.u)
    assert float((m.m1 - torch.tensor(I0)).abs().max()) < 1e-13
    rho = m.adjoint()
    for r in rho:
        assert float((r - rho[-1]).abs().max()) < 1e-14


def test_rk_constant_velocity_closed_forms():
    N, K, Nt = (24, 20), (10, 8), 6
    prob = Problem(N, K, Nt=Nt)
    c = (0.037, -0.021)
    I0, I1 = syn.blob_pair_2d(24, 1, 2.0)
    I0, I1 = I0[:, :20], I1[:, :20]
    m = Variant3RK(prob, I0, I1)
    m.setup(constant_velocity(K, c))
    m.state()
    for n, u in enumerate(m.u):
        ref = torch.tensor(constant_velocity(K, (n * prob.dt * c[0], n * prob.dt * c[1])))
        assert float((u - ref).abs().max()) < 1e-14
    # adjoint: per backward step each mode times R(2 pi i k.c dt)
    rho = m.adjoint()
    z = 2j * math.pi * _kdotc(K, c) * prob.dt
    top = sp.to_complex(rho[-1], 2)
    for n in range(Nt + 1):
        expect = top * (R(z) ** (Nt - n)).unsqueeze(0)
        got = sp.to_complex(rho[n], 2)
        assert float((got - expect).abs().max()) <= 1e-12 * float(top.abs().max())
    # incremental state: y' = lam y + b per mode, lam = -2 pi i k.c (D~u~ = 0 at every time)
    dv = torch.tensor(syn.random_bl_coefficients(2, K, 5))
    du = m.inc_state(dv)
    lam = -2j * math.pi * _kdotc(K, c)
    zl = lam * prob.dt
    phi = torch.where(zl.abs() > 0, (R(zl) - 1) / torch.where(zl.abs() > 0, zl, torch.ones_like(zl)),
                      torch.ones_like(zl))
    b = sp.to_complex(dv, 2)
    y = torch.zeros_like(b)
    for n in range(1, Nt + 1):
        y = R(zl).unsqueeze(0) * y + prob.dt * phi.unsqueeze(0) * b
        got = sp.to_complex(du[n], 2)
        assert float((got - y).abs().max()) <= 1e-12 * float(y.abs().max())


def _state_u1(Nt, v, prob_kw):
    prob = Problem(Nt=Nt, **prob_kw)
    I0 = np.zeros(prob.N)
    m = Variant3RK(prob, I0, I0)
    m.setup(v)
    m.state()
    return m.u[-1]


def test_rk_state_fourth_order_in_dt():
    kw = dict(N=(32, 32), K=(12, 12))
    v = torch.tensor(syn.random_bl_coefficients(2, (12, 12), 3))
    v = v * (0.15 / float(sp.include(v, (32, 32)).abs().max()))     # 0.15 of the torus per unit time
    ref = _state_u1(64, v, kw)
    e4 = float((_state_u1(4, v, kw) - ref).norm())
    e8 = float((_state_u1(8, v, kw) - ref).norm())
    assert e4 / e8 > 12.0


def _otd_dto_gaps(Nt):
    n, K = 32, 8
    prob = Problem((n, n), (K, K), Nt=Nt)
    I0, I1 = syn.blob_pair_2d(n, 2, 2.0)
    v = torch.tensor(syn.random_bl_coefficients(2, (K, K), 1))
    v = v * (0.05 / float(sp.include(v, prob.N).abs().max()))
    m = Variant3RK(prob, I0, I1)
    m.setup(v)
    m.state()
    m.adjoint()
    g = m.gradient()
    gd = dto.gradient(Variant3RK(prob, I0, I1), v)
    x = torch.tensor(syn.random_bl_coefficients(2, (K, K), 3))
    h = m.hess_matvec(x)
    hd = dto.gn_hessian_matvec(Variant3RK(prob, I0, I1), v, x)
    return float((g - gd).norm() / gd.norm()), float((h - hd).norm() / hd.norm())


def test_rk_otd_converges_to_dto_in_dt():
    g4, h4 = _otd_dto_gaps(4)
    g16, h16 = _otd_dto_gaps(16)
    assert g4 < 2e-2 and h4 < 2e-2
    assert g16 < 0.35 * g4 and h16 < 0.35 * h4
