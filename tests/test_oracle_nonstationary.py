"""Pins of the oracle's non-stationary velocities (Section 1.3; NSt rows of Tables 3-4), image-transport and
deformation-state variants.

* a velocity that is the same at every node reproduces the stationary solves exactly, and the node fields of
  the gradient and of the Hessian-vector product (for a time-constant direction) integrate over time, with
  the trapezoid weights, to the stationary gradient and Hessian-vector product;
* a velocity constant in space but changing in time moves the departure points by the trapezoid of its two
  node values, and the deformation state is the trapezoid sum of the velocities;
* the discrete objective's exact gradient matches central finite differences, and the optimise-then-
  discretise node gradient and Hessian (divided by the node weights) approach it as dt -> 0;
* Gauss-Newton in the node-field inner product decreases the energy monotonically.
"""
import math

import numpy as np
import pytest
import torch

from oracle import dto, spectral as sp
from oracle.gauss_newton import gauss_newton
from oracle.nonstationary import NSVariant1, NSVariant3
from oracle.problem import Problem
from oracle.variant1 import Variant1
from oracle.variant3 import Variant3
from paper_2006_06823_amd import synthetic as syn
from test_oracle_transport import constant_velocity

torch.set_num_threads(min(8, torch.get_num_threads()))


def _scaled(prob, seed, cfl):
    v = torch.tensor(syn.random_bl_coefficients(prob.d, prob.K, seed))
    return v * (cfl / (float(sp.include(v, prob.N).abs().max()) * prob.dt * max(prob.N)))


@pytest.mark.parametrize("V,NSV", [(Variant1, NSVariant1), (Variant3, NSVariant3)])
def test_time_constant_velocity_reduces_to_stationary(V, NSV):
    prob = Problem((24, 20), (8, 8), Nt=4)
    I0, I1 = syn.blob_pair_2d(24, 2, 2.0)
    I0, I1 = I0[:, :20], I1[:, :20]
    v = _scaled(prob, 3, 0.8)
    vn = v.unsqueeze(0).repeat(prob.Nt + 1, 1, 1, 1)
    a, b = V(prob, I0, I1), NSV(prob, I0, I1)
    for m, vel in ((a, v), (b, vn)):
        m.setup(vel)
        m.state()
        m.adjoint()
    Ea, Eb = float(a.objective()[0]), float(b.objective()[0])
    assert abs(Ea - Eb) <= 1e-14 * abs(Ea)
    ga, gb = a.gradient(), b.gradient()
    w = torch.tensor(prob.trapezoid_weights(), dtype=torch.float64).reshape(-1, 1, 1, 1)
    assert float(((w * gb).sum(0) - ga).abs().max()) <= 1e-12 * float(ga.abs().max())
    dv = torch.tensor(syn.random_bl_coefficients(2, prob.K, 5))
    ha = a.hess_matvec(dv)
    hb = b.hess_matvec(dv.unsqueeze(0).repeat(prob.Nt + 1, 1, 1, 1))
    assert float(((w * hb).sum(0) - ha).abs().max()) <= 1e-12 * float(ha.abs().max())


def test_space_constant_time_varying_velocity():
    N, K, Nt = (16, 12), (8, 8), 4
    prob = Problem(N, K, Nt=Nt)
    c = [(0.02 + 0.01 * n, -0.015 * n) for n in range(Nt + 1)]
    v = torch.stack([torch.tensor(constant_velocity(K, cn)) for cn in c], 0)
    I0, I1 = syn.blob_pair_2d(16, 1, 1.0)
    I0, I1 = I0[:, :12], I1[:, :12]
    m = NSVariant3(prob, I0, I1)
    m.setup(v)
    m.state()
    u = np.zeros(2)
    for n in range(Nt):
        for j in range(2):
            expect = -0.5 * prob.dt * (c[n][j] + c[n + 1][j]) * N[j]
            assert float((m.Xb[n][j] - expect).abs().max()) < 1e-13
            assert float((m.Xf[n][j] + expect).abs().max()) < 1e-13
        u += 0.5 * prob.dt * (np.array(c[n]) + np.array(c[n + 1]))
        ref = torch.tensor(constant_velocity(K, tuple(u)))
        assert float((m.u[n + 1] - ref).abs().max()) < 1e-14


@pytest.mark.parametrize("NSV", [NSVariant1, NSVariant3])
def test_nonstationary_dto_gradient_matches_central_differences(NSV):
    prob = Problem((24, 24), (8, 8), Nt=3)
    I0, I1 = syn.blob_pair_2d(24, 0, 2.0)
    v = torch.stack([_scaled(prob, 10 + n, 0.6) for n in range(prob.Nt + 1)], 0)
    g = dto.gradient(NSV(prob, I0, I1), v)
    d = torch.stack([torch.tensor(syn.random_bl_coefficients(2, prob.K, 20 + n)) for n in range(prob.Nt + 1)], 0)
    d = d * (v.norm() / d.norm())
    eps = 1e-5
    fd = (float(dto.objective(NSV(prob, I0, I1), v + eps * d)) -
          float(dto.objective(NSV(prob, I0, I1), v - eps * d))) / (2 * eps)
    an = float((g * d).sum())
    assert abs(fd - an) <= 1e-6 * abs(an)


def _gaps(NSV, Nt, n=32, K=8):
    prob = Problem((n, n), (K, K), Nt=Nt)
    I0, I1 = syn.blob_pair_2d(n, 2, 2.0)
    va = torch.zeros((2, K, K), dtype=torch.float64)
    vb = torch.zeros((2, K, K), dtype=torch.float64)
    va[:, :8, :8] = torch.tensor(syn.random_bl_coefficients(2, (8, 8), 1))
    vb[:, :8, :8] = torch.tensor(syn.random_bl_coefficients(2, (8, 8), 2))
    s = 0.05 / float(sp.include(va, prob.N).abs().max())
    # a smooth time profile sampled at the nodes
    v = torch.stack([s * (va * math.cos(math.pi * t) + 0.5 * vb * math.sin(math.pi * t))
                     for t in np.linspace(0.0, 1.0, Nt + 1)], 0)
    m = NSV(prob, I0, I1)
    m.setup(v)
    m.state()
    m.adjoint()
    w = torch.tensor(prob.trapezoid_weights(), dtype=torch.float64).reshape(-1, 1, 1, 1)
    g = m.gradient()
    gd = dto.gradient(NSV(prob, I0, I1), v) / w
    x1 = torch.zeros((2, K, K), dtype=torch.float64)
    x1[:, :8, :8] = torch.tensor(syn.random_bl_coefficients(2, (8, 8), 3))
    x = torch.stack([x1] * (Nt + 1), 0)
    h = m.hess_matvec(x)
    # the exact Gauss-Newton Hessian of the discrete objective has the regulariser block w_n L~ per node;
    # dto.gn_hessian_matvec adds L~ x unweighted (the stationary regulariser), so it is exchanged here
    Lx = torch.stack([sp.apply_L(xn, 2, prob.alpha, prob.s) for xn in x], 0)
    hd = (dto.gn_hessian_matvec(NSV(prob, I0, I1), v, x) - Lx) / w + Lx
    return float((g - gd).norm() / gd.norm()), float((h - hd).norm() / hd.norm())


def test_nonstationary_otd_converges_to_dto():
    """Deformation state: refinement in dt; image transport: in the band as well (its gradient holds the
    projections pi(m), pi(lambda), as in the stationary case)."""
    g4, h4 = _gaps(NSVariant3, 4)
    g16, h16 = _gaps(NSVariant3, 16)
    assert g16 < 0.5 * g4 and h16 < 0.5 * h4
    g1, h1 = _gaps(NSVariant1, 8, 64, 16)
    g2, h2 = _gaps(NSVariant1, 16, 128, 32)
    print("gaps", g4, h4, g16, h16, g1, h1, g2, h2)
    assert g2 < 0.2 * g1 and h2 < 0.2 * h1


def test_nonstationary_gauss_newton_decreases_energy():
    prob = Problem((32, 32), (8, 8), Nt=4)
    I0, I1 = syn.blob_pair_2d(32, 0, 2.0)
    model = NSVariant3(prob, I0, I1)
    v, rep = gauss_newton(model, np.zeros((prob.Nt + 1, 2, 8, 8)), max_gn=4, max_pcg=3, fixed_iters=True)
    Es = [h["E"] for h in rep.history] + [rep.E]
    assert all(b <= a for a, b in zip(Es, Es[1:])) and rep.E < 0.5 * rep.E0
