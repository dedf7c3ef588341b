"""Pins of the oracle's state-equation variant (Section 2.3.2): the maps phi, psi, the Jacobian J and the
gradient and Gauss-Newton Hessian built on them.

* zero velocity: every map is the identity, J = 1, the adjoint is constant in time;
* constant velocities: u~, nu~ and U~ have closed forms, a one-voxel-per-step velocity moves the state and
  the adjoint by whole voxels (np.roll), a fractional shift multiplies a single Fourier mode by the
  closed-form gain of the cubic B-spline interpolant (SciPy's B-spline basis, independent of the oracle);
* the discretisation of the J equation (-D~_t U~ = -div~ v~ + U~ star div~ v~) equals, with J~ = 1 - U~,
  the band-limited adjoint sweep of the deformation-state variant started from the constant 1
  (-D~_t rho~ = rho~ star div~ v~), an algebraic identity of the two schemes;
* psi(0) inverts phi(1) up to a residual that falls with dt, and J(0) agrees with det(D psi(0));
* at v = 0 the gradient and the Gauss-Newton Hessian have closed forms without any sweep;
* the optimise-then-discretise gradient and Hessian approach the exact derivatives of the discrete
  objective (which is the deformation-state variant's objective) as the band and dt are refined.
"""
import numpy as np
import torch

from oracle import bspline, dto, spectral as sp
from oracle.gauss_newton import jacobian_det
from oracle.problem import Problem, velocity_grid_units
from oracle.variant2 import Variant2
from oracle.variant3 import Variant3
from paper_2006_06823_amd import synthetic as syn
from test_oracle_bspline import single_mode_gain
from test_oracle_transport import constant_velocity

torch.set_num_threads(min(8, torch.get_num_threads()))


def _solve(prob, I0, I1, v):
    m = Variant2(prob, I0, I1)
    m.setup(v)
    m.state()
    m.inverse_state()
    m.adjoint()
    return m


def test_v2_zero_velocity_identity():
    prob = Problem((16, 12), (8, 8), Nt=4)
    I0, I1 = syn.blob_pair_2d(16, 0, 1.0)
    I0, I1 = I0[:, :12], I1[:, :12]
    m = _solve(prob, I0, I1, np.zeros((2, 8, 8)))
    for mn in m.m:
        assert float((mn - torch.tensor(I0)).abs().max()) < 1e-13
    for a in m.u + m.nu + m.U:
        assert float(a.abs().max()) == 0.0
    for Jn in m.J:
        assert float((Jn - 1.0).abs().max()) == 0.0
    lam1 = -2.0 * (torch.tensor(I0) - torch.tensor(I1))
    for ln in m.lam:
        assert float((ln - lam1).abs().max()) < 1e-13


def test_v2_integer_shift_is_exact_roll():
    """One voxel per step along axis 0: m(t_n) = roll(I0, n), lambda(t_n) = roll(lambda(1), -(Nt - n))."""
    N, K, Nt = (16, 12), (8, 8), 4
    prob = Problem(N, K, Nt=Nt)
    I0, I1 = syn.blob_pair_2d(16, 1, 1.0)
    I0, I1 = I0[:, :12], I1[:, :12]
    c = Nt / N[0]
    m = _solve(prob, I0, I1, constant_velocity(K, (c, 0.0)))
    lam1 = -2.0 * (np.roll(I0, Nt, axis=0) - I1)
    for n in range(Nt + 1):
        assert np.abs(m.m[n].numpy() - np.roll(I0, n, axis=0)).max() < 1e-12
        assert np.abs(m.lam[n].numpy() - np.roll(lam1, -(Nt - n), axis=0)).max() < 1e-12
        # u~(t_n) = t_n c and nu~(t_n) = -(1 - t_n) c: only the constant slot is non-zero; U~ = 0
        t = n * prob.dt
        assert float((m.u[n] - torch.tensor(constant_velocity(K, (t * c, 0.0)))).abs().max()) < 1e-14
        assert float((m.nu[n] - torch.tensor(constant_velocity(K, (-(1 - t) * c, 0.0)))).abs().max()) < 1e-14
        assert float(m.U[n].abs().max()) < 1e-15


def test_v2_fractional_shift_single_mode():
    """A fractional constant shift s per step: m(t_n) = Re(G(n s) e^{i w x}) and, with I1 = 0,
    lambda(t_n) = -2 Re(G(Nt s) G(-(Nt - n) s) e^{i w x})."""
    n, Nt, k, s = 32, 5, 3, 0.37
    prob = Problem((n, 8), (8, 4), Nt=Nt)
    i = np.arange(n)
    om = 2 * np.pi * k / n
    I0 = np.repeat(np.cos(om * i)[:, None], 8, axis=1)
    m = _solve(prob, I0, np.zeros_like(I0), constant_velocity(prob.K, (s * Nt / n, 0.0)))
    e = np.exp(1j * om * i)
    for t in range(Nt + 1):
        expect_m = np.real(single_mode_gain(om, s * t) * e)
        assert np.abs(m.m[t][:, 0].numpy() - expect_m).max() < 1e-12
        expect_l = -2.0 * np.real(single_mode_gain(om, s * Nt) * single_mode_gain(om, -s * (Nt - t)) * e)
        assert np.abs(m.lam[t][:, 3].numpy() - expect_l).max() < 1e-12


def test_v2_jacobian_scheme_equals_adjoint_sweep_of_one():
    """J~ = 1 - U~ from the printed U~ equation equals the density-adjoint sweep started from 1."""
    prob = Problem((24, 20), (8, 8), Nt=5)
    I0, I1 = syn.blob_pair_2d(24, 2, 2.0)
    I0, I1 = I0[:, :20], I1[:, :20]
    v = torch.tensor(syn.random_bl_coefficients(2, prob.K, 5))
    v = v * (0.9 / (float(sp.include(v, prob.N).abs().max()) * prob.dt * 24))
    m = _solve(prob, I0, I1, v)
    m3 = Variant3(prob, I0, I1)
    m3.setup(v)
    one = torch.zeros(prob.K, dtype=torch.float64)
    one[0, 0] = 1.0
    assert float((sp.include(one, prob.N) - 1.0).abs().max()) < 1e-14
    ref = m3.bl_adjoint_sweep(one)
    scale = float(max(Un.abs().max() for Un in m.U))
    assert scale > 1e-3                      # a velocity with divergence: J departs from 1
    for Un, Jn in zip(m.U, ref):
        assert float(((one - Un) - Jn).abs().max()) < 1e-13


def _smooth_case(n, K, Nt, seed=4, cfl=0.8):
    prob = Problem((n, n), (K, K), Nt=Nt)
    v8 = syn.random_bl_coefficients(2, (8, 8), seed)
    v = np.zeros((2, K, K))
    v[:, :8, :8] = v8
    v = torch.tensor(v)
    v = v * (cfl * 8 / (float(sp.include(v, prob.N).abs().max()) * prob.dt * n * Nt))
    return prob, v


def test_v2_psi0_inverts_phi1_and_jacobian_matches():
    """phi(1)(psi(0)(x)) = x up to the SL-RK2 error: from Nt = 4 to Nt = 8 the residual falls >= 2.5x (its
    floor is the band truncation of u~, nu~) and |J(0) - det(D psi(0))|, det(D psi(0)) = det(I - D iota(nu~(0))),
    falls >= 3x (second order in dt); 1.6 voxels of displacement, J(0) in [0.66, 1.49]."""
    res, jac = [], []
    for Nt in (4, 8):
        prob, v = _smooth_case(64, 32, Nt, cfl=0.2)
        I0 = np.zeros((64, 64))
        m = _solve(prob, I0, I0, v)
        N = prob.N
        X = bspline.grid_index(N)
        nu0 = velocity_grid_units(sp.include(m.nu[0], N), N)
        u1 = velocity_grid_units(sp.include(m.u[-1], N), N)
        y = X - nu0                                          # psi(0)(x) in grid units
        u1_at_y = torch.stack([bspline.evaluate(bspline.prefilter(u1[j], 2), y) for j in range(2)], 0)
        res.append(float((y - u1_at_y - X).abs().max()))
        det = jacobian_det(prob, m.nu[0])                    # det(I - D iota(nu~(0)))
        jac.append(float((m.J[0] - det).abs().max()))
    assert res[0] < 1e-3 and jac[0] < 2e-3
    assert res[1] < res[0] / 2.5 and jac[1] < jac[0] / 3.0


def test_v2_zero_velocity_derivatives_closed_form():
    """At v = 0: gradient pi(iota(pi(lambda1)) G0), Hessian L~ dv + 2 pi(iota(pi(2 g . iota(dv))) G0)
    with G0 = iota(grad~ pi(I0)), g = nabla P(I0) at the nodes, lambda1 = -2 (I0 - I1)."""
    prob = Problem((24, 20), (8, 8), Nt=4)
    I0, I1 = syn.blob_pair_2d(24, 3, 2.0)
    I0, I1 = I0[:, :20], I1[:, :20]
    m = _solve(prob, I0, I1, np.zeros((2, 8, 8)))
    g = m.gradient()
    G0 = sp.include(sp.grad(sp.project(torch.tensor(I0), prob.K), 2), prob.N)
    lam1 = -2.0 * torch.tensor(I0 - I1)
    closed = sp.project(sp.include(sp.project(lam1, prob.K), prob.N).unsqueeze(0) * G0, prob.K)
    assert float((g - closed).abs().max()) <= 1e-12 * float(closed.abs().max())
    _, gi = bspline.evaluate(bspline.prefilter(torch.tensor(I0), 2), bspline.grid_index(prob.N), grad=True)
    gg = gi * torch.tensor([24.0, 20.0], dtype=torch.float64).reshape(2, 1, 1)
    dv = torch.tensor(syn.random_bl_coefficients(2, prob.K, 7))
    h = m.hess_matvec(dv)
    dl1 = 2.0 * (gg * sp.include(dv, prob.N)).sum(0)         # -(2/sigma^2) dm(1), dm(1) = -g . iota(dv)
    ref = sp.apply_L(dv, 2, prob.alpha, prob.s) + sp.project(
        sp.include(sp.project(dl1, prob.K), prob.N).unsqueeze(0) * G0, prob.K)
    assert float((h - ref).abs().max()) <= 1e-12 * float(ref.abs().max())


def test_v2_objective_is_deformation_state_objective():
    prob, v = _smooth_case(32, 8, 4)
    I0, I1 = syn.blob_pair_2d(32, 4, 2.0)
    m2 = Variant2(prob, I0, I1)
    m2.setup(v)
    m2.state()
    m3 = Variant3(prob, I0, I1)
    m3.setup(v)
    m3.state()
    assert abs(float(m2.objective()[0]) - float(m3.objective()[0])) < 1e-14 * float(m3.objective()[0])


def _otd_dto_gaps(n, K, Nt):
    prob, v = _smooth_case(n, K, Nt, seed=1, cfl=0.4)
    rng = np.random.default_rng(0)
    img = syn.BlobImage2D(rng)
    X = syn.grid_coords((n, n))
    img.norm = img.raw(X).max()
    disp = syn.smooth_displacement((n, n), 2.0 * n / 32, seed=7919)
    u = disp(X)
    I0 = img(X)
    I1 = img([np.mod(X[j] - u[j], 1.0) for j in range(2)])
    m = _solve(prob, I0, I1, v)
    g = m.gradient()
    gd = dto.gradient(Variant2(prob, I0, I1), v)
    x = torch.tensor(syn.random_bl_coefficients(2, (K, K), 3))
    h = m.hess_matvec(x)
    hd = dto.gn_hessian_matvec(Variant2(prob, I0, I1), v, x)
    return float((g - gd).norm() / gd.norm()), float((h - hd).norm() / hd.norm())


def test_v2_otd_converges_to_dto():
    g1, h1 = _otd_dto_gaps(64, 16, 4)
    g2, h2 = _otd_dto_gaps(128, 32, 8)
    assert g1 < 0.2 and h1 < 0.2
    assert g2 < 0.35 * g1 and h2 < 0.35 * h1
