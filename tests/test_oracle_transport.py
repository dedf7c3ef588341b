"""Pins of the oracle's characteristics and SL-RK2 solves (Section 3, Table 1) against closed forms."""
import math

import numpy as np
import pytest
import torch

from oracle import semilag, spectral as sp, bspline
from oracle.gauss_newton import displacement_state, jacobian_det
from oracle.problem import Problem
from oracle.variant1 import Variant1
from oracle.variant3 import Variant3
from paper_2006_06823_amd import synthetic as syn


def constant_velocity(K, c):
    """BL velocity whose only non-zero slots are the constants (a spatially constant field)."""
    v = np.zeros((len(K),) + tuple(K))
    for j, cj in enumerate(c):
        v[(j,) + (0,) * len(K)] = cj
    return v


def test_characteristics_constant_and_zero_velocity():
    """P7: v = const gives X = x -/+ dt c exactly; v = 0 gives X = x."""
    N = (16, 12, 10)
    vg = torch.zeros((3,) + N, dtype=torch.float64)
    assert float(semilag.characteristics(vg, 0.1, -1).abs().max()) == 0.0
    c = (0.013, -0.021, 0.007)
    for j in range(3):
        vg[j] = c[j]
    dt = 0.1
    for direction in (-1, 1):
        X = semilag.characteristics(vg, dt, direction)
        for j in range(3):
            assert float((X[j] - direction * dt * c[j] * N[j]).abs().max()) < 1e-13


def test_characteristics_third_order_local_error():
    """P10: for v = a sin(2 pi x) the departure point has the closed form
    tan(pi X) = tan(pi x) exp(-2 pi a dt); the local error of the RK2 scheme falls ~8x per halving of dt."""
    n = 256
    a = 0.3
    x = np.arange(n) / n
    vg = torch.zeros(2, n, 4, dtype=torch.float64)
    vg[0] = torch.tensor(a * np.sin(2 * np.pi * x))[:, None]
    errs = []
    for dt in (0.1, 0.05, 0.025):
        X = semilag.characteristics(vg, dt, -1)[0, :, 0].numpy() / n + x
        # exact backward flow for dt (branch-safe form of the closed form)
        exact = np.arctan2(np.sin(np.pi * x) * np.exp(-2 * np.pi * a * dt), np.cos(np.pi * x)) / np.pi
        exact = np.where(exact < 0, exact + 1, exact)
        diff = (X - exact + 0.5) % 1.0 - 0.5
        errs.append(np.abs(diff).max())
    assert errs[0] / errs[1] > 6.0 and errs[1] / errs[2] > 6.0


def _pair2d(n=16, seed=0):
    return syn.blob_pair_2d(n, seed, 1.0)


def test_zero_velocity_identity():
    """P8: with v = 0 every solve is the identity in time: m(1) = I0, u~ = 0, adjoints constant, det = 1."""
    prob = Problem((16, 16), (8, 8), Nt=4)
    I0, I1 = _pair2d()
    v = np.zeros((2, 8, 8))
    m = Variant1(prob, I0, I1)
    m.setup(v)
    m1 = m.state()
    assert float((m1 - torch.tensor(I0)).abs().max()) < 1e-13
    lam = m.adjoint()
    for ln in lam:
        assert float((ln - lam[-1]).abs().max()) < 1e-13
    m3 = Variant3(prob, I0, I1)
    m3.setup(v)
    m1 = m3.state()
    assert float((m1 - torch.tensor(I0)).abs().max()) < 1e-13
    assert all(float(u.abs().max()) == 0.0 for u in m3.u)
    rho = m3.adjoint()
    for r in rho:
        assert float((r - rho[-1]).abs().max()) < 1e-13
    det = jacobian_det(prob, displacement_state(prob, v))
    assert float((det - 1).abs().max()) < 1e-14


@pytest.mark.parametrize("Nt", [4, 5])
def test_integer_shift_is_exact_roll(Nt):
    """P9: a constant velocity moving exactly one voxel per step transports I0 by np.roll (both variants)."""
    N = (16, 12)
    K = (8, 8)
    prob = Problem(N, K, Nt=Nt)
    I0, I1 = syn.blob_pair_2d(16, 1, 1.0)
    I0 = I0[:, :12]
    I1 = I1[:, :12]
    # one voxel per step along axis 0: dt * c * N0 = 1 -> c = Nt / N0; constant slot holds the mean
    v = constant_velocity(K, (Nt / N[0], 0.0))
    m = Variant1(prob, I0, I1)
    m.setup(v)
    m1 = m.state().numpy()
    assert np.abs(m1 - np.roll(I0, Nt, axis=0)).max() < 1e-12
    m3 = Variant3(prob, I0, I1)
    m3.setup(v)
    m1 = m3.state().numpy()
    assert np.abs(m1 - np.roll(I0, Nt, axis=0)).max() < 1e-12
    # u~(t_n) = t_n c exactly (only the constant slot is non-zero)
    for n, u in enumerate(m3.u):
        ref = torch.tensor(constant_velocity(K, (n * prob.dt * Nt / N[0], 0.0)))
        assert float((u - ref).abs().max()) < 1e-14


def test_fractional_constant_shift_closed_form():
    """P9: a single Fourier mode under a fractional constant shift is multiplied by G(omega, s)^Nt."""
    from test_oracle_bspline import single_mode_gain

    n, Nt = 32, 5
    prob = Problem((n, 8), (8, 4), Nt=Nt)
    k = 3
    i = np.arange(n)
    om = 2 * np.pi * k / n
    I0 = np.repeat(np.cos(om * i)[:, None], 8, axis=1)
    shift = 0.37                                 # voxels per step
    v = constant_velocity(prob.K, (shift * Nt / n, 0.0))
    m = Variant1(prob, I0, I0)
    m.setup(v)
    m1 = m.state().numpy()
    G = single_mode_gain(om, shift)
    expect = np.real(G ** Nt * np.exp(1j * om * i))
    assert np.abs(m1[:, 0] - expect).max() < 1e-12
    # deformation-state variant: one interpolation of the accumulated shift
    m3 = Variant3(prob, I0, I0)
    m3.setup(v)
    m1 = m3.state().numpy()
    expect3 = np.real(single_mode_gain(om, shift * Nt) * np.exp(1j * om * i))
    assert np.abs(m1[:, 0] - expect3).max() < 1e-12


def test_jacobian_single_mode_closed_form():
    """P17: det(I - D iota(u~)) for a single sine mode in u_0 is 1 - a sqrt(2) 2 pi k cos(2 pi k x0)."""
    N, K = (16, 12), (8, 8)
    prob = Problem(N, K)
    u = np.zeros((2,) + K)
    a, k = 0.02, 2
    u[0, 2 * k, 0] = a                            # sqrt(2) sin(2 pi k x0)
    det = jacobian_det(prob, u).numpy()
    X = syn.grid_coords(N)
    expect = 1 - a * math.sqrt(2) * 2 * math.pi * k * np.cos(2 * math.pi * k * X[0])
    assert np.abs(det - expect).max() < 1e-13
