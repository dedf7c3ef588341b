"""Pins of the oracle's PCG and Gauss-Newton driver (Section 2.2, eqs. BLNewton / BLKKT; Section 4.3)."""
import numpy as np
import pytest
import torch

from oracle import spectral as sp
from oracle.gauss_newton import pcg, gauss_newton, displacement_state, jacobian_det
from oracle.problem import Problem
from oracle.variant1 import Variant1
from oracle.variant3 import Variant3
from paper_2006_06823_amd import synthetic as syn


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, 50.0, n)
    return torch.tensor(Q @ np.diag(lam) @ Q.T)


def test_pcg_converges_to_direct_solve():
    """P16: PCG run to convergence equals numpy's dense solve."""
    A = _spd(30, 0)
    b = torch.tensor(np.random.default_rng(1).standard_normal(30))
    Minv = torch.diag(1.0 / torch.diag(A))
    x, it, flag, rn = pcg(lambda p: A @ p, b, lambda r: Minv @ r, 1e-13, 200)
    ref = np.linalg.solve(A.numpy(), b.numpy())
    assert flag == 0
    assert np.abs(x.numpy() - ref).max() < 1e-10 * np.abs(ref).max()


def test_pcg_iterate_is_krylov_minimiser():
    """P16: after k iterations PCG minimises the A-norm error over the preconditioned Krylov space."""
    n, k = 25, 4
    A = _spd(n, 2).numpy()
    b = np.random.default_rng(3).standard_normal(n)
    Minv = np.diag(1.0 / np.diag(A))
    x, it, flag, _ = pcg(lambda p: torch.tensor(A) @ p, torch.tensor(b), lambda r: torch.tensor(Minv) @ r,
                         0.0, k, fixed=True)
    # basis of span{M^-1 b, (M^-1 A) M^-1 b, ...}
    basis = [Minv @ b]
    for _ in range(k - 1):
        basis.append(Minv @ (A @ basis[-1]))
    Vb, _ = np.linalg.qr(np.stack(basis, 1))
    y = np.linalg.solve(Vb.T @ A @ Vb, Vb.T @ b)
    ref = Vb @ y
    assert np.abs(x.numpy() - ref).max() < 1e-9 * np.abs(ref).max()


def test_pcg_negative_curvature_stops():
    """Truncated CG: an indefinite operator stops at the first non-positive curvature."""
    A = torch.diag(torch.tensor([-1.0, 2.0, 3.0], dtype=torch.float64))
    b = torch.tensor([1.0, 0.0, 0.0], dtype=torch.float64)
    x, it, flag, _ = pcg(lambda p: A @ p, b, lambda r: r, 1e-12, 5)
    assert flag == 3 and it == 0
    assert torch.allclose(x, b)


@pytest.mark.parametrize("V", [Variant1, Variant3])
def test_gauss_newton_decreases_energy_and_registers(V):
    """P17: Armijo keeps E monotone; the synthetic pair is registered (MSE_rel well below 1)."""
    prob = Problem((32, 32), (8, 8), Nt=5)
    I0, I1 = syn.blob_pair_2d(32, 0, 2.0)
    model = V(prob, I0, I1)
    v, rep = gauss_newton(model, np.zeros((2, 8, 8)), max_gn=4, max_pcg=3, fixed_iters=True)
    Es = [h["E"] for h in rep.history] + [rep.E]
    assert all(b <= a + 1e-15 for a, b in zip(Es, Es[1:]))
    assert rep.mse_rel < 0.6
    det = jacobian_det(prob, displacement_state(prob, v))
    assert float(det.min()) > 0.0
