"""GPU-vs-oracle parity of the two-level spectral preconditioner (coarse level N/2, band 2 floor(K/4);
L~^-1 above the coarse band, inner PCG on the coarse Gauss-Newton Hessian inside it, flexible outer CG):
Gauss-Newton runs with identical decisions and velocities against the oracle's driver with the same
preconditioner (2D FP64: velocity <= 1e-8; 3D FP32: <= 1e-4), and the argument checks."""
import numpy as np
import pytest
import torch

from gpu_common import close, images, oracle_model
from oracle.gauss_newton import gauss_newton
from oracle.multilevel import TwoLevel
from oracle.problem import Problem as OProblem
from oracle.variant1 import Variant1
from oracle.variant3 import Variant3
from paper_2006_06823_amd import lddmm_bl as L
from paper_2006_06823_amd import synthetic as syn

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("variant", [1, 3])
def test_two_level_gn_2d_fp64_matches_oracle(variant):
    N, K, Nt = (64, 64), (16, 16), 5
    I0, I1 = syn.blob_pair_2d(64, 0, 4.0)
    ctx = L.Context(L.Problem(N, K, nt=Nt, variant=variant, precision=L.FP64))
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    ctx.set_images(t(I0), t(I1))
    v = torch.zeros((2,) + K, dtype=torch.float64, device="cuda")
    st, rep = ctx.gn_solve(v, max_gn=4, max_pcg=3, fixed_iters=True, ml_inner=5)
    V = Variant1 if variant == 1 else Variant3
    prob = OProblem(N, K, Nt=Nt)
    vo, ro = gauss_newton(V(prob, I0, I1), np.zeros((2,) + K), max_gn=4, max_pcg=3, fixed_iters=True,
                          precond=TwoLevel(V, prob, I0, I1, inner=5))
    print(f"[two-level] variant {variant} gpu {rep['decisions']} oracle {ro.decisions}", flush=True)
    assert rep["decisions"] == ro.decisions
    assert close(v, vo, "velocity after 4 GN iterations") <= 1e-8
    assert abs(rep["E"] - ro.E) <= 1e-10 * abs(ro.E)


def test_two_level_gn_3d_fp32_matches_oracle():
    N, K, Nt = (40, 36, 44), (12, 10, 14), 4
    I0, I1 = images(N, 1)
    ctx = L.Context(L.Problem(N, K, nt=Nt, variant=L.DEFORMATION_STATE, precision=L.FP32))
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    ctx.set_images(t(I0), t(I1))
    v = torch.zeros((3,) + K, dtype=torch.float32, device="cuda")
    st, rep = ctx.gn_solve(v, max_gn=2, max_pcg=3, fixed_iters=True, ml_inner=4)
    prob = OProblem(N, K, Nt=Nt)
    vo, ro = gauss_newton(Variant3(prob, I0, I1), np.zeros((3,) + K), max_gn=2, max_pcg=3, fixed_iters=True,
                          precond=TwoLevel(Variant3, prob, I0, I1, inner=4))
    assert rep["decisions"] == ro.decisions
    assert close(v, vo, "velocity after 2 GN iterations") <= 1e-4


def test_two_level_argument_checks():
    ctx = L.Context(L.Problem((17, 16, 16), (8, 8, 8), nt=2, variant=L.DEFORMATION_STATE))
    I = torch.zeros((17, 16, 16), dtype=torch.float32, device="cuda")
    ctx.set_images(I, I)
    v = torch.zeros((3, 8, 8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(L.LddmmError):          # odd grid size
        ctx.gn_solve(v, max_gn=1, max_pcg=1, ml_inner=2)
    ctx2 = L.Context(L.Problem((16, 16, 16), (8, 8, 8), nt=2, variant=L.DEFORMATION_STATE))
    ctx2.set_images(I[:16], I[:16])
    Z = torch.zeros((1, 3, 8, 8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(L.LddmmError):          # excludes the low-rank preconditioner
        ctx2.gn_solve(v, max_gn=1, max_pcg=1, ml_inner=2, Z=Z)
