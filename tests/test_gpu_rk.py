"""GPU-vs-oracle parity of the explicit RK4 comparator (the deformation-state equations of Section 2.3.3
in Eulerian form, classical four-stage Runge-Kutta, exact truncated products) through the C ABI: state
u~_n, m(1), adjoint rho~(0), gradient, Gauss-Newton Hessian-vector product and its incremental fields,
and a 2D FP64 Gauss-Newton run with identical decisions.  Tolerances: FP32 rel-L2 <= 1e-5 (element-wise
<= 1e-4), FP64 <= 1e-10."""
import numpy as np
import pytest
import torch

from gpu_common import close, images, velocity
from oracle.eulerian_rk import Variant3RK
from oracle.gauss_newton import gauss_newton
from oracle.problem import Problem as OProblem
from paper_2006_06823_amd import lddmm_bl as L
from paper_2006_06823_amd import synthetic as syn

pytestmark = pytest.mark.gpu

CASES = [
    # (dim, N, K, Nt, precision)
    (3, (40, 36, 44), (12, 10, 14), 8, L.FP32),
    (2, (64, 64), (16, 16), 25, L.FP64),
    (2, (48, 40), (14, 12), 10, L.FP32),
    (3, (17, 9, 33), (6, 4, 10), 4, L.FP32),
]


def tol(precision):
    return 1e-10 if precision == L.FP64 else 1e-5


def dev(x, ctx):
    return torch.tensor(np.ascontiguousarray(x), dtype=ctx.dtype, device=ctx.device)


def rk_context(N, K, Nt, precision):
    return L.Context(L.Problem(N, K, nt=Nt, variant=L.DEFORMATION_STATE, precision=precision,
                               integrator=L.EULER_RK4))


@pytest.mark.parametrize("dim,N,K,Nt,precision", CASES)
def test_rk4_comparator_parity(dim, N, K, Nt, precision):
    print(f"[case] dim {dim} N {N} K {K} Nt {Nt} precision {precision}", flush=True)
    I0, I1 = images(N, 2)
    ctx = rk_context(N, K, Nt, precision)
    ctx.set_images(dev(I0, ctx), dev(I1, ctx))
    # 0.8 voxel of displacement per SL step of Nt = 10, whatever Nt the RK scheme takes
    v = velocity(N, K, 10, 3, cfl_vox=0.8)
    om = Variant3RK(OProblem(tuple(N), tuple(K), Nt=Nt), I0, I1)
    t = tol(precision)
    E, m1 = ctx.state_solve(dev(v, ctx), want_m1=True)
    om.setup(v)
    om.state()
    for a, b in zip(E, [float(x) for x in om.objective()]):
        assert abs(a - b) <= 10 * t * abs(b)
    for n in (1, Nt // 2, Nt):
        assert close(ctx.get_field(L.FIELD_STATE, n).reshape(om.u[n].shape), om.u[n], f"u~_{n}") <= t
    assert close(m1, om.m1, "m1") <= t
    g, _ = ctx.adjoint_solve()
    om.adjoint()
    assert close(ctx.get_field(L.FIELD_ADJOINT0).reshape(om.rho[0].shape), om.rho[0], "rho~_0") <= t
    assert close(g, om.gradient(), "gradient") <= t
    dv = syn.random_bl_coefficients(dim, K, 11)
    h = ctx.hess_matvec(dev(dv, ctx))
    assert close(h, om.hess_matvec(dv), "hessian") <= t
    du, dr = om.last_inc
    for n in (1, Nt):
        assert close(ctx.get_field(L.FIELD_INC_STATE, n).reshape(du[n].shape), du[n], f"du~_{n}") <= t
    for n in (0, Nt // 2):
        assert close(ctx.get_field(L.FIELD_INC_ADJOINT, n).reshape(dr[n].shape), dr[n], f"drho~_{n}") <= t


def test_rk4_comparator_gn_2d_fp64_matches_oracle():
    N, K, Nt = (64, 64), (16, 16), 25
    I0, I1 = syn.blob_pair_2d(64, 0, 4.0)
    ctx = rk_context(N, K, Nt, L.FP64)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    ctx.set_images(t(I0), t(I1))
    v = torch.zeros((2,) + K, dtype=torch.float64, device="cuda")
    st, rep = ctx.gn_solve(v, max_gn=4, max_pcg=5, fixed_iters=True)
    om = Variant3RK(OProblem(N, K, Nt=Nt), I0, I1)
    vo, ro = gauss_newton(om, np.zeros((2,) + K), max_gn=4, max_pcg=5, fixed_iters=True)
    print(f"[gn] rk4 gpu {rep['decisions']} oracle {ro.decisions}", flush=True)
    assert rep["decisions"] == ro.decisions
    assert close(v, vo, "velocity after 4 GN iterations") <= 1e-8
    assert rep["E"] < rep["E0"]


def test_rk4_comparator_rejects_other_variants():
    for variant in (L.IMAGE_TRANSPORT, L.STATE_EQUATION):
        with pytest.raises(L.LddmmError):
            L.Context(L.Problem((16, 16, 16), (8, 8, 8), nt=4, variant=variant, integrator=L.EULER_RK4))
