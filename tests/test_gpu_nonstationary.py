"""GPU-vs-oracle parity of non-stationary velocities (a velocity per time node; Section 1.3, NSt rows of
Tables 3-4) for the image-transport and deformation-state variants, through the C ABI: per-step departure
points, state, adjoint, node-field gradient and Gauss-Newton Hessian-vector product and incremental fields,
and a 2D FP64 Gauss-Newton run with identical decisions.  Tolerances: FP32 rel-L2 <= 1e-5 (element-wise
<= 1e-4), FP64 <= 1e-10."""
import numpy as np
import pytest
import torch

from gpu_common import close, images, velocity
from oracle.gauss_newton import gauss_newton
from oracle.nonstationary import NSVariant1, NSVariant3
from oracle.problem import Problem as OProblem
from paper_2006_06823_amd import lddmm_bl as L
from paper_2006_06823_amd import synthetic as syn

pytestmark = pytest.mark.gpu

CASES = [
    # (dim, N, K, Nt, precision)
    (3, (40, 36, 44), (12, 10, 14), 4, L.FP32),
    (2, (64, 64), (16, 16), 5, L.FP64),
    (3, (17, 9, 33), (6, 4, 10), 2, L.FP32),
]


def tol(precision):
    return 1e-10 if precision == L.FP64 else 1e-5


def dev(x, ctx):
    return torch.tensor(np.ascontiguousarray(x), dtype=ctx.dtype, device=ctx.device)


def node_velocity(N, K, Nt, seed):
    """A different random band-limited field at every node, each at 0.8 voxel per step."""
    return np.stack([velocity(N, K, Nt, seed + n, cfl_vox=0.8) for n in range(Nt + 1)], 0)


@pytest.mark.parametrize("variant", [1, 3])
@pytest.mark.parametrize("dim,N,K,Nt,precision", CASES)
def test_nonstationary_parity(variant, dim, N, K, Nt, precision):
    print(f"[case] variant {variant} dim {dim} N {N} K {K} Nt {Nt} precision {precision}", flush=True)
    I0, I1 = images(N, 4)
    ctx = L.Context(L.Problem(N, K, nt=Nt, variant=variant, precision=precision, nonstationary=True))
    ctx.set_images(dev(I0, ctx), dev(I1, ctx))
    v = node_velocity(N, K, Nt, 30)
    om = (NSVariant1 if variant == 1 else NSVariant3)(OProblem(tuple(N), tuple(K), Nt=Nt), I0, I1)
    t = tol(precision)
    E, m1 = ctx.state_solve(dev(v, ctx), want_m1=True)
    om.setup(v)
    m1o = om.state()
    for a, b in zip(E, [float(x) for x in om.objective()]):
        assert abs(a - b) <= 10 * t * abs(b)
    for n in (0, Nt - 1):
        assert close(ctx.get_field(L.FIELD_DEP_BACKWARD, n).reshape(om.Xb[n].shape), om.Xb[n], f"Xb_{n}") <= t
        assert close(ctx.get_field(L.FIELD_DEP_FORWARD, n).reshape(om.Xf[n].shape), om.Xf[n], f"Xf_{n}") <= t
    assert close(m1, m1o, "m1") <= t
    if variant == 3:
        for n in (1, Nt):
            assert close(ctx.get_field(L.FIELD_STATE, n).reshape(om.u[n].shape), om.u[n], f"u~_{n}") <= t
    g, ginf = ctx.adjoint_solve()
    om.adjoint()
    go = om.gradient()
    assert close(g, go, "node gradient") <= t
    dv = np.stack([syn.random_bl_coefficients(dim, K, 40 + n) for n in range(Nt + 1)], 0)
    h = ctx.hess_matvec(dev(dv, ctx))
    ho = om.hess_matvec(dv)
    assert close(h, ho, "node Hessian") <= t
    di, da = om.last_inc
    got = ctx.get_field(L.FIELD_INC_STATE, Nt).reshape(di[Nt].shape)
    assert close(got, di[Nt], "inc state at 1") <= t
    got = ctx.get_field(L.FIELD_INC_ADJOINT, 0).reshape(da[0].shape)
    assert close(got, da[0], "inc adjoint at 0") <= t


@pytest.mark.parametrize("variant", [1, 3])
def test_nonstationary_gn_2d_fp64_matches_oracle(variant):
    N, K, Nt = (64, 64), (16, 16), 5
    I0, I1 = syn.blob_pair_2d(64, 0, 4.0)
    ctx = L.Context(L.Problem(N, K, nt=Nt, variant=variant, precision=L.FP64, nonstationary=True))
    tt = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    ctx.set_images(tt(I0), tt(I1))
    v = torch.zeros((Nt + 1, 2) + K, dtype=torch.float64, device="cuda")
    st, rep = ctx.gn_solve(v, max_gn=4, max_pcg=4, fixed_iters=True)
    om = (NSVariant1 if variant == 1 else NSVariant3)(OProblem(N, K, Nt=Nt), I0, I1)
    vo, ro = gauss_newton(om, np.zeros((Nt + 1, 2) + K), max_gn=4, max_pcg=4, fixed_iters=True)
    print(f"[gn] nonstationary variant {variant} gpu {rep['decisions']} oracle {ro.decisions}", flush=True)
    assert rep["decisions"] == ro.decisions
    assert close(v, vo, "velocity after 4 GN iterations") <= 1e-8
    assert abs(rep["E"] - ro.E) <= 1e-10 * abs(ro.E) and rep["E"] < rep["E0"]


def test_nonstationary_argument_checks():
    with pytest.raises(L.LddmmError):
        L.Context(L.Problem((16, 16, 16), (8, 8, 8), nt=3, variant=L.STATE_EQUATION, nonstationary=True))
    with pytest.raises(L.LddmmError):
        L.Context(L.Problem((16, 16, 16), (8, 8, 8), nt=3, variant=L.DEFORMATION_STATE, nonstationary=True,
                            integrator=L.EULER_RK4))
    ctx = L.Context(L.Problem((16, 16, 16), (8, 8, 8), nt=3, variant=L.DEFORMATION_STATE, nonstationary=True))
    with pytest.raises(ValueError):          # a stationary-shaped velocity
        ctx.state_solve(torch.zeros((3, 8, 8, 8), dtype=torch.float32, device="cuda"))
