"""GPU-vs-oracle parity of the state-equation variant (Section 2.3.2) through the C ABI: the maps
u~ (phi), nu~ (psi) and J~ = 1 - U~ at every node, the images m(t_n) = I0 o phi(t_n), the adjoints
lambda(t_n) = J(t_n) lambda(1) o psi(t_n), the gradient, the Gauss-Newton Hessian-vector product and its
incremental fields.  Tolerances as for the other variants: FP32 rel-L2 <= 1e-5 (element-wise <= 1e-4),
FP64 <= 1e-10."""
import numpy as np
import pytest
import torch

from gpu_common import close, images, oracle_model, velocity
from oracle import spectral as sp
from paper_2006_06823_amd import lddmm_bl as L
from paper_2006_06823_amd import synthetic as syn

pytestmark = pytest.mark.gpu

CASES = [
    # (dim, N, K, Nt, precision, cfl)
    (3, (40, 36, 44), (12, 10, 14), 4, L.FP32, 0.8),
    (2, (64, 64), (16, 16), 10, L.FP64, 0.8),
    (2, (48, 40), (14, 12), 5, L.FP32, 0.8),
    # departure points and whole-deformation displacements far outside any staged brick
    (3, (40, 36, 44), (12, 10, 14), 3, L.FP32, 2.5),
    # one time step; a band with a single real mode on one axis; odd sizes on every axis
    (3, (12, 10, 14), (4, 2, 4), 1, L.FP32, 0.8),
    (3, (17, 9, 33), (6, 4, 10), 2, L.FP32, 0.8),
]


def tol(precision):
    return 1e-10 if precision == L.FP64 else 1e-5


def dev(x, ctx):
    return torch.tensor(np.ascontiguousarray(x), dtype=ctx.dtype, device=ctx.device)


@pytest.mark.parametrize("dim,N,K,Nt,precision,cfl", CASES)
def test_state_equation_variant_parity(dim, N, K, Nt, precision, cfl):
    print(f"[case] dim {dim} N {N} K {K} Nt {Nt} precision {precision} cfl {cfl}", flush=True)
    I0, I1 = images(N, 3)
    ctx = L.Context(L.Problem(N, K, nt=Nt, variant=L.STATE_EQUATION, precision=precision))
    ctx.set_images(dev(I0, ctx), dev(I1, ctx))
    v = velocity(N, K, Nt, 4, cfl_vox=cfl)
    om = oracle_model(2, N, K, Nt, I0, I1)
    t = tol(precision)
    E, m1 = ctx.state_solve(dev(v, ctx), want_m1=True)
    om.setup(v)
    om.state()
    om.inverse_state()
    Eo = [float(x) for x in om.objective()]
    for a, b in zip(E, Eo):
        assert abs(a - b) <= 10 * t * abs(b)
    assert close(m1, om.m1, "m1") <= t
    one = torch.zeros(om.U[0].shape, dtype=torch.float64)
    one.view(-1)[0] = 1.0
    for n in range(Nt + 1):
        if n > 0:
            assert close(ctx.get_field(L.FIELD_STATE, n).reshape(om.u[n].shape), om.u[n], f"u~_{n}") <= t
        if n < Nt:
            assert close(ctx.get_field(L.FIELD_INVERSE_STATE, n).reshape(om.nu[n].shape), om.nu[n],
                         f"nu~_{n}") <= t
        assert close(ctx.get_field(L.FIELD_JACOBIAN_STATE, n).reshape(one.shape), one - om.U[n], f"J~_{n}") <= t
        assert close(ctx.get_field(L.FIELD_IMAGE, n).reshape(om.m[n].shape), om.m[n], f"m_{n}") <= t
    # adjoint at every node and the gradient
    g, ginf = ctx.adjoint_solve()
    om.adjoint()
    go = om.gradient()
    for n in (0, Nt // 2, Nt):
        assert close(ctx.get_field(L.FIELD_ADJOINT_GRID, n).reshape(om.lam[n].shape), om.lam[n],
                     f"lambda_{n}") <= t
    assert close(g, go, "gradient") <= t
    ginf_o = float(sp.include(go, N).abs().max())
    assert abs(ginf - ginf_o) <= 10 * t * ginf_o
    # Gauss-Newton Hessian-vector product and its incremental fields
    dv = syn.random_bl_coefficients(dim, K, 11)
    h = ctx.hess_matvec(dev(dv, ctx))
    ho = om.hess_matvec(dv)
    assert close(h, ho, "hessian") <= t
    du, dl = om.last_inc
    for n in (1, Nt):
        assert close(ctx.get_field(L.FIELD_INC_STATE, n).reshape(du[n].shape), du[n], f"du~_{n}") <= t
    for n in (0, Nt):
        dlt = sp.project(dl[n], tuple(K))
        assert close(ctx.get_field(L.FIELD_INC_ADJOINT, n).reshape(dlt.shape), dlt, f"dlambda~_{n}") <= t


def test_state_equation_graph_replay_equals_eager(monkeypatch):
    """The captured matvec of the state-equation variant equals its eager launch sequence bitwise."""
    N, K, Nt = (40, 36, 44), (12, 10, 14), 4
    I0, I1 = images(N, 5)
    v = velocity(N, K, Nt, 6)
    dv = syn.random_bl_coefficients(3, K, 7)
    out = []
    for eager in (False, True):
        if eager:
            monkeypatch.setenv("LDDMM_BL_NO_GRAPH", "1")
        ctx = L.Context(L.Problem(N, K, nt=Nt, variant=L.STATE_EQUATION, precision=L.FP32))
        ctx.set_images(dev(I0, ctx), dev(I1, ctx))
        ctx.state_solve(dev(v, ctx))
        h1 = ctx.hess_matvec(dev(dv, ctx))
        h2 = ctx.hess_matvec(dev(dv, ctx))
        out.append((h1.clone(), h2.clone()))
    assert torch.equal(out[0][0], out[0][1])
    assert torch.equal(out[0][0], out[1][0])
