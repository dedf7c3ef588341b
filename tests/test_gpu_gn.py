"""Gauss-Newton-Krylov on the GPU against the oracle's driver: the 2D configuration (64^2, band 16^2,
Nt = 10, FP64, 10 GN x 5 PCG with fixed iteration counts), all three variants.

Both drivers log their discrete decisions per GN iteration (PCG iterations, truncation on non-positive
curvature, Armijo backtracks; Section 2.2 eqs. BLNewton / BLKKT with the Armijo reading).  Near
convergence an Armijo test compares energy differences at the rounding level, where the FFT-based
oracle and the contraction-based GPU path may take different accept/reject decisions (both correct).
The test therefore compares the decision sequences of the full run and reports the first iteration where
they differ; up to that iteration both drivers are re-run and must agree strictly (identical decisions,
velocity within 1e-8); the full run's final velocity is held to the 1e-3 target.
"""
import numpy as np
import pytest
import torch

from gpu_common import close, oracle_model, rel_l2
from oracle.gauss_newton import gauss_newton
from paper_2006_06823_amd import lddmm_bl as L
from paper_2006_06823_amd import synthetic as syn

pytestmark = pytest.mark.gpu


def _run_2d(variant, max_gn):
    N, K, Nt = (64, 64), (16, 16), 10
    I0, I1 = syn.blob_pair_2d(64, 0, 4.0)
    ctx = L.Context(L.Problem(N, K, nt=Nt, variant=variant, precision=L.FP64))
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    ctx.set_images(t(I0), t(I1))
    v = torch.zeros((2,) + K, dtype=torch.float64, device="cuda")
    st, rep = ctx.gn_solve(v, max_gn=max_gn, max_pcg=5, fixed_iters=True)
    om = oracle_model(variant, N, K, Nt, I0, I1)
    vo, ro = gauss_newton(om, np.zeros((2,) + K), max_gn=max_gn, max_pcg=5, fixed_iters=True)
    return ctx, v, rep, vo, ro


def _first_difference(a, b):
    for i, (x, y) in enumerate(zip(a, b)):
        if tuple(x) != tuple(y):
            return i
    return None if len(a) == len(b) else min(len(a), len(b))


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_gn_2d_fp64_decision_sequences(variant):
    ctx, v, rep, vo, ro = _run_2d(variant, 10)
    gpu, ora = rep["decisions"], ro.decisions
    j = _first_difference(gpu, ora)
    print(f"[gn] variant {variant} gpu decisions {gpu}", flush=True)
    print(f"[gn] variant {variant} oracle decisions {ora}", flush=True)
    print(f"[gn] variant {variant} first differing GN iteration: {j}", flush=True)
    assert close(v, vo, "final velocity") <= 1e-3
    assert abs(rep["E"] - ro.E) <= 1e-6 * abs(ro.E)
    assert rep["E"] < rep["E0"] and rep["mse_rel"] < 0.5
    assert 0.0 < rep["det_min"] <= 1.0 <= rep["det_max"]
    if j is None:
        assert close(v, vo, "velocity, identical decisions") <= 1e-8
        return
    # the drivers may part only where Armijo compares energies at the rounding level, after the early
    # iterations whose decrease is far above it
    assert j >= 4, f"decision sequences differ already at GN iteration {j}"
    ctx2, v2, rep2, vo2, ro2 = _run_2d(variant, j)
    assert rep2["decisions"] == ro2.decisions == ora[:j]
    assert close(v2, vo2, f"velocity after {j} GN iterations") <= 1e-8
    assert abs(rep2["E"] - ro2.E) <= 1e-8 * abs(ro2.E)


@pytest.mark.parametrize("variant", [1, 3])
def test_gn_2d_fp64_report_extrema_match_the_jacobian_call(variant):
    ctx, v, rep, vo, ro = _run_2d(variant, 3)
    (dmin, dmax), _ = ctx.jacobian()
    assert rep["det_min"] == dmin and rep["det_max"] == dmax
    assert rep["decisions"] == ro.decisions


def test_gn_3d_fp32_small_matches_oracle():
    """FP32 3D GN (fixed 3 GN x 3 PCG) ends within rel-L2 1e-3 of the FP64 oracle's velocity."""
    N, K, Nt = (32, 32, 32), (8, 8, 8), 5
    I0, I1 = syn.phantom_pair_3d(N, 5, max_disp_vox=2.0)
    ctx = L.Context(L.Problem(N, K, nt=Nt, variant=L.DEFORMATION_STATE, precision=L.FP32))
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    ctx.set_images(t(I0), t(I1))
    v = torch.zeros((3,) + K, dtype=torch.float32, device="cuda")
    st, rep = ctx.gn_solve(v, max_gn=3, max_pcg=3, fixed_iters=True)
    om = oracle_model(3, N, K, Nt, I0.astype(np.float64), I1.astype(np.float64))
    vo, ro = gauss_newton(om, np.zeros((3,) + K), max_gn=3, max_pcg=3, fixed_iters=True)
    assert rep["backtracks"] == ro.backtracks
    assert close(v, vo) <= 1e-3


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_gn_reuses_a_held_state_at_the_same_velocity(variant):
    """A state solve at the starting velocity just before gn_solve is reused by it (the solve skips its
    own first state solve); the result is bitwise the one of a fresh context.  A state held at another
    velocity, or invalidated by new images, is not reused."""
    N, K, Nt = (24, 20, 28), (8, 6, 10), 3
    I0, I1 = syn.phantom_pair_3d(N, 3, max_disp_vox=1.5)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    v0 = t(0.02 * syn.random_bl_coefficients(3, K, 4))

    def solve(prep):
        ctx = L.Context(L.Problem(N, K, nt=Nt, variant=variant, precision=L.FP32))
        ctx.set_images(t(I0), t(I1))
        prep(ctx)
        v = v0.clone()
        st, rep = ctx.gn_solve(v, max_gn=3, max_pcg=3, fixed_iters=True)
        return v, rep

    ref_v, ref = solve(lambda ctx: None)
    held_v, held = solve(lambda ctx: ctx.state_solve(v0.clone()))
    other_v, other = solve(lambda ctx: ctx.state_solve(torch.zeros_like(v0)))
    renewed_v, renewed = solve(lambda ctx: (ctx.state_solve(v0.clone()), ctx.set_images(t(I1), t(I0)),
                                            ctx.set_images(t(I0), t(I1))))
    for v, rep in ((held_v, held), (other_v, other), (renewed_v, renewed)):
        assert torch.equal(v, ref_v)
        assert rep["E0"] == ref["E0"] and rep["E"] == ref["E"] and rep["gn_iters"] == ref["gn_iters"]


@pytest.mark.parametrize("variant,twolevel", [(1, False), (2, False), (3, False), (3, True)])
def test_gn_graph_replay_equals_eager_launches(variant, twolevel, monkeypatch):
    """gn_solve runs its Hessian matvecs as replays of one captured HIP graph and keeps the PCG step
    lengths on the device (one host round trip per PCG iteration); with LDDMM_BL_NO_GRAPH set the same
    kernels are launched one by one.  Both give bitwise the same velocity, report and decisions, with the
    plain and with the two-level preconditioner (random directions Z, r = 2)."""
    N, K, Nt = (32, 28, 24), (8, 8, 6), 4
    I0, I1 = syn.phantom_pair_3d(N, 6, max_disp_vox=2.0)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    Z = t(0.01 * np.stack([syn.random_bl_coefficients(3, K, 40 + i) for i in range(2)])) if twolevel else None

    def solve():
        ctx = L.Context(L.Problem(N, K, nt=Nt, variant=variant, precision=L.FP32))
        ctx.set_images(t(I0), t(I1))
        v = torch.zeros((3,) + K, dtype=torch.float32, device="cuda")
        st, rep = ctx.gn_solve(v, max_gn=3, max_pcg=4, fixed_iters=True, Z=Z)
        ctx.close()
        return v, rep

    v_graph, r_graph = solve()
    monkeypatch.setenv("LDDMM_BL_NO_GRAPH", "1")
    v_eager, r_eager = solve()
    print(f"[gn] graph vs eager decisions {r_graph['decisions']} / {r_eager['decisions']}", flush=True)
    assert torch.equal(v_graph, v_eager)
    assert r_graph["E"] == r_eager["E"] and r_graph["decisions"] == r_eager["decisions"]
    assert r_graph["hess_matvecs"] == r_eager["hess_matvecs"] > 0
