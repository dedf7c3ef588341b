"""Every workgroup tile the brick autotuner can choose, against the FP64 oracle.

The autotuner times its candidates on the box it runs on, so any of them may end up
running the interpolation steps; each is fixed in turn through the tuner cache (the
boundary's tune_set) before the context of the shape is created.  Both shapes have
ragged tails on every axis for every tile; in the second every tile's block count is a
multiple of 8, so the bricks run with their XCD-ordered block mapping.  The displacement
of 0.8 voxel per step keeps the stencils in the staged bricks.  Tolerance: the FP32
trajectory bound of the other parity tests, rel-L2 <= 1e-5.
"""
import functools

import numpy as np
import pytest
import torch

from gpu_common import close, images, oracle_model, rel_l2, velocity
from paper_2006_06823_amd import lddmm_bl as L
from paper_2006_06823_amd import synthetic as syn

pytestmark = pytest.mark.gpu

SHAPES = [((40, 36, 44), (12, 10, 14)), ((28, 30, 36), (10, 10, 12))]
NT = 3


@functools.lru_cache(maxsize=None)
def references(N, K):
    I0, I1 = images(N, 7)
    v = velocity(N, K, NT, 8)
    dv = syn.random_bl_coefficients(3, K, 9)
    ref = {}
    for variant in (1, 3):
        om = oracle_model(variant, N, K, NT, I0, I1)
        om.setup(v)
        om.state()
        om.adjoint()
        ref[variant] = (om.gradient(), om.hess_matvec(dv))
    return I0, I1, v, dv, ref


@pytest.mark.parametrize("tile", range(8))
@pytest.mark.parametrize("N,K", SHAPES)
def test_every_brick_tile_matches_oracle(N, K, tile):
    assert L.tune_candidates("brick") == 8
    I0, I1, v, dv, ref = references(N, K)
    try:
        for key in L.brick_tune_keys(N):
            L.tune_set(key, tile)
        for variant in (1, 3):
            print(f"shape {N} tile {tile} variant {variant}", flush=True)
            ctx = L.Context(L.Problem(N, K, nt=NT, variant=variant, precision=L.FP32))
            assert all(L.tune_get(k) == tile for k in L.brick_tune_keys(N))
            dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device=ctx.device)
            ctx.set_images(dev(I0), dev(I1))
            ctx.state_solve(dev(v))
            g, _ = ctx.adjoint_solve()
            g_ref, h_ref = ref[variant]
            assert close(g, g_ref) <= 1e-5
            assert close(ctx.hess_matvec(dev(dv)), h_ref) <= 1e-5
    finally:
        for key in L.brick_tune_keys(N):
            L.tune_set(key, -1)


def test_dft_workgroup_caps_tuned_and_bitwise_equal():
    """A split-bf16 context (its DFT does not run the plane-wise path) times the workgroup caps of its
    first-axis contractions when it is created, under "dft:" keys.  A cap only changes how many column
    tiles each workgroup walks, so every candidate gives bitwise the same state, gradient and Hessian
    matvec: the smallest and the largest cap, forced on every such key, against the tuned choice."""
    N, K = (96, 96, 96), (32, 32, 32)
    I0, I1 = images(N, 11)
    v = velocity(N, K, NT, 12)
    dv = syn.random_bl_coefficients(3, K, 13)

    def run():
        ctx = L.Context(L.Problem(N, K, nt=NT, variant=3, precision=L.BF16_DFT))
        dev = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device=ctx.device)
        ctx.set_images(dev(I0), dev(I1))
        E, _ = ctx.state_solve(dev(v))
        g, _ = ctx.adjoint_solve()
        return E, g, ctx.hess_matvec(dev(dv))

    E0, g0, h0 = run()
    keys = [k for k in L.tune_table() if k.startswith("dft:")]
    print("dft keys:", {k: L.tune_get(k) for k in keys}, flush=True)
    assert keys and all(0 <= L.tune_get(k) < L.tune_candidates("dft") for k in keys)
    tuned = {k: L.tune_get(k) for k in keys}
    try:
        for choice in (0, L.tune_candidates("dft") - 1):
            for k in keys:
                L.tune_set(k, choice)
            print(f"dft caps forced to candidate {choice}", flush=True)
            E, g, h = run()
            assert E == E0
            assert torch.equal(g, g0)
            assert torch.equal(h, h0)
    finally:
        for k, c in tuned.items():
            L.tune_set(k, c)
