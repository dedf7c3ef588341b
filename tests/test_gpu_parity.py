"""GPU-vs-oracle parity of the HIP library, called through its C ABI.

Tolerances: FP32 truncated DFT rel-L2 <= 1e-6; FP32 trajectories, gradients
and Hessian-vector products rel-L2 <= 1e-5; FP64 (the 2D configuration)
<= 1e-10.  Sizes span several 32-wide tiles with ragged tails.
"""
import numpy as np
import pytest
import torch

from gpu_common import close, images, oracle_model, rel_l2, velocity
from oracle import spectral as sp
from paper_2006_06823_amd import lddmm_bl as L

pytestmark = pytest.mark.gpu

CASES = [
    # (dim, N, K, Nt, precision)
    (3, (40, 36, 44), (12, 10, 14), 4, L.FP32),
    (2, (64, 64), (16, 16), 10, L.FP64),
    (2, (48, 40), (14, 12), 5, L.FP32),
]


def tol(precision, kind="traj"):
    if precision == L.FP64:
        return 1e-10
    return 1e-6 if kind == "dft" else 1e-5


def dev(x, ctx):
    return torch.tensor(np.ascontiguousarray(x), dtype=ctx.dtype, device=ctx.device)


def make(variant, dim, N, K, Nt, precision, seed=0, cfl=0.8):
    I0, I1 = images(N, seed)
    ctx = L.Context(L.Problem(N, K, nt=Nt, variant=variant, precision=precision))
    ctx.set_images(dev(I0, ctx), dev(I1, ctx))
    v = velocity(N, K, Nt, seed + 1, cfl_vox=cfl)
    om = oracle_model(variant, N, K, Nt, I0, I1)
    return ctx, om, v


# first-axis shapes of every DFT kernel path: expansion (K0 <= 64), contraction with one and two
# 32-row output tiles (64 < N0 <= 192, K0 <= 32 / K0 > 32), ragged tails on every axis
DFT_CASES = CASES + [
    (3, (80, 36, 44), (40, 12, 14), 4, L.FP32),
    (3, (100, 20, 70), (24, 12, 30), 4, L.FP32),
    # an inner axis longer than the fused inner-axis kernels take (192): the separable float path
    (3, (20, 24, 200), (8, 10, 36), 2, L.FP32),
    # inner-axis matrices too large to stage in 64 KB of LDS: the fused kernels read them from global
    # memory (the projection for every field count, the expansion for 7 fields)
    (3, (40, 72, 192), (16, 48, 48), 2, L.FP32),
    # more row splits x fields x first-axis slabs than one round of workgroups holds: with 3 and 7
    # fields the projection's workgroups walk 2 and 3 slabs each (the last ones fewer)
    (3, (128, 192, 64), (64, 16, 16), 2, L.FP32),
]


@pytest.mark.parametrize("dim,N,K,Nt,precision", DFT_CASES)
def test_truncated_dft_parity(dim, N, K, Nt, precision):
    ctx = L.Context(L.Problem(N, K, nt=Nt, precision=precision))
    rng = np.random.default_rng(5)
    for nf in (1, 3, 7):
        f = rng.standard_normal((nf,) + tuple(N))
        got = ctx.project(dev(f, ctx).reshape((nf,) + tuple(N)) if nf > 1 else dev(f[0], ctx), nf)
        ref = sp.project(torch.tensor(f), K)
        assert close(got.reshape(ref.shape), ref) <= tol(precision, "dft")
        c = np.stack([np.random.default_rng(s).standard_normal(K) for s in range(nf)])
        for j, k in enumerate(K):
            sl = [slice(None)] * (dim + 1)
            sl[j + 1] = k - 1
            c[tuple(sl)] = 0.0
        got = ctx.include(dev(c, ctx) if nf > 1 else dev(c[0], ctx), nf)
        ref = sp.include(torch.tensor(c), N)
        assert close(got.reshape(ref.shape), ref) <= tol(precision, "dft")


@pytest.mark.parametrize("N,K", [((256, 256, 256), (64, 64, 64)), ((250, 252, 254), (62, 60, 64))])
def test_truncated_dft_parity_largest_grid(N, K):
    """The largest grid and band of the kernels' envelope (band 64 per axis, two 32-row tiles on every
    axis, 8 x 8 column tiles per plane) and a ragged one just below it: projection and inclusion of one
    field and of three against the FP64 oracle's FFT."""
    ctx = L.Context(L.Problem(N, K, nt=1, precision=L.FP32))
    rng = np.random.default_rng(9)
    for nf in (1, 3):
        print(f"[largest grid] N {N} K {K} fields {nf}", flush=True)
        f = rng.standard_normal((nf,) + tuple(N)).astype(np.float32)
        got = ctx.project(dev(f, ctx) if nf > 1 else dev(f[0], ctx), nf)
        ref = sp.project(torch.tensor(f, dtype=torch.float64), K)
        assert close(got.reshape(ref.shape), ref, f"project {N}") <= tol(L.FP32, "dft")
        c = rng.standard_normal((nf,) + tuple(K))
        for j, k in enumerate(K):
            sl = [slice(None)] * 4
            sl[j + 1] = k - 1
            c[tuple(sl)] = 0.0
        got = ctx.include(dev(c, ctx) if nf > 1 else dev(c[0], ctx), nf)
        ref = sp.include(torch.tensor(c), N)
        assert close(got.reshape(ref.shape), ref, f"include {N}") <= tol(L.FP32, "dft")
    ctx.close()


@pytest.mark.parametrize("variant", [1, 3])
@pytest.mark.parametrize("dim,N,K,Nt,precision", CASES)
def test_state_adjoint_gradient_parity(variant, dim, N, K, Nt, precision):
    ctx, om, v = make(variant, dim, N, K, Nt, precision)
    E, m1 = ctx.state_solve(dev(v, ctx), want_m1=True)
    om.setup(v)
    om.state()
    Eo = [float(x) for x in om.objective()]
    # characteristics and divergence
    assert close(ctx.get_field(L.FIELD_DEP_BACKWARD).reshape(om.Xb.shape), om.Xb) <= tol(precision)
    assert close(ctx.get_field(L.FIELD_DEP_FORWARD).reshape(om.Xf.shape), om.Xf) <= tol(precision)
    assert close(ctx.get_field(L.FIELD_DIV_V).reshape(om.divv.shape), om.divv) <= tol(precision)
    # state trajectory
    if variant == 1:
        for n in range(Nt + 1):
            assert close(ctx.get_field(L.FIELD_STATE, n).reshape(om.m[n].shape), om.m[n]) <= tol(precision)
        m1o = om.m[-1]
    else:
        for n in range(1, Nt + 1):
            assert close(ctx.get_field(L.FIELD_STATE, n).reshape(om.u[n].shape), om.u[n]) <= tol(precision)
        m1o = om.m1
    assert close(m1, m1o) <= tol(precision)
    for a, b in zip(E, Eo):
        assert abs(a - b) <= tol(precision) * abs(b) * 10
    # adjoint and gradient
    g, ginf = ctx.adjoint_solve()
    om.adjoint()
    go = om.gradient()
    if variant == 1:
        assert close(ctx.get_field(L.FIELD_ADJOINT0).reshape(om.lam[0].shape), om.lam[0]) <= tol(precision)
    else:
        assert close(ctx.get_field(L.FIELD_ADJOINT0).reshape(om.rho[0].shape), om.rho[0]) <= tol(precision)
    assert close(g, go) <= tol(precision)
    ginf_o = float(sp.include(go, N).abs().max())
    assert abs(ginf - ginf_o) <= tol(precision) * ginf_o * 10


@pytest.mark.parametrize("variant", [1, 3])
def test_large_displacement_parity(variant):
    """Departure points more than a voxel away (2.5 voxels per step): the interpolation leaves its
    staged brick and gathers from global memory; results still match the oracle."""
    N, K, Nt = (40, 36, 44), (12, 10, 14), 3
    ctx, om, v = make(variant, 3, N, K, Nt, L.FP32, seed=4, cfl=2.5)
    ctx.state_solve(dev(v, ctx))
    om.setup(v)
    om.state()
    assert close(ctx.get_field(L.FIELD_DEP_BACKWARD).reshape(om.Xb.shape), om.Xb) <= 1e-5
    g, _ = ctx.adjoint_solve()
    om.adjoint()
    assert close(g, om.gradient()) <= 1e-5
    from paper_2006_06823_amd import synthetic as syn
    dv = syn.random_bl_coefficients(3, K, 12)
    assert close(ctx.hess_matvec(dev(dv, ctx)), om.hess_matvec(dv)) <= 1e-5


@pytest.mark.parametrize("variant", [1, 3])
@pytest.mark.parametrize("dim,N,K,Nt,precision", CASES)
def test_hess_matvec_parity(variant, dim, N, K, Nt, precision):
    ctx, om, v = make(variant, dim, N, K, Nt, precision)
    ctx.state_solve(dev(v, ctx))
    om.setup(v)
    om.state()
    from paper_2006_06823_amd import synthetic as syn
    dv = syn.random_bl_coefficients(dim, K, 11)
    h = ctx.hess_matvec(dev(dv, ctx))
    ho = om.hess_matvec(dv)
    assert close(h, ho) <= tol(precision)
    dm, dl = om.last_inc
    for n in (1, Nt // 2, Nt):
        got = ctx.get_field(L.FIELD_INC_STATE, n).reshape(dm[n].shape)
        assert close(got, dm[n]) <= tol(precision)
    for n in (0, Nt // 2, Nt):
        got = ctx.get_field(L.FIELD_INC_ADJOINT, n).reshape(dl[n].shape)
        assert close(got, dl[n]) <= tol(precision)


# image-transport Hessian on grids with a long first axis (first-axis contractions of one and two
# 32-slot tiles, odd and ragged second and third axes); a CFL of 1.9 voxels sends part of the
# departure points out of the staged interpolation bricks to the global gather
LONG_AXIS_CASES = [((96, 21, 36), (24, 12, 14), 4, 0.8), ((100, 18, 40), (40, 10, 12), 3, 1.9)]


@pytest.mark.parametrize("N,K,Nt,cfl", LONG_AXIS_CASES)
def test_hess_matvec_parity_long_first_axis(N, K, Nt, cfl):
    ctx, om, v = make(1, 3, N, K, Nt, L.FP32, seed=6, cfl=cfl)
    ctx.state_solve(dev(v, ctx))
    om.setup(v)
    om.state()
    from paper_2006_06823_amd import synthetic as syn
    dv = syn.random_bl_coefficients(3, K, 13)
    h = ctx.hess_matvec(dev(dv, ctx))
    assert close(h, om.hess_matvec(dv)) <= 1e-5
    dm, dl = om.last_inc
    for n in (1, Nt):
        assert close(ctx.get_field(L.FIELD_INC_STATE, n).reshape(dm[n].shape), dm[n]) <= 1e-5
    for n in (0, Nt - 1):
        assert close(ctx.get_field(L.FIELD_INC_ADJOINT, n).reshape(dl[n].shape), dl[n]) <= 1e-5


@pytest.mark.parametrize("variant", [1, 3])
def test_hess_matvec_parity_separable_dft_path(variant):
    """An inner axis above 192 points: every ι / π of the solves and the matvec runs as three
    separate axis contractions instead of the fused inner-axis kernels."""
    N, K, Nt = (20, 24, 200), (8, 10, 36), 2
    ctx, om, v = make(variant, 3, N, K, Nt, L.FP32, seed=9)
    ctx.state_solve(dev(v, ctx))
    om.setup(v)
    om.state()
    g, _ = ctx.adjoint_solve()
    om.adjoint()
    assert close(g, om.gradient()) <= 1e-5
    from paper_2006_06823_amd import synthetic as syn
    dv = syn.random_bl_coefficients(3, K, 14)
    assert close(ctx.hess_matvec(dev(dv, ctx)), om.hess_matvec(dv)) <= 1e-5


# degenerate and odd configurations: one time step, a band with a single real mode on one axis
# (K_j = 2: the constant and the pad slot), odd grid sizes on every axis
SMALL_CASES = [((12, 10, 14), (4, 2, 4), 1), ((17, 9, 33), (6, 4, 10), 2)]


@pytest.mark.parametrize("variant", [1, 3])
@pytest.mark.parametrize("N,K,Nt", SMALL_CASES)
def test_small_and_odd_configurations(variant, N, K, Nt):
    ctx, om, v = make(variant, 3, N, K, Nt, L.FP32, seed=12)
    ctx.state_solve(dev(v, ctx))
    om.setup(v)
    om.state()
    g, _ = ctx.adjoint_solve()
    om.adjoint()
    assert close(g, om.gradient()) <= 1e-5
    from paper_2006_06823_amd import synthetic as syn
    dv = syn.random_bl_coefficients(3, K, 15)
    assert close(ctx.hess_matvec(dev(dv, ctx)), om.hess_matvec(dv)) <= 1e-5


def test_dot_fp64_reduction():
    """Device FP64 reductions over FP32 data equal the sum computed in double on the host (1e-12)."""
    ctx = L.Context(L.Problem((32, 32, 32), (8, 8, 8), precision=L.FP32))
    rng = np.random.default_rng(3)
    a = rng.standard_normal(1_000_003).astype(np.float32)
    b = rng.standard_normal(1_000_003).astype(np.float32)
    got = ctx.dot(torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda"))
    ref = float(np.dot(a.astype(np.float64), b.astype(np.float64)))
    assert abs(got - ref) <= 1e-12 * np.sqrt(len(a)) * max(1.0, abs(ref))


@pytest.mark.parametrize("variant", [1, 3])
def test_bf16_dft_error_vs_oracle(variant):
    """Split-bf16 truncated DFT (first-axis stages on bf16 matrix cores, float accumulation): the errors
    against the FP64 oracle are stated, not held to the float tolerance; the bound here (5e-4) is what
    the 16-bit-per-operand split guarantees with margin for 10-step sweeps."""
    N, K, Nt = (40, 36, 44), (12, 10, 14), 4
    I0, I1 = images(N, 0)
    ctx = L.Context(L.Problem(N, K, nt=Nt, variant=variant, precision=L.BF16_DFT))
    ctx.set_images(dev(I0, ctx), dev(I1, ctx))
    v = velocity(N, K, Nt, 1)
    om = oracle_model(variant, N, K, Nt, I0, I1)
    E, m1 = ctx.state_solve(dev(v, ctx), want_m1=True)
    om.setup(v)
    om.state()
    g, _ = ctx.adjoint_solve()
    om.adjoint()
    from paper_2006_06823_amd import synthetic as syn
    dv = syn.random_bl_coefficients(3, K, 11)
    h = ctx.hess_matvec(dev(dv, ctx))
    errs = {"m1": rel_l2(m1, om.m[-1] if variant == 1 else om.m1), "grad": rel_l2(g, om.gradient()),
            "hess": rel_l2(h, om.hess_matvec(dv))}
    print("bf16 split-DFT rel-L2 errors", variant, errs)
    assert max(errs.values()) <= 5e-4


def test_bf16_dft_parity_walking_expansion():
    """Split-bf16 first-axis stages of pi / iota on a grid with more column tiles than one round of
    workgroups holds: with 3 and 7 fields every expansion workgroup walks several tiles (1 field:
    one tile each). Held to the split-bf16 bound of the test above."""
    N, K = (80, 128, 128), (24, 16, 16)
    ctx = L.Context(L.Problem(N, K, nt=2, precision=L.BF16_DFT))
    rng = np.random.default_rng(8)
    for nf in (1, 3, 7):
        f = rng.standard_normal((nf,) + N)
        got = ctx.project(dev(f, ctx), nf) if nf > 1 else ctx.project(dev(f[0], ctx), 1)
        ref = sp.project(torch.tensor(f), K)
        assert close(got.reshape(ref.shape), ref) <= 5e-4
        c = rng.standard_normal((nf,) + K)
        for j, k in enumerate(K):
            sl = [slice(None)] * 4
            sl[j + 1] = k - 1
            c[tuple(sl)] = 0.0
        got = ctx.include(dev(c, ctx), nf) if nf > 1 else ctx.include(dev(c[0], ctx), 1)
        ref = sp.include(torch.tensor(c), N)
        assert close(got.reshape(ref.shape), ref) <= 5e-4


@pytest.mark.parametrize("dim,N,K,Nt,precision", CASES)
def test_jacobian_parity(dim, N, K, Nt, precision):
    """det(I - D iota(u~(1))) in double on the device vs the oracle, element-wise (both variants'
    contexts; the image-transport one integrates u~ on demand)."""
    from oracle.gauss_newton import displacement_state, jacobian_det
    from oracle.problem import Problem as OP
    for variant in (1, 3):
        ctx, om, v = make(variant, dim, N, K, Nt, precision, cfl=1.5)
        ctx.state_solve(dev(v, ctx))
        (dmin, dmax), det = ctx.jacobian(want_map=True)
        prob = OP(tuple(N), tuple(K), Nt=Nt)
        ref = jacobian_det(prob, displacement_state(prob, v))
        tol_abs = 1e-10 if precision == L.FP64 else 2e-5
        assert float((det.cpu() - ref).abs().max()) <= tol_abs
        assert abs(dmin - float(ref.min())) <= tol_abs and abs(dmax - float(ref.max())) <= tol_abs


@pytest.mark.parametrize("variant", [1, 3])
def test_fused_product_grid_pass_equals_separate_kernels(variant, monkeypatch):
    """The product-grid products (fl = x div v and the gradient / Hessian terms) formed by the fused
    per-plane pass and by the separate expansion and reduction kernels (LDDMM_BL_NO_PROD_FUSE): both
    against the oracle, and against each other to rounding.  The product grid (32 x 40 x 48 for this
    band) spans four ragged 32 x 32 tiles per plane, whose partials the fused pass sums in pairs."""
    N, K, Nt = (64, 72, 80), (20, 24, 30), 3
    from paper_2006_06823_amd import synthetic as syn
    dv = syn.random_bl_coefficients(3, K, 15)
    out = []
    for fused in (True, False):
        if not fused:
            monkeypatch.setenv("LDDMM_BL_NO_PROD_FUSE", "1")
        ctx, om, v = make(variant, 3, N, K, Nt, L.FP32, seed=12)
        ctx.state_solve(dev(v, ctx))
        g, _ = ctx.adjoint_solve()
        h = ctx.hess_matvec(dev(dv, ctx))
        out.append((g, h))
    om.setup(v)
    om.state()
    om.adjoint()
    for g, h in out:
        assert close(g, om.gradient()) <= 1e-5
        assert close(h, om.hess_matvec(dv)) <= 1e-5
    assert close(out[0][0], out[1][0]) <= 1e-6
    assert close(out[0][1], out[1][1]) <= 1e-6


def test_hess_matvec_graphs_on_caller_buffers(monkeypatch):
    """lddmm_bl_hess_matvec replays graphs captured on the caller's buffers (the four most recent pointer
    pairs): against eager launches (LDDMM_BL_NO_GRAPH) bitwise, for six pairs (the first ones dropped and
    captured again) and for new contents in a cached pair's input; one buffer as both dv and h is
    refused."""
    from paper_2006_06823_amd import synthetic as syn
    N, K, Nt = (40, 36, 44), (12, 10, 14), 4
    dvs = [syn.random_bl_coefficients(3, K, 30 + i) for i in range(7)]

    def run():
        ctx, om, v = make(1, 3, N, K, Nt, L.FP32, seed=3)
        ctx.state_solve(dev(v, ctx))
        ins = [dev(d, ctx) for d in dvs[:6]]
        outs = [torch.empty_like(ins[0]) for _ in range(6)]
        res = []
        for _ in range(2):
            for a, b in zip(ins, outs):
                ctx.hess_matvec(a, out=b)
                res.append(b.clone())
        ins[0].copy_(dev(dvs[6], ctx))
        res.append(ctx.hess_matvec(ins[0], out=outs[0]).clone())
        x = dev(dvs[1], ctx)
        with pytest.raises(L.LddmmError):
            ctx.hess_matvec(x, out=x)
        return res

    graph = run()
    monkeypatch.setenv("LDDMM_BL_NO_GRAPH", "1")
    eager = run()
    for a, b in zip(graph, eager):
        assert torch.equal(a, b)
    assert torch.equal(graph[0], graph[6]) and not torch.equal(graph[12], graph[0])


def test_hess_matvec_enqueued_on_the_stream():
    """lddmm_bl_hess_matvec only enqueues its work: eight calls on one (dv, h) pair whose input is
    rewritten by the caller's own stream between them, with no host wait anywhere, give bitwise the
    results of the same calls each followed by a device synchronisation."""
    from paper_2006_06823_amd import synthetic as syn
    N, K, Nt = (40, 36, 44), (12, 10, 14), 4
    ctx, om, v = make(1, 3, N, K, Nt, L.FP32, seed=5)
    ctx.state_solve(dev(v, ctx))
    srcs = [dev(syn.random_bl_coefficients(3, K, 60 + i), ctx) for i in range(8)]
    a = torch.empty_like(srcs[0])
    b = torch.empty_like(srcs[0])
    ref = []
    for s_ in srcs:
        a.copy_(s_)
        ctx.hess_matvec(a, out=b)
        torch.cuda.synchronize()
        ref.append(b.clone())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        got = []
        for s_ in srcs:
            a.copy_(s_)
            ctx.hess_matvec(a, out=b)
            got.append(b.clone())
    torch.cuda.synchronize()
    for x, y in zip(got, ref):
        assert torch.equal(x, y)
    assert not torch.equal(ref[0], ref[1])
