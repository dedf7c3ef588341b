"""Parity at the benchmark sizes, in the launch configuration bench.py times.

* Image-transport variant at 128^3 / band 32^3 / Nt = 10 (the Hessian-matvec benchmark): state,
  gradient and Hessian matvec against the full oracle (rel-L2 <= 1e-5).
* Deformation-state variant at 160 x 192 x 160 / band 40 x 48 x 40: at v = 0 the Hessian and the
  gradient have closed forms the oracle evaluates cheaply (L~ x + (2/sigma^2) pi(g1 (g1 . iota x)) and
  pi(-(2/sigma^2)(I0 - I1) g1), g1 = grad P(I0)); checked element-wise at full size.
"""
import numpy as np
import pytest
import torch

from gpu_common import close, oracle_model, rel_l2
from oracle import bspline, spectral as sp
from paper_2006_06823_amd import lddmm_bl as L
from paper_2006_06823_amd import synthetic as syn

pytestmark = pytest.mark.gpu


def test_variant1_128_full_oracle():
    N, K, Nt = (128, 128, 128), (32, 32, 32), 10
    I0, I1 = syn.phantom_pair_3d(N, seed=1, max_disp_vox=8.0)
    ctx = L.Context(L.Problem(N, K, nt=Nt, variant=L.IMAGE_TRANSPORT, precision=L.FP32))
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    ctx.set_images(t(I0), t(I1))
    vc = syn.random_bl_coefficients(3, K, seed=2)
    vg = sp.include(torch.tensor(vc), N)
    scale = torch.tensor([128.0] * 3, dtype=torch.float64).reshape(3, 1, 1, 1)
    v = vc * (8.0 / float((vg * scale).abs().max()))
    dv = syn.random_bl_coefficients(3, K, seed=3)
    E, m1 = ctx.state_solve(t(v), want_m1=True)
    g, _ = ctx.adjoint_solve()
    h = ctx.hess_matvec(t(dv))
    om = oracle_model(1, N, K, Nt, I0.astype(np.float64), I1.astype(np.float64))
    om.setup(v)
    om.state()
    assert close(m1, om.m[-1]) <= 1e-5
    om.adjoint()
    assert close(g, om.gradient()) <= 1e-5
    assert close(h, om.hess_matvec(dv)) <= 1e-5


def test_variant3_c3_size_zero_velocity_closed_forms():
    N, K, Nt = (160, 192, 160), (40, 48, 40), 10
    I0, I1 = syn.phantom_pair_3d(N, seed=2, max_disp_vox=8.0)
    ctx = L.Context(L.Problem(N, K, nt=Nt, variant=L.DEFORMATION_STATE, precision=L.FP32))
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    ctx.set_images(t(I0), t(I1))
    ctx.state_solve(torch.zeros((3,) + K, dtype=torch.float32, device="cuda"))
    g, _ = ctx.adjoint_solve()
    x = syn.random_bl_coefficients(3, K, seed=4)
    h = ctx.hess_matvec(t(x))
    I0d = torch.tensor(I0.astype(np.float64))
    _, gi = bspline.evaluate(bspline.prefilter(I0d, 3), bspline.grid_index(N), grad=True)
    g1 = gi * torch.tensor([float(n) for n in N], dtype=torch.float64).reshape(3, 1, 1, 1)
    g_ref = sp.project(-2.0 * (I0d - torch.tensor(I1.astype(np.float64))) * g1, K)
    assert close(g, g_ref) <= 1e-5
    xg = sp.include(torch.tensor(x), N)
    h_ref = sp.apply_L(torch.tensor(x), 3, 0.0025, 2) + 2.0 * sp.project(g1 * (g1 * xg).sum(0), K)
    assert close(h, h_ref) <= 1e-5


@pytest.mark.parametrize("variant", [1, 3])
def test_c3_size_constant_velocity_exact_shift(variant):
    """A constant velocity transports the image by an exact shift (Section 3.1: the characteristic of a
    constant field is x - dt v).  With a shift of whole voxels per step every interpolation hits grid
    nodes, where the cubic B-spline reproduces the samples, so m(1) = I0 rolled by the total shift; the
    data term follows in closed form.  Checked at the deformation-state benchmark size for both variants."""
    N, K, Nt = (160, 192, 160), (40, 48, 40), 10
    I0, I1 = syn.phantom_pair_3d(N, seed=2, max_disp_vox=8.0)
    ctx = L.Context(L.Problem(N, K, nt=Nt, variant=variant, precision=L.FP32))
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    ctx.set_images(t(I0), t(I1))
    shift = (10, -20, 30)  # voxels per unit time: (1, -2, 3) voxels per step
    v = np.zeros((3,) + K)
    for j in range(3):
        v[j, 0, 0, 0] = shift[j] / N[j]  # slot 0 holds the constant function 1
    E, m1 = ctx.state_solve(t(v), want_m1=True)
    ref = np.roll(I0.astype(np.float64), shift, axis=(0, 1, 2))
    assert close(m1, torch.tensor(ref)) <= 1e-5
    data = float(((ref - I1.astype(np.float64)) ** 2).mean())
    assert abs(E[2] - data) <= 1e-5 * data
    reg = 0.5 * sum(float(v[j, 0, 0, 0]) ** 2 for j in range(3))  # L~ = 1 on the constant slot
    assert abs(E[1] - reg) <= 1e-6 * reg


# --- full size at a sub-voxel velocity against stored oracle values ---------------------------------
import os  # noqa: E402
import sys  # noqa: E402

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_fullsize_golden as G  # noqa: E402


def _golden(name):
    path = G.golden_path(name)
    assert os.path.exists(path), f"stored oracle values missing: {path} (tests/golden/make_fullsize_golden.py)"
    return np.load(path, allow_pickle=False)


def test_c3_subvoxel_velocity_against_stored_oracle():
    """Deformation-state variant at 160 x 192 x 160 / band 40 x 48 x 40, Nt = 10, at a velocity of 0.8
    voxel per step, so every characteristic and interpolation falls between grid nodes (Table 1 rows 3,
    4, 7, 8; Section 3.1).  u~_n, m(1), the Jacobian map, the gradient and one Hessian matvec are compared
    with the FP64 oracle's values on a seeded sample of coefficients and nodes (the oracle takes tens of
    minutes at this size, so tests/golden/make_fullsize_golden.py stored them)."""
    z = _golden("c3")
    N, K, I0, I1, vseed, dseed, nsamp, _ = G.case("c3")
    assert tuple(z["N"]) == N and tuple(z["K"]) == K
    qi, pi = G.sample_indices(N, K, nsamp)
    v = G.scaled_velocity(N, K, vseed)
    dv = syn.random_bl_coefficients(3, K, dseed)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    print(f"[c3] {N} / {K}: state, Jacobian, adjoint, matvec", flush=True)
    ctx = L.Context(L.Problem(N, K, nt=G.NT, variant=L.DEFORMATION_STATE, precision=L.FP32))
    ctx.set_images(t(I0), t(I1))
    E, m1 = ctx.state_solve(t(v), want_m1=True)
    for j in range(3):
        assert abs(E[j] - z["E"][j]) <= 1e-5 * abs(z["E"][j])
    for n in (1, 5, G.NT):
        u = ctx.get_field(L.FIELD_STATE, n).double().cpu().numpy()
        assert close(u[qi], z[f"u{n}"], f"u~_{n}") <= 1e-5
    assert close(m1.reshape(-1).double().cpu().numpy()[pi], z["m1"], "m(1)") <= 1e-5
    (dmin, dmax), det = ctx.jacobian(want_map=True)
    assert close(det.reshape(-1).cpu().numpy()[pi], z["det"], "det") <= 1e-5
    assert abs(dmin - z["det_minmax"][0]) <= 1e-5 and abs(dmax - z["det_minmax"][1]) <= 1e-5 * z["det_minmax"][1]
    g, _ = ctx.adjoint_solve()
    assert close(g.reshape(-1).double().cpu().numpy()[qi], z["grad"], "gradient") <= 1e-5
    assert abs(float(g.double().norm()) - z["norms"][0]) <= 1e-5 * z["norms"][0]
    h = ctx.hess_matvec(t(dv))
    assert close(h.reshape(-1).double().cpu().numpy()[qi], z["hess"], "Hessian matvec") <= 1e-5
    assert abs(float(h.double().norm()) - z["norms"][1]) <= 1e-5 * z["norms"][1]
