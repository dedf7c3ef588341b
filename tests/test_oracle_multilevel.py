"""Pins of the oracle's two-level spectral preconditioner (the multi-level preconditioning the paper's
Discussion names as the next step; the reading is stated in oracle/multilevel.py).

* band restriction and extension: R E = I, and E R c is the low-pass of c computed independently through
  the complex Fourier coefficients (frequencies above the coarse band zeroed);
* image restriction: block means checked by brute force;
* with constant images the data term of the Gauss-Newton Hessian vanishes, H = L~, and the preconditioner
  is exactly L~^-1 (its inner solve is exact after one iteration);
* flexible CG with a fixed SPD preconditioner takes the PCG iterates;
* in a Gauss-Newton run the two-level preconditioner lowers the gradient further than L~^-1 alone.
"""
import math

import numpy as np
import torch

from oracle import spectral as sp
from oracle.gauss_newton import gauss_newton, pcg
from oracle.multilevel import TwoLevel, coarse_sizes, extend_band, restrict_band, restrict_image
from oracle.problem import Problem
from oracle.variant1 import Variant1
from oracle.variant3 import Variant3
from paper_2006_06823_amd import synthetic as syn

torch.set_num_threads(min(8, torch.get_num_threads()))


def test_band_restriction_and_extension():
    K, Kc = (12, 10, 16), (6, 4, 8)
    c = torch.tensor(syn.random_bl_coefficients(3, K, 1))
    cc = restrict_band(c, Kc)
    assert float((restrict_band(extend_band(cc, K), Kc) - cc).abs().max()) == 0.0
    low = extend_band(cc, K)
    # independent: the complex coefficients with |k_j| > Kc_j / 2 - 1 on any axis zeroed
    ch = sp.to_complex(c, 3)
    for j in range(3):
        f = sp.freqs(K[j]).abs() > (Kc[j] // 2 - 1)
        shape = [1, 1, 1]
        shape[j] = K[j] - 1
        ch = ch * (~f).reshape(shape).to(ch.dtype)
    ref = sp.from_complex(ch, K)
    assert float((low - ref).abs().max()) < 1e-13


def test_image_restriction_block_means():
    rng = np.random.default_rng(3)
    f = rng.normal(size=(6, 4, 8))
    r = restrict_image(f, 3).numpy()
    for a in range(3):
        for b in range(2):
            for c in range(4):
                assert abs(r[a, b, c] - f[2 * a:2 * a + 2, 2 * b:2 * b + 2, 2 * c:2 * c + 2].mean()) < 1e-15


def test_two_level_is_regulariser_inverse_without_data_term():
    prob = Problem((32, 24), (12, 8), Nt=4)
    I0 = np.full((32, 24), 0.3)
    for V in (Variant1, Variant3):
        pre = TwoLevel(V, prob, I0, I0, inner=3)
        v = torch.tensor(syn.random_bl_coefficients(2, prob.K, 2)) * 1e-2
        pre.set_velocity(v)
        r = torch.tensor(syn.random_bl_coefficients(2, prob.K, 4))
        ref = sp.apply_L(r, 2, prob.alpha, prob.s, inverse=True)
        assert float((pre(r) - ref).abs().max()) < 1e-13 * float(ref.abs().max())


def test_flexible_cg_equals_pcg_for_a_fixed_preconditioner():
    rng = np.random.default_rng(5)
    B = rng.normal(size=(40, 40))
    A = torch.tensor(B @ B.T + 40 * np.eye(40))
    Dinv = torch.tensor(1.0 / (1.0 + np.arange(40.0)))
    b = torch.tensor(rng.normal(size=40))
    mv = lambda x: A @ x
    pre = lambda r: Dinv * r
    x1, _, _, _ = pcg(mv, b, pre, 0.0, 8, fixed=True)
    x2, _, _, _ = pcg(mv, b, pre, 0.0, 8, fixed=True, flexible=True)
    assert float((x1 - x2).norm()) <= 1e-8 * float(x1.norm())


def test_two_level_with_exact_inner_solve_is_block_newton_step():
    """With as many inner iterations as the coarse band has live unknowns, the inner PCG reaches the coarse
    Newton step: M^-1 r = L~^-1 (r - E R r) + E C^-1 R r with C^-1 from a dense solve of the coarse Hessian
    (assembled column by column on the live slots, the pad slots being outside the band).  At v = 0, where
    the optimise-then-discretise Hessian is exactly symmetric, so that PCG ends at the solution."""
    prob = Problem((16, 16), (8, 8), Nt=3)
    I0, I1 = syn.blob_pair_2d(16, 1, 1.0)
    v = torch.zeros((2,) + prob.K, dtype=torch.float64)
    Nc, Kc = coarse_sizes(prob.N, prob.K)
    live = torch.zeros((2,) + Kc, dtype=torch.bool)
    live[:, :Kc[0] - 1, :Kc[1] - 1] = True
    nlive = int(live.sum())
    pre = TwoLevel(Variant3, prob, I0, I1, inner=nlive)
    pre.set_velocity(v)
    cols = []
    for i in range(nlive):
        e = torch.zeros(nlive, dtype=torch.float64)
        e[i] = 1.0
        x = torch.zeros((2,) + Kc, dtype=torch.float64)
        x[live] = e
        cols.append(pre.coarse.hess_matvec(x)[live])
    C = torch.stack(cols, 1)
    r = torch.tensor(syn.random_bl_coefficients(2, prob.K, 7))
    rc = restrict_band(r, Kc)
    xc = torch.zeros((2,) + Kc, dtype=torch.float64)
    xc[live] = torch.linalg.solve(C, rc[live])
    ref = sp.apply_L(r - extend_band(rc, prob.K), 2, prob.alpha, prob.s, inverse=True) + extend_band(xc, prob.K)
    assert float((pre(r) - ref).norm()) <= 1e-8 * float(ref.norm())


def test_two_level_gauss_newton_decreases_the_energy():
    """The two-level preconditioned Gauss-Newton iteration is a descent method (monotone energy, smaller
    gradient at the end); whether it beats L~^-1 alone depends on the problem (printed, not asserted)."""
    prob = Problem((64, 64), (16, 16), Nt=5)
    I0, I1 = syn.blob_pair_2d(64, 0, 4.0)
    out = {}
    for name in ("plain", "two-level"):
        model = Variant3(prob, I0, I1)
        pre = TwoLevel(Variant3, prob, I0, I1, inner=5) if name == "two-level" else None
        v, rep = gauss_newton(model, np.zeros((2, 16, 16)), max_gn=4, max_pcg=3, fixed_iters=True, precond=pre)
        Es = [h["E"] for h in rep.history] + [rep.E]
        assert all(b <= a for a, b in zip(Es, Es[1:]))
        assert rep.grad_inf_rel < 0.05 and rep.E < 0.5 * rep.E0
        out[name] = (rep.grad_inf_rel, rep.E)
    print("[two-level] (rel grad, E) after 4 GN x 3 PCG:", out)
