"""Batched registration of subjects with uneven grids and bands in one lockstep solve (one HIP graph
launch per PCG iteration covering the subjects still iterating) equals the subjects solved one at a time, and the
single-subject GPU solves match the oracle (checked elsewhere)."""
import numpy as np
import pytest
import torch

from gpu_common import close, rel_l2
from paper_2006_06823_amd import lddmm_bl as L
from paper_2006_06823_amd import synthetic as syn

pytestmark = pytest.mark.gpu

SUBJECTS = [((32, 32, 32), (8, 8, 8)), ((40, 36, 44), (12, 10, 12)), ((48, 48, 48), (16, 16, 16))]


def _subject(i, N, K, template_seed=99):
    I0, I1 = syn.phantom_pair_3d(N, 1000 + i, max_disp_vox=2.0, template_seed=template_seed)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    return t(I0), t(I1)


@pytest.mark.parametrize("variant", [1, 3])
def test_batched_equals_individual(variant):
    probs, I0s, I1s, vs = [], [], [], []
    for i, (N, K) in enumerate(SUBJECTS):
        probs.append(L.Problem(N, K, nt=4, variant=variant, precision=L.FP32))
        a, b = _subject(i, N, K)
        I0s.append(a)
        I1s.append(b)
        vs.append(torch.zeros((3,) + K, dtype=torch.float32, device="cuda"))
    st, reps = L.gn_solve_batched(probs, I0s, I1s, vs, max_gn=3, max_pcg=3, fixed_iters=True)
    for i, p in enumerate(probs):
        ctx = L.Context(p)
        ctx.set_images(I0s[i], I1s[i])
        v = torch.zeros_like(vs[i])
        st1, rep = ctx.gn_solve(v, max_gn=3, max_pcg=3, fixed_iters=True)
        assert reps[i]["gn_iters"] == rep["gn_iters"]
        assert reps[i]["backtracks"] == rep["backtracks"]
        assert close(vs[i], v) <= 1e-6
        assert abs(reps[i]["E"] - rep["E"]) <= 1e-6 * abs(rep["E"])
        assert reps[i]["E"] < reps[i]["E0"]


def test_batched_eager_branches_equal_graph(monkeypatch):
    """More subjects than branch streams (10 over 8): the matvecs launched eagerly on the branches
    (LDDMM_BL_NO_GRAPH) and replayed from the captured graph give bitwise the same registrations."""
    shapes = [((24 + 4 * (i % 3), 24, 28), (8, 8, 8)) for i in range(10)]

    def run():
        probs, I0s, I1s, vs = [], [], [], []
        for i, (N, K) in enumerate(shapes):
            probs.append(L.Problem(N, K, nt=3, variant=L.DEFORMATION_STATE, precision=L.FP32))
            a, b = _subject(i, N, K)
            I0s.append(a)
            I1s.append(b)
            vs.append(torch.zeros((3,) + K, dtype=torch.float32, device="cuda"))
        st, reps = L.gn_solve_batched(probs, I0s, I1s, vs, max_gn=2, max_pcg=2, fixed_iters=True)
        return vs, reps

    vg, rg = run()
    monkeypatch.setenv("LDDMM_BL_NO_GRAPH", "1")
    ve, re_ = run()
    for a, b, x, y in zip(vg, ve, rg, re_):
        assert torch.equal(a, b)
        assert (x["E"], x["gn_iters"], x["backtracks"]) == (y["E"], y["gn_iters"], y["backtracks"])
        assert x["E"] < x["E0"]


@pytest.mark.parametrize("variant", [1, 3])
def test_batched_converging_subjects_equal_individual(variant):
    """Without fixed iteration counts the subjects stop at different Gauss-Newton and PCG iterations
    (an easy pair with a small displacement next to harder ones); a subject whose PCG or Gauss-Newton
    loop has stopped leaves the launched work, and every subject's registration still equals its
    one-at-a-time solve."""
    disp = [0.5, 2.0, 3.0, 1.0]
    shapes = [((32, 32, 32), (8, 8, 8)), ((40, 36, 44), (12, 10, 12)), ((48, 48, 48), (16, 16, 16)),
              ((32, 40, 32), (12, 12, 12))]
    probs, I0s, I1s, vs = [], [], [], []
    for i, (N, K) in enumerate(shapes):
        probs.append(L.Problem(N, K, nt=4, variant=variant, precision=L.FP32))
        I0, I1 = syn.phantom_pair_3d(N, 2000 + i, max_disp_vox=disp[i], template_seed=7)
        t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
        I0s.append(t(I0))
        I1s.append(t(I1))
        vs.append(torch.zeros((3,) + K, dtype=torch.float32, device="cuda"))
    st, reps = L.gn_solve_batched(probs, I0s, I1s, vs, max_gn=8, max_pcg=12, grad_rtol=5e-2)
    iters = set()
    for i, p in enumerate(probs):
        ctx = L.Context(p)
        ctx.set_images(I0s[i], I1s[i])
        v = torch.zeros_like(vs[i])
        st1, rep = ctx.gn_solve(v, max_gn=8, max_pcg=12, grad_rtol=5e-2)
        print(f"subject {i}: gn {rep['gn_iters']} pcg {rep['pcg_iters_total']} E {rep['E']:.6g}/{rep['E0']:.6g}")
        assert (reps[i]["gn_iters"], reps[i]["pcg_iters_total"], reps[i]["backtracks"]) == \
            (rep["gn_iters"], rep["pcg_iters_total"], rep["backtracks"])
        assert close(vs[i], v) <= 1e-6
        assert abs(reps[i]["E"] - rep["E"]) <= 1e-6 * abs(rep["E"])
        iters.add((rep["gn_iters"], rep["pcg_iters_total"]))
    assert len(iters) > 1  # the subjects did stop at different iterations
