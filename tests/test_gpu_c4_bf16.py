"""The uneven-grid batch with the split-bf16 truncated DFT against the FP64 oracle, at real subject sizes.

Four subjects of the batch (N = 96, 144, 176, 192 with bands 32, 40, 48, 48; deformation-state variant,
Nt = 10, velocities of 0.8 voxel per step) are checked at a fixed velocity: u~(1), m(1), the gradient and
one Hessian matvec of a split-bf16 context and of an FP32 context against the oracle's values stored by
tests/golden/make_fullsize_golden.py (seeded samples of coefficients and nodes).  The split carries 16
mantissa bits of each operand (hi + lo bf16), a relative operand error of at most 2^-17 = 7.6e-6 per
product; the contraction sums of length <= 192 average these errors, and the measured errors sit at
0.9-2.6e-6 rel-L2 and <= 1e-5 element-wise, so the split-bf16 path is held to the FP32 bound (rel-L2
<= 1e-5, element-wise <= 1e-4).  Then the batched Gauss-Newton-Krylov solve of the four subjects (one
HIP graph per PCG iteration over all of them) equals the subjects solved one at a time."""
import os
import sys

import numpy as np
import pytest
import torch

from gpu_common import close
from paper_2006_06823_amd import lddmm_bl as L
from paper_2006_06823_amd import synthetic as syn

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_fullsize_golden as G  # noqa: E402

pytestmark = pytest.mark.gpu

BF16_BOUND = 1e-5  # split-bf16, see the module docstring
FP32_BOUND = 1e-5


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


@pytest.mark.parametrize("subject", G.C4_SUBJECTS)
def test_subject_against_stored_oracle(subject):
    name = f"c4_{subject}"
    path = G.golden_path(name)
    assert os.path.exists(path), f"stored oracle values missing: {path}"
    z = np.load(path, allow_pickle=False)
    N, K, I0, I1, vseed, dseed, nsamp, _ = G.case(name)
    assert tuple(z["N"]) == N and tuple(z["K"]) == K
    qi, pi = G.sample_indices(N, K, nsamp)
    v, dv = G.scaled_velocity(N, K, vseed), syn.random_bl_coefficients(3, K, dseed)
    for prec, bound in ((L.BF16_DFT, BF16_BOUND), (L.FP32, FP32_BOUND)):
        tag = f"subject {subject} {N[0]}^3/{K[0]} {'bf16-split' if prec == L.BF16_DFT else 'fp32'}"
        print(f"[c4] {tag}", flush=True)
        ctx = L.Context(L.Problem(N, K, nt=G.NT, variant=L.DEFORMATION_STATE, precision=prec))
        ctx.set_images(_t(I0), _t(I1))
        E, m1 = ctx.state_solve(_t(v), want_m1=True)
        print(f"[parity] {tag} objective rel {abs(E[0] - z['E'][0]) / abs(z['E'][0]):.3e}", flush=True)
        assert abs(E[0] - z["E"][0]) <= bound * abs(z["E"][0])
        u = ctx.get_field(L.FIELD_STATE, G.NT).double().cpu().numpy()
        assert close(u[qi], z[f"u{G.NT}"], f"{tag} u~(1)") <= bound
        assert close(m1.reshape(-1).double().cpu().numpy()[pi], z["m1"], f"{tag} m(1)") <= bound
        g, _ = ctx.adjoint_solve()
        assert close(g.reshape(-1).double().cpu().numpy()[qi], z["grad"], f"{tag} gradient") <= bound
        h = ctx.hess_matvec(_t(dv))
        assert close(h.reshape(-1).double().cpu().numpy()[qi], z["hess"], f"{tag} Hessian matvec") <= bound
        ctx.close()


def test_batched_real_sizes_equal_individual_solves():
    """One batched split-bf16 solve over the four real-size subjects equals their single solves."""
    probs, I0s, I1s, v0s = [], [], [], []
    for i in G.C4_SUBJECTS:
        N, K, I0, I1, vseed, _, _, _ = G.case(f"c4_{i}")
        probs.append(L.Problem(N, K, nt=G.NT, variant=L.DEFORMATION_STATE, precision=L.BF16_DFT))
        I0s.append(_t(I0))
        I1s.append(_t(I1))
        v0s.append(_t(0.5 * G.scaled_velocity(N, K, vseed)))
    vs = [v.clone() for v in v0s]
    print("[c4] batched solve over 4 subjects", flush=True)
    st, reps = L.gn_solve_batched(probs, I0s, I1s, vs, max_gn=1, max_pcg=2, fixed_iters=True)
    for i, p in enumerate(probs):
        ctx = L.Context(p)
        ctx.set_images(I0s[i], I1s[i])
        v = v0s[i].clone()
        st1, rep = ctx.gn_solve(v, max_gn=1, max_pcg=2, fixed_iters=True)
        assert reps[i]["decisions"] == rep["decisions"]
        assert close(vs[i], v, f"batched vs single, subject {G.C4_SUBJECTS[i]}") <= 1e-6
        assert abs(reps[i]["E"] - rep["E"]) <= 1e-6 * abs(rep["E"])
        assert reps[i]["det_min"] > 0
        ctx.close()
