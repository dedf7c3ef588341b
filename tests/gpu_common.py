"""Shared set-up of the GPU parity tests: seeded inputs fed to both the HIP library and the oracle."""
import numpy as np
import torch

from oracle import spectral as sp
from oracle.problem import Problem as OProblem
from oracle.variant1 import Variant1
from oracle.variant2 import Variant2
from oracle.variant3 import Variant3
from paper_2006_06823_amd import synthetic as syn


def rel_l2(a, b):
    a = torch.as_tensor(a).double().cpu().reshape(-1)
    b = torch.as_tensor(b).double().cpu().reshape(-1)
    return float((a - b).norm() / b.norm().clamp_min(1e-300))


def max_rel(a, b):
    """Element-wise bound: max |a - b| / max |b|."""
    a = torch.as_tensor(a).double().cpu().reshape(-1)
    b = torch.as_tensor(b).double().cpu().reshape(-1)
    return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))


ELEM_FACTOR = 10.0


def close(a, b, label=""):
    """Error measure every parity assertion uses: the larger of the rel-L2 error and the element-wise
    max |a - b| / max |b| divided by ELEM_FACTOR, so that `close(a, b) <= tol` asserts both
    rel-L2 <= tol and max-element error <= 10 tol.  The factor: a field's largest rounding errors
    sit where its largest coefficients are amplified (the periodic cubic B-spline prefilter has gain up
    to 3 per axis, a 64-tap sum per interpolation, Nt steps), so the element-wise error relative to the
    field's maximum runs a few times above its rel-L2 error even when every element is right; a wrong
    tile, slab or tail shows up as an element-wise error of the size of the field itself, far above
    10 tol.  Both figures are printed, so a run states the measured errors."""
    r, m = rel_l2(a, b), max_rel(a, b)
    print(f"[parity] {label} rel_l2 {r:.3e} max_rel {m:.3e}", flush=True)
    return max(r, m / ELEM_FACTOR)


def images(N, seed):
    """Source/target pair: 2D Gaussian blobs or 3D brain-like phantom (float64 arrays)."""
    if len(N) == 2:
        if N[0] == N[1]:
            I0, I1 = syn.blob_pair_2d(N[0], seed, max_disp_vox=N[0] / 16)
        else:
            n = max(N)
            I0, I1 = syn.blob_pair_2d(n, seed, max_disp_vox=n / 16)
            I0, I1 = I0[:N[0], :N[1]], I1[:N[0], :N[1]]
        return np.ascontiguousarray(I0), np.ascontiguousarray(I1)
    I0, I1 = syn.phantom_pair_3d(tuple(N), seed, max_disp_vox=min(N) / 16)
    return I0.astype(np.float64), I1.astype(np.float64)


def velocity(N, K, Nt, seed, cfl_vox=0.8):
    """Random BL velocity scaled so that max_x |v_j| dt N_j = cfl_vox voxels per step (oracle iota)."""
    d = len(N)
    v = torch.tensor(syn.random_bl_coefficients(d, K, seed))
    vg = sp.include(v, N)
    scale = torch.tensor([float(n) for n in N], dtype=torch.float64).reshape((-1,) + (1,) * d)
    vmax = float((vg * scale).abs().max()) / Nt
    return (v * (cfl_vox / vmax)).numpy()


def oracle_model(variant, N, K, Nt, I0, I1):
    prob = OProblem(tuple(N), tuple(K), Nt=Nt)
    return {1: Variant1, 2: Variant2, 3: Variant3}[variant](prob, I0, I1)
