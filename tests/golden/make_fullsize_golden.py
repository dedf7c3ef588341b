"""Write the oracle's values at full benchmark sizes for the GPU parity tests.

Calls only the FP64 oracle (oracle/) and the seeded input generators; nothing here comes from the
HIP path.  At these sizes the oracle needs minutes to tens of minutes per solve on a few host cores,
too slow for a GPU run, so its results are stored: the values at a seeded random sample of band
coefficients and grid nodes (the tests draw the same sample from the same seed).

Cases (deformation-state variant, Section 2.3.3; Nt = 10; velocities scaled to 0.8 voxel per step,
a sub-voxel CFL, so departure points fall between nodes):
  c3          160 x 192 x 160 / band 40 x 48 x 40, phantom pair seed 2 (8-voxel displacement),
              velocity seed 5, Hessian direction seed 3; stores u~_n at n = 1, 5, 10, m(1), the
              gradient, the Hessian matvec, det(I - D iota(u~(1))) and its extrema (16384 samples).
  c4_<i>      batched subject i of the uneven-grid batch (N_i in {96, ..., 192}, band
              K_i = clamp(8 ceil(N_i / 32), 32, 48), subject pair seed 1000 + i against the template
              phantom seed 999): velocity seed 2000 + i, direction seed 3000 + i; stores u~(1), m(1),
              the gradient and the Hessian matvec (8192 samples).  Subjects 7, 5, 4, 1 have
              N = 96, 144, 176, 192.
Usage: python tests/golden/make_fullsize_golden.py c3 c4_7 c4_5 c4_4 c4_1
"""
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import spectral as sp  # noqa: E402
from oracle.gauss_newton import jacobian_det  # noqa: E402
from oracle.problem import Problem  # noqa: E402
from oracle.variant3 import Variant3  # noqa: E402
from paper_2006_06823_amd import synthetic as syn  # noqa: E402

NT = 10
SAMPLE_SEED = 77
C4_SUBJECTS = (7, 5, 4, 1)


def batched_subject_size(i):
    """Grid and band of batched subject i (the uneven-grid batch's recipe)."""
    n = 96 + 16 * int(np.random.default_rng(1000 + i).integers(0, 7))
    k = min(48, max(32, 8 * -(-n // 32)))
    return (n, n, n), (k, k, k)


def case(name):
    """(N, K, I0, I1, velocity seed, direction seed, samples, with the c3 extras)."""
    if name == "c3":
        N, K = (160, 192, 160), (40, 48, 40)
        I0, I1 = syn.phantom_pair_3d(N, seed=2, max_disp_vox=8.0)
        return N, K, I0, I1, 5, 3, 16384, True
    i = int(name.split("_")[1])
    N, K = batched_subject_size(i)
    I0, I1 = syn.phantom_pair_3d(N, 1000 + i, max_disp_vox=8.0, template_seed=999)
    return N, K, I0, I1, 2000 + i, 3000 + i, 8192, False


def golden_path(name):
    if name == "c3":
        return os.path.join(HERE, "c3_deformation_state_160x192x160.npz")
    N, _ = batched_subject_size(int(name.split("_")[1]))
    return os.path.join(HERE, f"c4_subject{name.split('_')[1]}_{N[0]}.npz")


def scaled_velocity(N, K, seed, cfl_vox=0.8):
    """Band coefficients scaled so that max_x |v_j| dt N_j = cfl_vox voxels per step."""
    v = torch.tensor(syn.random_bl_coefficients(3, K, seed))
    vg = sp.include(v, N)
    scale = torch.tensor([float(n) for n in N], dtype=torch.float64).reshape(3, 1, 1, 1)
    vmax = float((vg * scale).abs().max()) / NT
    return (v * (cfl_vox / vmax)).numpy()


def sample_indices(N, K, nsamp):
    """Seeded sample of flat indices into a BL vector [3][K] and a grid scalar [N]."""
    rng = np.random.default_rng(SAMPLE_SEED)
    q = 3 * int(np.prod(K))
    p = int(np.prod(N))
    return np.sort(rng.choice(q, nsamp, replace=False)), np.sort(rng.choice(p, nsamp, replace=False))


def main(name):
    t0 = time.time()
    log = lambda s: print(f"[{name} {time.time() - t0:7.1f} s] {s}", flush=True)
    N, K, I0, I1, vseed, dseed, nsamp, extras = case(name)
    v = scaled_velocity(N, K, vseed)
    dv = syn.random_bl_coefficients(3, K, dseed)
    om = Variant3(Problem(N, K, Nt=NT), I0.astype(np.float64), I1.astype(np.float64))
    om.setup(v)
    log("set-up done")
    om.state()
    E = [float(x) for x in om.objective()]
    log("state done")
    qi, pi = sample_indices(N, K, nsamp)
    res = dict(N=np.array(N), K=np.array(K), Nt=np.array(NT), seeds=np.array([vseed, dseed, SAMPLE_SEED]),
               E=np.array(E), m1=om.m1.reshape(-1).numpy()[pi])
    if extras:
        det = jacobian_det(om.p, om.u[-1]).reshape(-1)
        res["det_minmax"] = np.array([float(det.min()), float(det.max())])
        res["det"] = det.numpy()[pi]
        for n in (1, 5):
            res[f"u{n}"] = om.u[n].reshape(-1).numpy()[qi]
        log("Jacobian done")
    res[f"u{NT}"] = om.u[NT].reshape(-1).numpy()[qi]
    om.adjoint()
    g = om.gradient()
    log("adjoint done")
    h = om.hess_matvec(dv)
    log("matvec done")
    res.update(grad=g.reshape(-1).numpy()[qi], hess=h.reshape(-1).numpy()[qi],
               norms=np.array([float(g.norm()), float(h.norm())]))
    out = golden_path(name)
    np.savez_compressed(out, **res)
    log(f"wrote {out}")


if __name__ == "__main__":
    for nm in (sys.argv[1:] or ["c3"] + [f"c4_{i}" for i in C4_SUBJECTS]):
        main(nm)
