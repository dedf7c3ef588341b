"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random numbers and renders closed-form images; it holds
none of the registration method's arithmetic (no band-limited transforms, no
interpolation, no transport).  Both the HIP library and the CPU oracle receive
the arrays produced here.

Conventions: the image domain is the periodic unit torus [0,1)^d sampled at the
nodes x_j = i_j / N_j (C order, last axis contiguous).  Intensities follow the
paper's convention of images scaled to [0, 1] (Section 4.2, registration
pipeline).  The paper evaluates on brain MRI collections that are not available
here; the phantoms below stand in for them with the same structure (nested
tissue shells with three intensity levels, ventricles, acquisition noise) and
brain-like grid sizes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "grid_coords",
    "smooth_displacement",
    "BlobImage2D",
    "BrainPhantom3D",
    "blob_pair_2d",
    "phantom_pair_3d",
    "random_bl_coefficients",
    "slot_frequency",
]


def grid_coords(shape):
    """Node coordinates of the unit torus, one float64 array per axis."""
    axes = [np.arange(n, dtype=np.float64) / n for n in shape]
    return np.meshgrid(*axes, indexing="ij")


def slot_frequency(K: int) -> np.ndarray:
    """Frequency magnitude held by each real-basis slot of one axis.

    Slot 0 is the constant, slots 2k-1 / 2k hold cos / sin of frequency k, and
    the last slot of an even K is an always-zero pad (returned as -1).
    """
    f = np.zeros(K, dtype=np.int64)
    for a in range(1, K):
        f[a] = (a + 1) // 2
    if K % 2 == 0:
        f[K - 1] = -1
    return f


class SmoothDisplacement:
    """Analytic low-frequency periodic displacement u(x) = sum_m a_m sin(2 pi k_m.x + th_m).

    Values are in unit-torus units.  The target image is rendered as
    I1(x) = I0(x - u(x)), evaluated in closed form (no interpolation).
    """

    def __init__(self, d, modes_per_comp, rng):
        self.d = d
        self.k = []      # per component: [M, d] integer wave vectors
        self.amp = []    # per component: [M]
        self.phase = []  # per component: [M]
        for _ in range(d):
            ks = []
            while len(ks) < modes_per_comp:
                k = rng.integers(-1, 2, size=d)
                if np.any(k != 0):
                    ks.append(k)
            self.k.append(np.array(ks, dtype=np.float64))
            self.amp.append(rng.uniform(0.5, 1.0, size=modes_per_comp))
            self.phase.append(rng.uniform(0.0, 2 * np.pi, size=modes_per_comp))
        self.scale = 1.0

    def __call__(self, X):
        """X: list of d coordinate arrays -> list of d displacement arrays."""
        out = []
        for c in range(self.d):
            u = np.zeros_like(X[0])
            for m in range(len(self.amp[c])):
                arg = sum(2 * np.pi * self.k[c][m, j] * X[j] for j in range(self.d))
                u = u + self.amp[c][m] * np.sin(arg + self.phase[c][m])
            out.append(self.scale * u)
        return out

    def jacobian_det_min(self, X):
        """min over points of det(I - Du), from the closed-form derivative."""
        D = np.zeros((self.d, self.d) + X[0].shape)
        for c in range(self.d):
            for m in range(len(self.amp[c])):
                arg = sum(2 * np.pi * self.k[c][m, j] * X[j] for j in range(self.d))
                cs = np.cos(arg + self.phase[c][m])
                for j in range(self.d):
                    D[c, j] += self.scale * self.amp[c][m] * 2 * np.pi * self.k[c][m, j] * cs
        A = np.moveaxis(np.eye(self.d)[:, :, None] - D.reshape(self.d, self.d, -1), 2, 0)
        return float(np.linalg.det(A).min())


def smooth_displacement(shape, max_disp_vox, seed, modes_per_comp=3):
    """Random analytic displacement scaled so max_x |u(x)| = max_disp_vox voxels.

    The Euclidean length is measured in voxel units (u_j * N_j) on the grid.
    """
    rng = np.random.default_rng(seed)
    d = len(shape)
    disp = SmoothDisplacement(d, modes_per_comp, rng)
    X = grid_coords(shape)
    u = disp(X)
    mag = np.sqrt(sum((u[j] * shape[j]) ** 2 for j in range(d))).max()
    disp.scale = max_disp_vox / mag
    return disp


class BlobImage2D:
    """Sum of anisotropic Gaussian blobs on the unit torus, periodised over the 3x3 nearest images."""

    def __init__(self, rng, n_blobs=6):
        self.a = rng.uniform(0.3, 1.0, size=n_blobs)
        self.mu = rng.uniform(0.2, 0.8, size=(n_blobs, 2))
        sig = rng.uniform(0.03, 0.10, size=(n_blobs, 2))
        ang = rng.uniform(0.0, np.pi, size=n_blobs)
        self.prec = []
        for b in range(n_blobs):
            c, s = np.cos(ang[b]), np.sin(ang[b])
            R = np.array([[c, -s], [s, c]])
            cov = R @ np.diag(sig[b] ** 2) @ R.T
            self.prec.append(np.linalg.inv(cov))
        self.norm = 1.0

    def raw(self, X):
        out = np.zeros_like(X[0])
        for b in range(len(self.a)):
            P = self.prec[b]
            for o1 in (-1, 0, 1):
                for o2 in (-1, 0, 1):
                    d1 = X[0] - self.mu[b, 0] - o1
                    d2 = X[1] - self.mu[b, 1] - o2
                    q = P[0, 0] * d1 * d1 + 2 * P[0, 1] * d1 * d2 + P[1, 1] * d2 * d2
                    out += self.a[b] * np.exp(-0.5 * q)
        return out

    def __call__(self, X):
        return self.raw(X) / self.norm


def _smooth_step(z):
    """0.5 (1 - tanh(z)): 1 inside (z << 0), 0 outside."""
    return 0.5 * (1.0 - np.tanh(z))


class BrainPhantom3D:
    """Nested ellipsoid shells (0.8 core, 0.5, 0.2 outer ring) with two 0.2 ventricles.

    Edges are tanh-smoothed over about one voxel of the grid it is rendered for.
    """

    def __init__(self, rng, edge_vox_shape):
        self.center = 0.5 + rng.uniform(-0.02, 0.02, size=3)
        angles = np.deg2rad(rng.uniform(-10.0, 10.0, size=3))
        self.R = _euler(*angles)
        self.axes = np.array([0.36, 0.42, 0.33]) * (1.0 + rng.uniform(-0.08, 0.08, size=3))
        self.r1 = 0.55 + rng.uniform(-0.05, 0.05)
        self.r2 = 0.80 + rng.uniform(-0.05, 0.05)
        # ventricles: small ellipsoids inside the core, mirrored about the first axis
        off = 0.12 + rng.uniform(-0.02, 0.02)
        self.vent_c = [np.array([-off, 0.05, 0.0]), np.array([off, 0.05, 0.0])]
        self.vent_ax = np.array([0.06, 0.16, 0.08]) * (1.0 + rng.uniform(-0.1, 0.1, size=3))
        self.width = 1.0 / float(np.mean(edge_vox_shape))  # one voxel in unit-torus units

    def __call__(self, X):
        y = [X[j] - self.center[j] for j in range(3)]
        # body frame: q = R^T y
        q = [sum(self.R[i, j] * y[i] for i in range(3)) for j in range(3)]
        r = np.sqrt(sum((q[j] / self.axes[j]) ** 2 for j in range(3)))
        w = self.width / float(np.mean(self.axes))
        img = (0.2 * _smooth_step((r - 1.0) / w)
               + 0.3 * _smooth_step((r - self.r2) / w)
               + 0.3 * _smooth_step((r - self.r1) / w))
        for vc in self.vent_c:
            rv = np.sqrt(sum(((q[j] - vc[j] * self.axes[j]) / (self.vent_ax[j] * self.axes[j])) ** 2
                             for j in range(3)))
            wv = self.width / float(np.mean(self.vent_ax * self.axes))
            img = img - 0.6 * _smooth_step((rv - 1.0) / wv)
        return img


def _euler(a, b, c):
    ca, sa, cb, sb, cc, sc = np.cos(a), np.sin(a), np.cos(b), np.sin(b), np.cos(c), np.sin(c)
    Rx = np.array([[1, 0, 0], [0, ca, -sa], [0, sa, ca]])
    Ry = np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
    Rz = np.array([[cc, -sc, 0], [sc, cc, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def _warped_coords(X, disp):
    if disp is None:
        return X
    u = disp(X)
    return [np.mod(X[j] - u[j], 1.0) for j in range(len(X))]


def blob_pair_2d(n=64, seed=0, max_disp_vox=4.0):
    """Source/target pair for the 2D case: Gaussian-blob source, target warped by a smooth map.

    Returns (I0, I1) as float64 [n][n] arrays with the source normalised to max 1.
    """
    rng = np.random.default_rng(seed)
    img = BlobImage2D(rng)
    X = grid_coords((n, n))
    img.norm = img.raw(X).max()
    disp = smooth_displacement((n, n), max_disp_vox, seed=seed + 7919)
    I0 = img(X)
    I1 = img(_warped_coords(X, disp))
    return I0, I1


def phantom_pair_3d(shape, seed, max_disp_vox=8.0, noise=0.02, template_seed=None):
    """Brain-like phantom pair on a 3D grid.

    I0 is the phantom with iid N(0, noise^2) noise; I1 is the phantom (or, when
    template_seed is given, the template phantom) evaluated at x - u(x) for a
    smooth random displacement of max length max_disp_vox voxels, plus
    independent noise.  Returns float32 arrays [N1][N2][N3].
    """
    rng = np.random.default_rng(seed)
    ph = BrainPhantom3D(rng, shape)
    X = grid_coords(shape)
    src = ph if template_seed is None else BrainPhantom3D(np.random.default_rng(template_seed), shape)
    disp = smooth_displacement(shape, max_disp_vox, seed=seed + 7919)
    I0 = src(X) + noise * rng.standard_normal(shape)
    I1 = ph(_warped_coords(X, disp)) + noise * rng.standard_normal(shape)
    return I0.astype(np.float32), I1.astype(np.float32)


def phantom_with_noise_3d(shape, seed, noise=0.02):
    """The brain-like phantom of phantom_pair_3d, unwarped, and two independent N(0, noise^2) fields: the
    template of a pair whose target is produced elsewhere, and the noise of each image.  Float32 [N1][N2][N3]."""
    rng = np.random.default_rng(seed)
    ph = BrainPhantom3D(rng, shape)
    P = ph(grid_coords(shape))
    n0 = noise * rng.standard_normal(shape)
    n1 = noise * rng.standard_normal(shape)
    return P.astype(np.float32), n0.astype(np.float32), n1.astype(np.float32)


def random_bl_coefficients(ncomp, K, seed, decay=0.1):
    """iid N(0,1) real-basis coefficients [ncomp][K1]..[Kd] with a smooth spectral envelope.

    The envelope 1 / (1 + decay |k|^2) favours low frequencies (|k| is the
    Euclidean norm of the per-axis frequencies held by the slot); the constant
    mode and every pad slot are zero.  Scale to a target velocity magnitude
    after drawing.
    """
    rng = np.random.default_rng(seed)
    K = tuple(int(k) for k in K)
    freqs = [slot_frequency(k) for k in K]
    grids = np.meshgrid(*freqs, indexing="ij")
    pad = np.zeros(K, dtype=bool)
    k2 = np.zeros(K)
    for g in grids:
        pad |= g < 0
        k2 += np.maximum(g, 0) ** 2
    env = 1.0 / (1.0 + decay * k2)
    env[pad] = 0.0
    env[(0,) * len(K)] = 0.0
    c = rng.standard_normal((ncomp,) + K) * env
    return c
