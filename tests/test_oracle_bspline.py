"""Pins of the oracle's cubic B-spline interpolator against SciPy and closed forms."""
import numpy as np
import pytest
import scipy.ndimage as ndi
import torch
from scipy.interpolate import BSpline

from oracle import bspline, spectral as sp
from paper_2006_06823_amd import synthetic as syn


@pytest.mark.parametrize("shape", [(12, 14), (7, 9, 6)])
def test_evaluate_matches_scipy_map_coordinates(shape):
    """P5: prefilter + evaluation equal scipy's order-3 'grid-wrap' interpolation."""
    rng = np.random.default_rng(0)
    g = rng.standard_normal(shape)
    pts = rng.uniform(-3.0, 2 * max(shape), (len(shape), 200))
    ref = ndi.map_coordinates(g, pts, order=3, mode="grid-wrap")
    got = bspline.evaluate(bspline.prefilter(torch.tensor(g), len(shape)), torch.tensor(pts)).numpy()
    assert np.abs(got - ref).max() < 1e-12


@pytest.mark.parametrize("shape", [(16, 10), (6, 8, 10)])
def test_prefilter_matches_scipy_spline_filter(shape):
    """P6: FFT-division prefilter equals scipy's recursive spline_filter with periodic wrap."""
    g = np.random.default_rng(1).standard_normal(shape)
    ref = ndi.spline_filter(g, order=3, mode="grid-wrap")
    assert np.abs(bspline.prefilter(torch.tensor(g), len(shape)).numpy() - ref).max() < 1e-12


def test_nodes_and_constants_reproduced():
    """P5: the interpolant passes through the samples and reproduces constants exactly."""
    g = torch.tensor(np.random.default_rng(2).standard_normal((9, 11)))
    nodes = bspline.grid_index((9, 11))
    assert float((bspline.interp_samples(g, torch.zeros(2, 9, 11), 2) - g).abs().max()) < 1e-13
    const = torch.full((9, 11), 0.37, dtype=torch.float64)
    pts = nodes + torch.tensor(np.random.default_rng(3).uniform(-5, 5, (2, 9, 11)))
    assert float((bspline.evaluate(bspline.prefilter(const, 2), pts) - 0.37).abs().max()) < 1e-14


def _cubic_bspline_scipy():
    return BSpline.basis_element([-2.0, -1.0, 0.0, 1.0, 2.0], extrapolate=False)


def single_mode_gain(omega, shift):
    """Closed-form response of the interpolant of exp(i omega n) evaluated at n - shift.

    G = sum_l exp(i omega l) beta3(shift + l) / B^(omega), B^ = (2 + cos omega)/3,
    with beta3 evaluated by SciPy's B-spline basis (independent of the oracle).
    """
    b = _cubic_bspline_scipy()
    tot = 0.0 + 0.0j
    for l in range(-4, 5):
        x = shift + l
        if -2.0 < x < 2.0:
            tot += np.exp(1j * omega * l) * float(b(x))
    return tot / ((2.0 + np.cos(omega)) / 3.0)


def test_single_mode_shift_gain():
    """P5: a single Fourier mode shifted by a fractional amount has the closed-form gain."""
    n = 32
    for k, shift in [(1, 0.3), (5, 0.75), (11, -0.4)]:
        om = 2 * np.pi * k / n
        i = np.arange(n)
        f = np.cos(om * i)
        got = bspline.interp_samples(torch.tensor(f), torch.full((1, n), -shift, dtype=torch.float64), 1).numpy()
        G = single_mode_gain(om, shift)
        expect = np.real(G * np.exp(1j * om * i))
        assert np.abs(got - expect).max() < 1e-13


def test_gradient_matches_finite_difference():
    """P5: the analytic spline gradient equals a central difference of the interpolant."""
    rng = np.random.default_rng(4)
    coef = torch.tensor(rng.standard_normal((8, 9, 7)))
    pts = torch.tensor(rng.uniform(0, 9, (3, 50)))
    _, gr = bspline.evaluate(coef, pts, grad=True)
    h = 1e-6
    for j in range(3):
        e = torch.zeros(3, 1, dtype=torch.float64)
        e[j] = h
        fd = (bspline.evaluate(coef, pts + e) - bspline.evaluate(coef, pts - e)) / (2 * h)
        assert float((fd - gr[j]).abs().max()) < 1e-7


def test_bl_prefilter_equals_spectral_scaling():
    """P6: for a band-limited field the prefilter is the diagonal scale prod_j 3/(2+cos(2 pi k_j/N_j))."""
    N, K = (20, 16), (8, 6)
    c = syn.random_bl_coefficients(1, K, 5)[0]
    ch = sp.to_complex(torch.tensor(c), 2)
    scale = torch.ones(ch.shape, dtype=torch.float64)
    for j in range(2):
        kk = sp.freqs(K[j])
        s = 3.0 / (2.0 + torch.cos(2 * np.pi * kk / N[j]))
        shp = [1, 1]
        shp[j] = -1
        scale = scale * s.reshape(shp)
    folded = sp.include(sp.from_complex(ch * scale, K), N)
    ref = ndi.spline_filter(sp.include(c, N).numpy(), order=3, mode="grid-wrap")
    assert np.abs(folded.numpy() - ref).max() < 1e-12
