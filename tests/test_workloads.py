"""Host checks of the synthetic-input module (no GPU, no solver)."""

import numpy as np
import pytest
from scipy import ndimage

from paper_1210_2687_amd import workloads as WL


def test_edge_taper_keeps_the_centre_and_blurs_the_edges():
    g = WL.rng(5)
    y = g.uniform(size=(60, 72))
    h = WL.kernel_uniform(9)
    t = WL.edge_taper(y, h)
    blurred = ndimage.convolve(y, h, mode="wrap")
    # weight 1 at distance >= k from both edges of an axis (zero autocorrelation there)
    assert np.array_equal(t[9:-9, 9:-9], y[9:-9, 9:-9])
    # weight 0 on the outermost rows and columns (autocorrelation at lag 0)
    assert np.allclose(t[0, :], blurred[0, :]) and np.allclose(t[:, -1], blurred[:, -1])
    # in between, a convex combination
    lo, hi = np.minimum(y, blurred), np.maximum(y, blurred)
    assert np.all(t >= lo - 1e-12) and np.all(t <= hi + 1e-12)


def test_boundary_pair_shapes_and_valid_region():
    md, bc, et, x_obs, y_obs = WL.boundary_pair(0, observed=96, k=25)
    assert md.shape == (120, 120) and bc.shape == et.shape == x_obs.shape == y_obs.shape == (96, 96)
    assert WL.is_smooth7(120) and WL.is_smooth7(96)
    assert md.mask[12:108, 12:108].all() and md.mask.sum() == 96 * 96
    assert np.array_equal(md.y[12:108, 12:108], bc.y)
    # the valid region of the observation involves no wrap-around: it equals the
    # blur of the true image computed without periodic extension (up to noise)
    full = ndimage.convolve(md.x_true, md.kernel, mode="constant")[12:108, 12:108]
    assert np.max(np.abs(full - y_obs)) < 6e-3


@pytest.mark.parametrize("H,W,k", [(64, 64, 19), (33, 70, 31), (32, 32, 31), (9, 12, 9), (96, 160, 7)])
def test_observation_blur_is_the_periodic_convolution(H, W, k):
    # the generator's spectral blur against scipy's direct periodic convolution
    # (the same definition as the model's A), asymmetric kernels included
    from scipy import ndimage
    g = np.random.default_rng(H * W + k)
    x = g.uniform(size=(H, W))
    h = np.abs(g.standard_normal((k, k)))
    ref = ndimage.convolve(x, h, mode="wrap")
    assert np.max(np.abs(WL._blur_periodic(x, h) - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("H,W,sigma", [(64, 64, 16.0), (8, 8, 32.0), (33, 70, 5.0)])
def test_random_field_smoothing_is_the_periodic_gaussian_filter(H, W, sigma):
    from scipy import ndimage
    n = np.random.default_rng(int(sigma)).standard_normal((H, W))
    ref = ndimage.gaussian_filter(n, sigma, mode="wrap")
    assert np.max(np.abs(WL._smooth_periodic(n, sigma) - ref)) <= 1e-13 * np.max(np.abs(ref))
