"""Host checks of the synthetic-input module (no GPU, no solver)."""

import numpy as np
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
