"""Pins for oracle/operators.py against definitions, library routines and invariants."""

import numpy as np
import pytest
from scipy import signal

import oracle as O


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv_matches_scipy_wrap_convolution():
    # scipy's full-then-'same' convolution with periodic boundary is the textbook
    # definition; an asymmetric kernel pins origin and flip.
    x = _rand((16, 20), 1)
    h = np.abs(_rand((5, 5), 2))
    ref = signal.convolve2d(x, h, mode="same", boundary="wrap")
    np.testing.assert_allclose(O.conv_A(x, h), ref, rtol=0, atol=1e-12)


def test_conv_adjoint_identity():
    x, z = _rand((12, 18), 3), _rand((12, 18), 4)
    h = _rand((7, 7), 5)
    lhs = np.sum(O.conv_A(x, h) * z)
    rhs = np.sum(x * O.conv_At(z, h))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0)


def test_conv_of_constant_is_dc_gain():
    h = np.abs(_rand((9, 9), 6))
    out = O.conv_A(np.ones((10, 14)), h)
    np.testing.assert_allclose(out, h.sum(), rtol=1e-14)


def test_differences_brute_force_and_adjoint():
    x = _rand((5, 7), 7)
    H, W = x.shape
    dh = np.array([[x[r, (c + 1) % W] - x[r, c] for c in range(W)] for r in range(H)])
    dv = np.array([[x[(r + 1) % H, c] - x[r, c] for c in range(W)] for r in range(H)])
    np.testing.assert_array_equal(O.diff_h(x), dh)
    np.testing.assert_array_equal(O.diff_v(x), dv)
    p = _rand((5, 7), 8)
    assert abs(np.sum(O.diff_h(x) * p) - np.sum(x * O.diff_ht(p))) < 1e-13
    assert abs(np.sum(O.diff_v(x) * p) - np.sum(x * O.diff_vt(p))) < 1e-13


def test_naive_dft_matches_numpy_fft():
    x = _rand((12, 10), 9) + 1j * _rand((12, 10), 10)
    np.testing.assert_allclose(O.dft2(x), np.fft.fft2(x), rtol=0, atol=1e-11)
    np.testing.assert_allclose(O.idft2(O.dft2(x)), x, rtol=0, atol=1e-13)


@pytest.mark.parametrize("shape,k", [((16, 16), 5), ((15, 21), 7), ((8, 8), 3)])
def test_fft_diagonalises_convolution(shape, k):
    # A = U^* Lambda U  (eq. (19)): IDFT(Lambda DFT(x)) equals the direct periodic sum
    x = _rand(shape, 11)
    h = _rand((k, k), 12)
    Lam = O.kernel_spectrum(h, *shape)
    via_dft = np.real(O.idft2(Lam * O.dft2(x)))
    np.testing.assert_allclose(via_dft, O.conv_A(x, h), rtol=0, atol=1e-12)
    # and the adjoint is conj(Lambda)
    via_dft_t = np.real(O.idft2(np.conj(Lam) * O.dft2(x)))
    np.testing.assert_allclose(via_dft_t, O.conv_At(x, h), rtol=0, atol=1e-12)


def test_difference_spectra_closed_form():
    H, W = 12, 10
    Dh, Dv = O.diff_spectra(H, W)
    k1 = np.arange(H)[:, None]
    k2 = np.arange(W)[None, :]
    np.testing.assert_allclose(np.abs(Dh) ** 2, np.broadcast_to(2 - 2 * np.cos(2 * np.pi * k2 / W), (H, W)), atol=1e-13)
    np.testing.assert_allclose(np.abs(Dv) ** 2, np.broadcast_to(2 - 2 * np.cos(2 * np.pi * k1 / H), (H, W)), atol=1e-13)


@pytest.mark.parametrize("J", [1, 2, 3])
def test_haar_parseval_and_adjoint(J):
    x = _rand((16, 24), 13)
    c = O.haar_analysis(x, J)
    assert c.shape == (3 * J + 1, 16, 24)
    np.testing.assert_allclose(O.haar_synthesis(c, J), x, atol=1e-13)      # P^T P = I
    assert abs(np.sum(c * c) - np.sum(x * x)) < 1e-11                      # energy
    cc = _rand(c.shape, 14)
    assert abs(np.sum(c * cc) - np.sum(x * O.haar_synthesis(cc, J))) < 1e-11


def test_haar_one_level_hand_indexed():
    # Level 1 (dilation 1) written out index by index.
    x = _rand((4, 6), 15)
    H, W = x.shape
    c = O.haar_analysis(x, 1)
    for r in range(H):
        for col in range(W):
            a = x[r, col]
            b = x[r, (col + 1) % W]
            cdn = x[(r + 1) % H, col]
            d = x[(r + 1) % H, (col + 1) % W]
            lh = ((a - b) + (cdn - d)) / 4.0   # low vertical, high horizontal
            hl = ((a + b) - (cdn + d)) / 4.0   # high vertical, low horizontal
            hh = ((a - b) - (cdn - d)) / 4.0
            ll = (a + b + cdn + d) / 4.0
            np.testing.assert_allclose(c[:, r, col], [lh, hl, hh, ll], atol=1e-15)


def test_haar_second_level_uses_dilation_two():
    # Rows constant, columns periodic [1, 1, -1, -1]: the level-1 low-low band is
    # a = [1, 0, -1, 0, ...] and the level-2 (dilation 2) low-vertical /
    # high-horizontal band is (a[c] - a[c+2]) / 2 = [1, 0, -1, 0, ...]
    # (a dilation of 1 would give [.5, .5, -.5, -.5, ...]).
    x = np.tile(np.array([1.0, 1.0, -1.0, -1.0] * 2), (8, 1))
    c = O.haar_analysis(x, 2)
    expect = np.tile(np.array([1.0, 0.0, -1.0, 0.0] * 2), (8, 1))
    np.testing.assert_allclose(c[3], expect, atol=1e-15)
