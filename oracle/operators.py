"""Linear operators of the deconvolution model, written out from their definitions.

Test infrastructure only (see ``oracle/__init__``). Every function here is
float64 and deliberately naive:

* ``conv_A`` / ``conv_At``: the blur A as periodic convolution on the unknown
  (padded) domain and its adjoint, as explicit sums over kernel taps. The
  paper lets A carry any boundary condition because the mask M discards every
  output pixel that depends on it; periodic is chosen for convenience
  (Sec. IV-A, eq. (34)). Kernel of odd size k = 2l+1, centred at (l, l).
* ``diff_h`` / ``diff_v`` and adjoints: the horizontal / vertical first
  differences with periodic boundary that make up D_i in the TV term
  (Sec. III-C, eq. (26)); forward differences (reading: the paper names the
  differences but not their direction).
* ``dft2`` / ``idft2``: the unitary-up-to-scale 2-D DFT U as products with
  dense DFT matrices (Sec. III-A, eq. (19)); O(n (H+W)), no FFT.
* ``kernel_spectrum`` / ``diff_spectra``: the diagonals Lambda, Delta^h,
  Delta^v of eq. (32), obtained by applying ``dft2`` to the impulse responses
  of A, D^h and D^v.
* ``haar_analysis`` / ``haar_synthesis``: the undecimated ("redundant") Haar
  Parseval frame P and its adjoint P^T used for frame-analysis
  regularisation (Sec. III-B, eq. (21); Sec. V uses a redundant Haar frame).

Parity pins: tests/test_oracle_operators.py (adjoint identities, A 1 = (sum h) 1,
agreement with scipy.signal.convolve2d(boundary='wrap'), naive DFT against
numpy.fft.fft2, P^T P = I and energy preservation, a hand-indexed 1-level Haar
example, dense 8x8 matrix checks).
"""

import numpy as np

__all__ = [
    "conv_A", "conv_At", "diff_h", "diff_v", "diff_ht", "diff_vt",
    "dft_matrix", "dft2", "idft2", "kernel_spectrum", "diff_spectra",
    "haar_analysis", "haar_synthesis", "haar_num_bands",
]


def _check_kernel(h):
    h = np.asarray(h, dtype=np.float64)
    if h.ndim != 2 or h.shape[0] != h.shape[1] or h.shape[0] % 2 != 1:
        raise ValueError("kernel must be square with odd side")
    return h


def conv_A(x, h):
    """(A x)[r, c] = sum_{a,b=-l..l} h[a+l, b+l] * x[(r-a) mod H, (c-b) mod W].

    Periodic convolution of the unknown image x (H x W) with the k x k kernel h
    (k = 2l+1). This is A of eq. (34) with the periodic boundary the paper
    adopts for convenience (Sec. IV-A).
    """
    x = np.asarray(x, dtype=np.float64)
    h = _check_kernel(h)
    l = h.shape[0] // 2
    out = np.zeros_like(x)
    for a in range(-l, l + 1):
        for b in range(-l, l + 1):
            w = h[a + l, b + l]
            if w != 0.0:
                # np.roll(x, (a, b))[r, c] = x[r - a, c - b]
                out += w * np.roll(x, (a, b), axis=(0, 1))
    return out


def conv_At(z, h):
    """(A^T z)[r, c] = sum_{a,b} h[a+l, b+l] * z[(r+a) mod H, (c+b) mod W]."""
    z = np.asarray(z, dtype=np.float64)
    h = _check_kernel(h)
    l = h.shape[0] // 2
    out = np.zeros_like(z)
    for a in range(-l, l + 1):
        for b in range(-l, l + 1):
            w = h[a + l, b + l]
            if w != 0.0:
                out += w * np.roll(z, (-a, -b), axis=(0, 1))
    return out


def diff_h(x):
    """(D^h x)[r, c] = x[r, (c+1) mod W] - x[r, c]  (horizontal difference)."""
    x = np.asarray(x, dtype=np.float64)
    return np.roll(x, -1, axis=1) - x


def diff_v(x):
    """(D^v x)[r, c] = x[(r+1) mod H, c] - x[r, c]  (vertical difference)."""
    x = np.asarray(x, dtype=np.float64)
    return np.roll(x, -1, axis=0) - x


def diff_ht(p):
    """((D^h)^T p)[r, c] = p[r, (c-1) mod W] - p[r, c]."""
    p = np.asarray(p, dtype=np.float64)
    return np.roll(p, 1, axis=1) - p


def diff_vt(p):
    """((D^v)^T p)[r, c] = p[(r-1) mod H, c] - p[r, c]."""
    p = np.asarray(p, dtype=np.float64)
    return np.roll(p, 1, axis=0) - p


def dft_matrix(N):
    """Dense DFT matrix F[j, k] = exp(-2 pi i (j k mod N) / N), float64/complex128.

    The product j*k is reduced modulo N in exact integer arithmetic before the
    angle is formed, so every entry is a correctly rounded N-th root of unity.
    """
    j = np.arange(N, dtype=np.int64)
    jk = np.mod(np.outer(j, j), N)
    ang = (-2.0 * np.pi / N) * jk.astype(np.float64)
    return np.cos(ang) + 1j * np.sin(ang)


_DFT_CACHE = {}


def _F(N):
    F = _DFT_CACHE.get(N)
    if F is None:
        F = dft_matrix(N)
        _DFT_CACHE[N] = F
    return F


def dft2(x):
    """X[k1, k2] = sum_{r,c} x[r, c] exp(-2 pi i (k1 r / H + k2 c / W)).

    Naive separable DFT as dense matrix products, F_H x F_W (F is symmetric).
    This is (up to the scale sqrt(HW)) the operator U of eq. (19).
    """
    x = np.asarray(x)
    H, W = x.shape
    return _F(H) @ x.astype(np.complex128) @ _F(W)


def idft2(X):
    """Inverse of ``dft2``: x = conj(F_H) X conj(F_W) / (H W)."""
    X = np.asarray(X, dtype=np.complex128)
    H, W = X.shape
    return (np.conj(_F(H)) @ X @ np.conj(_F(W))) / (H * W)


def kernel_spectrum(h, H, W):
    """Diagonal Lambda of A = U^* Lambda U (eq. (19)): the DFT of A's impulse response.

    The impulse response of ``conv_A`` on an H x W grid is the kernel placed
    with its centre at pixel (0, 0) and wrapped periodically.
    """
    delta = np.zeros((H, W))
    delta[0, 0] = 1.0
    return dft2(conv_A(delta, h))


def diff_spectra(H, W):
    """Diagonals Delta^h, Delta^v of eq. (32): DFTs of the impulse responses of D^h, D^v."""
    delta = np.zeros((H, W))
    delta[0, 0] = 1.0
    return dft2(diff_h(delta)), dft2(diff_v(delta))


# ---------------------------------------------------------------------------
# Undecimated Haar Parseval frame (analysis operator P, adjoint P^T).
#
# Level j = 1..J uses dilation s = 2^(j-1) and the periodic 1-D filters
#   low:  (L x)[i] = (x[i] + x[i+s]) / 2,   high: (Hi x)[i] = (x[i] - x[i+s]) / 2,
# whose squared transfer functions add to one, so every level (and by
# recursion on the low-low band the whole multi-level frame) satisfies
# P^T P = I, the Parseval property the z-step relies on (Sec. III-B).
# Band order (reading; the paper does not fix one): for j = 1..J the three
# detail bands [L_v Hi_h, Hi_v L_h, Hi_v Hi_h] of level j, then the final
# low-low band L_v L_h of level J: 3J + 1 bands of H x W each.
# ---------------------------------------------------------------------------

def haar_num_bands(J):
    return 3 * J + 1


def _lo(x, s, axis):
    return 0.5 * (x + np.roll(x, -s, axis=axis))


def _hi(x, s, axis):
    return 0.5 * (x - np.roll(x, -s, axis=axis))


def _lo_t(c, s, axis):
    return 0.5 * (c + np.roll(c, s, axis=axis))


def _hi_t(c, s, axis):
    return 0.5 * (c - np.roll(c, s, axis=axis))


def haar_analysis(x, J):
    """P x: array of shape (3J+1, H, W) in the band order described above."""
    a = np.asarray(x, dtype=np.float64)
    bands = []
    for j in range(1, J + 1):
        s = 2 ** (j - 1)
        lv = _lo(a, s, 0)
        hv = _hi(a, s, 0)
        bands.append(_hi(lv, s, 1))   # low vertical, high horizontal
        bands.append(_lo(hv, s, 1))   # high vertical, low horizontal
        bands.append(_hi(hv, s, 1))   # high vertical, high horizontal
        a = _lo(lv, s, 1)             # low-low, recursed on
    bands.append(a)
    return np.stack(bands)


def haar_synthesis(c, J):
    """P^T c for coefficients c of shape (3J+1, H, W)."""
    c = np.asarray(c, dtype=np.float64)
    if c.shape[0] != 3 * J + 1:
        raise ValueError("expected 3J+1 bands")
    a = c[3 * J]
    for j in range(J, 0, -1):
        s = 2 ** (j - 1)
        b_lh, b_hl, b_hh = c[3 * (j - 1)], c[3 * (j - 1) + 1], c[3 * (j - 1) + 2]
        lv = _lo_t(a, s, 1) + _hi_t(b_lh, s, 1)
        hv = _lo_t(b_hl, s, 1) + _hi_t(b_hh, s, 1)
        a = _lo_t(lv, s, 0) + _hi_t(hv, s, 0)
    return a
