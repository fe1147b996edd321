"""Seeded synthetic deconvolution problems (inputs only, no solver arithmetic).

Both the HIP path and the oracle are fed from here; this module computes no
step of the ADMM method. It draws a piecewise-constant / piecewise-smooth
image x, a blur kernel h, an observation mask m and produces the observation
y = m * (h (*) x + n), where the blur of the *full* image (periodic boundary,
via ``scipy.ndimage.convolve``) followed by the mask is how the paper builds
its unknown-boundary data (Sec. V: blur the whole image, keep the valid
region). The paper's benchmark photographs are not available; these images
stand in for them at the paper's shapes and at the shapes of the workloads
below.

Recipe (all draws from ``numpy.random.Generator(PCG64(seed))``):

* image: background U[0,1]; Poisson(8 n / 128^2) shapes (cap 400), each an
  axis-aligned rectangle (sides U[0.05,0.4] min(H,W)) or a rotated ellipse
  (semi-axes U[0.03,0.25] min(H,W)), intensity U[0,1], painted in order;
  optional Gaussian random field (white noise smoothed by a periodic Gaussian
  of std ``grf_scale`` px truncated at 4 std, zero mean, unit std, times 0.2)
  added, then clipped to [0,1];
* kernels: uniform 1/k^2; Gaussian exp(-(a^2+b^2)/(2 s^2)); linear motion (a
  centred segment of length L at angle theta, 64 samples splatted bilinearly);
  disk (pixel coverage of a radius-r disk by 16x16 supersampling); all
  normalised to unit sum;
* masks: the valid region (rows and columns l .. side-1-l for a (2l+1)^2
  kernel, Sec. IV-A), optionally minus i.i.d. missing interior pixels or minus
  randomly chosen 8x8 blocks on an 8-aligned grid;
* noise: N(0, sigma^2) on the observed pixels; unobserved entries of y are 0.
"""

from dataclasses import dataclass, field
import math

import numpy as np
from scipy import ndimage

__all__ = [
    "Problem", "rng", "synth_image", "kernel_uniform", "kernel_gaussian",
    "kernel_motion", "kernel_disk", "valid_mask", "observe", "next_smooth7",
    "is_smooth7", "config1", "config2", "config3", "config4", "config5_problem", "comparison_problem",
    "COMPARISON_BLURS",
]


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Problem:
    """One deconvolution problem: y = m * (h (*) x_true + n) on an H x W unknown domain."""
    y: np.ndarray          # float64 H x W, zero where m == 0
    mask: np.ndarray       # uint8 H x W, 1 = observed
    kernel: np.ndarray     # float64 k x k, odd k, unit sum
    lam: float
    mu1: float
    mu2: float
    x_true: np.ndarray = field(repr=False, default=None)
    reg: str = "tv"        # "tv", "frame" (analysis, FA) or "synthesis" (FS)
    levels: int = 0        # frame levels J for reg == "frame"

    @property
    def shape(self):
        return self.y.shape


def _gauss_taps(sigma):
    """Sampled Gaussian of std sigma truncated at 4 sigma, unit sum (taps -r..r)."""
    r = int(4.0 * sigma + 0.5)
    t = np.exp(-0.5 * (np.arange(-r, r + 1, dtype=np.float64) / sigma) ** 2)
    return t / t.sum(), r


def _smooth_periodic(noise, sigma):
    """Separable periodic Gaussian smoothing (the same truncated kernel on each
    axis, wrapped onto the grid), applied as a product of transfer functions."""
    H, W = noise.shape
    taps, r = _gauss_taps(sigma)

    def transfer(n, half):
        k = np.zeros(n)
        np.add.at(k, np.arange(-r, r + 1) % n, taps)
        return np.fft.rfft(k) if half else np.fft.fft(k)

    spec = np.fft.rfft2(noise) * (transfer(H, False)[:, None] * transfer(W, True)[None, :])
    return np.fft.irfft2(spec, s=(H, W))


def synth_image(g, H, W, grf_scale=None):
    """Piecewise-constant rectangles/ellipses on a uniform background, optional GRF."""
    x = np.full((H, W), g.uniform())
    n = H * W
    nshape = min(400, int(g.poisson(8.0 * n / 128.0 ** 2)))
    s = float(min(H, W))

    def box(lo, hi, n):
        # integer pixel range [i0, i1) that contains every pixel i with lo <= i <= hi
        return max(0, int(math.floor(lo))), min(n, int(math.floor(hi)) + 1)

    for _ in range(nshape):
        val = g.uniform()
        if g.uniform() < 0.5:
            hh, ww = g.uniform(0.05, 0.4, size=2) * s
            r0 = g.uniform(0, H)
            c0 = g.uniform(0, W)
            i0, i1 = box(r0, r0 + hh, H)
            j0, j1 = box(c0, c0 + ww, W)
            rr, cc = np.mgrid[i0:i1, j0:j1]
            sel = (rr >= r0) & (rr < r0 + hh) & (cc >= c0) & (cc < c0 + ww)
        else:
            a, b = g.uniform(0.03, 0.25, size=2) * s
            r0 = g.uniform(0, H)
            c0 = g.uniform(0, W)
            th = g.uniform(0, math.pi)
            R = max(a, b)          # the ellipse lies inside this circle about its centre
            i0, i1 = box(r0 - R, r0 + R, H)
            j0, j1 = box(c0 - R, c0 + R, W)
            rr, cc = np.mgrid[i0:i1, j0:j1]
            dr, dc = rr - r0, cc - c0
            u = dc * math.cos(th) + dr * math.sin(th)
            v = -dc * math.sin(th) + dr * math.cos(th)
            sel = (u / a) ** 2 + (v / b) ** 2 <= 1.0
        if sel.size:
            x[i0:i1, j0:j1][sel] = val
    if grf_scale:
        f = _smooth_periodic(g.standard_normal((H, W)), grf_scale)
        f = (f - f.mean()) / max(f.std(), 1e-12)
        x = np.clip(x + 0.2 * f, 0.0, 1.0)
    return x


def kernel_uniform(k):
    return np.full((k, k), 1.0 / (k * k))


def kernel_gaussian(k, sigma):
    l = k // 2
    a = np.arange(-l, l + 1, dtype=np.float64)
    h = np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / (2.0 * sigma * sigma))
    return h / h.sum()


def kernel_motion(k, length, theta):
    """Centred linear-motion segment of the given length and angle on a k x k support."""
    l = k // 2
    h = np.zeros((k, k))
    ns = 64
    for s in range(ns):
        t = ((s + 0.5) / ns - 0.5) * length
        px = l + t * math.cos(theta)        # column coordinate
        py = l - t * math.sin(theta)        # row coordinate
        x0, y0 = int(math.floor(px)), int(math.floor(py))
        fx, fy = px - x0, py - y0
        for dy, wy in ((0, 1.0 - fy), (1, fy)):
            for dx, wx in ((0, 1.0 - fx), (1, fx)):
                yy, xx = y0 + dy, x0 + dx
                if 0 <= yy < k and 0 <= xx < k:
                    h[yy, xx] += wy * wx
    return h / h.sum()


def kernel_disk(radius, k=None):
    """Out-of-focus blur: coverage of a radius-r disk, 16x16 supersampling per pixel."""
    if k is None:
        k = 2 * int(math.ceil(radius)) + 1
    l = k // 2
    sub = (np.arange(16) + 0.5) / 16.0 - 0.5
    h = np.zeros((k, k))
    for i in range(k):
        for j in range(k):
            yy = (i - l) + sub[:, None]
            xx = (j - l) + sub[None, :]
            h[i, j] = np.mean(xx * xx + yy * yy <= radius * radius)
    return h / h.sum()


def valid_mask(H, W, l):
    """1 on the valid region rows/cols l .. side-1-l (pixels of A x free of the boundary)."""
    m = np.zeros((H, W), dtype=np.uint8)
    m[l:H - l, l:W - l] = 1
    return m


def _blur_periodic(x, h):
    """(h (*) x)[r, c] = sum_{a,b} h[a+l, b+l] x[(r-a) mod H, (c-b) mod W]: the
    periodic blur of the whole image, as a product of spectra (the kernel
    wrapped onto the grid with its centre tap at the origin)."""
    H, W = x.shape
    k = h.shape[0]
    l = k // 2
    kp = np.zeros((H, W))
    a = (np.arange(k) - l) % H
    b = (np.arange(k) - l) % W
    np.add.at(kp, (a[:, None], b[None, :]), h)
    return np.fft.irfft2(np.fft.rfft2(x) * np.fft.rfft2(kp), s=(H, W))


def observe(g, x, h, mask, sigma):
    """y = m * (periodic blur of the full image + N(0, sigma^2)); zero off the mask."""
    blurred = _blur_periodic(x, h)
    y = blurred + sigma * g.standard_normal(x.shape)
    return np.where(mask > 0, y, 0.0)


def is_smooth7(n):
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


def next_smooth7(n):
    while not is_smooth7(n):
        n += 1
    return n


# --------------------------------------------------------------------------
# Workloads. Seeds: 1000 * workload + problem index.
# --------------------------------------------------------------------------

def config1(seed_offset=0):
    """128x128, 9x9 uniform blur, valid 120x120, sigma 1e-3, lambda 2e-4, mu 1e-3."""
    g = rng(1000 * 1 + seed_offset)
    H = W = 128
    x = synth_image(g, H, W)
    h = kernel_uniform(9)
    m = valid_mask(H, W, 4)
    y = observe(g, x, h, m, 1e-3)
    return Problem(y=y, mask=m, kernel=h, lam=2e-4, mu1=1e-3, mu2=1e-3, x_true=x)


def config2(index, size=512):
    """Batch member ``index`` (0..7) of the 8 x 512^2 TV workload.

    Images 0-3: 19x19 Gaussian blur sigma 3; images 4-7: 15-px linear motion
    blur at a random angle on a 15x15 support. Mask: valid region minus 40%
    i.i.d. missing interior pixels. sigma = 2e-3, lambda 2e-4, mu 1e-3.
    """
    g = rng(1000 * 2 + index)
    H = W = size
    x = synth_image(g, H, W, grf_scale=32.0)
    if index < 4:
        h = kernel_gaussian(19, 3.0)
    else:
        h = kernel_motion(15, 15.0, g.uniform(0, math.pi))
    l = h.shape[0] // 2
    m = valid_mask(H, W, l)
    m &= (g.uniform(size=(H, W)) >= 0.4).astype(np.uint8)
    y = observe(g, x, h, m, 2e-3)
    return Problem(y=y, mask=m, kernel=h, lam=2e-4, mu1=1e-3, mu2=1e-3, x_true=x)


def config3(size=1024, levels=3):
    """1024^2 frame-analysis workload: 13x13 disk r=6, valid region minus 20% of 8x8 blocks."""
    g = rng(1000 * 3)
    H = W = size
    x = synth_image(g, H, W, grf_scale=32.0)
    h = kernel_disk(6.0, 13)
    l = 6
    m = valid_mask(H, W, l)
    # 8-aligned blocks fully inside the valid interior; drop round(0.2 * count) of them
    r0 = ((l + 7) // 8) * 8
    rows = list(range(r0, H - l - 7, 8))
    cols = list(range(r0, W - l - 7, 8))
    blocks = [(r, c) for r in rows for c in cols]
    nb = int(round(0.2 * len(blocks)))
    for i in g.choice(len(blocks), size=nb, replace=False):
        r, c = blocks[i]
        m[r:r + 8, c:c + 8] = 0
    y = observe(g, x, h, m, 1e-3)
    return Problem(y=y, mask=m, kernel=h, lam=2e-4, mu1=1e-3, mu2=1e-3, x_true=x,
                   reg="frame", levels=levels)


def config4(index, side_lo=128, side_hi=1024):
    """Ragged-batch member: sides uniform in [lo, hi] (H != W) rounded up to 7-smooth,
    kernel family uniform over {Gaussian (sigma k/6), uniform, motion (L = k)} of odd
    size 5..31, lambda log-uniform in [1e-5, 1e-3], mu by the Sec. V heuristic,
    valid-region mask, sigma 1e-3."""
    g = rng(1000 * 4 + index)
    while True:
        H, W = (int(v) for v in g.integers(side_lo, side_hi + 1, size=2))
        if H != W:
            break
    H, W = next_smooth7(H), next_smooth7(W)
    k = int(g.choice(np.arange(5, 32, 2)))
    fam = int(g.integers(0, 3))
    if fam == 0:
        h = kernel_gaussian(k, k / 6.0)
    elif fam == 1:
        h = kernel_uniform(k)
    else:
        h = kernel_motion(k, float(k), g.uniform(0, math.pi))
    lam = float(10.0 ** g.uniform(-5, -3))
    mu2 = 10.0 * lam
    mu1 = min(1.0, 5000.0 * mu2)
    x = synth_image(g, H, W)
    m = valid_mask(H, W, k // 2)
    y = observe(g, x, h, m, 1e-3)
    return Problem(y=y, mask=m, kernel=h, lam=lam, mu1=mu1, mu2=mu2, x_true=x)


def config5_problem(index, size=256):
    """Warm-start data: config-2 image family at ``size``, kernels from the ragged
    families with k <= 19, lambda 2e-4, mu 1e-3, sigma 2e-3. Training draws use
    indices [0, 10^6), evaluation draws start at 10^6 (disjoint seeds)."""
    g = rng(1000 * 5 + 7919 * index)
    H = W = size
    k = int(g.choice(np.arange(5, 20, 2)))
    fam = int(g.integers(0, 3))
    if fam == 0:
        h = kernel_gaussian(k, k / 6.0)
    elif fam == 1:
        h = kernel_uniform(k)
    else:
        h = kernel_motion(k, float(k), g.uniform(0, math.pi))
    x = synth_image(g, H, W, grf_scale=32.0 * size / 512.0)
    m = valid_mask(H, W, k // 2)
    y = observe(g, x, h, m, 2e-3)
    return Problem(y=y, mask=m, kernel=h, lam=2e-4, mu1=1e-3, mu2=1e-3, x_true=x)


def edge_taper(y, h):
    """Edge tapering of an observation before a periodic-boundary solve (the "ET" baseline).

    Written from the published description of edge tapering: the output is a
    weighted sum of y and its periodic blur by h, with weights equal to one in
    the centre and falling to zero at the image edges over a width set by the
    autocorrelation of the kernel. Per axis, the weight at distance d from the
    nearer edge is 1 - a(d) / a(0), a the autocorrelation of the kernel's
    projection on that axis; the 2-D weight is the product of the two axes'.
    Near the edges the data then agree with the periodic model's wrap-around.
    """
    y = np.asarray(y, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)

    def axis_weight(proj, N):
        a = np.correlate(proj, proj, mode="full")[len(proj) - 1:]   # lags 0 .. k-1
        a = a / a[0]
        d = np.minimum(np.arange(N), N - 1 - np.arange(N))
        w = np.ones(N)
        near = d < len(a)
        w[near] = 1.0 - a[d[near]]
        return w

    wv = axis_weight(h.sum(axis=1), y.shape[0])
    wh = axis_weight(h.sum(axis=0), y.shape[1])
    w = wv[:, None] * wh[None, :]
    blurred = ndimage.convolve(y, h, mode="wrap")
    return w * y + (1.0 - w) * blurred


def boundary_pair(index, observed=480, k=25, family="uniform", sigma=1e-3, lam=2e-4, mu=1e-3,
                  reg="tv", levels=3):
    """The same observation posed three ways, for the unknown-boundary comparison of Sec. V.

    The image lives on an (observed + k - 1)^2 domain; y is its blur restricted
    to the central observed^2 pixels that the kernel reaches without crossing
    the image edge (the valid region), plus noise. Returned:

    * ``md``: the mask-decoupled problem on the full domain, mask = the valid
      region, y embedded in it (the boundary pixels are unknown);
    * ``bc``: the same y as a problem on the observed^2 domain alone, mask = 1,
      which makes the periodic-boundary model the method falls back to when
      M = I (Sec. IV-A);
    * ``et``: as ``bc`` with the observation edge-tapered (``edge_taper``);
    * ``x_obs``: the true image on the observed region (ISNR reference);
    * ``y_obs``: the observed^2 data.

    Both sides are 7-smooth for the default sizes (480 and 504). ``reg``:
    "tv" or "frame" (with ``levels``).
    """
    g = rng(1000 * 6 + index)
    l = k // 2
    H = W = observed + 2 * l
    if family == "uniform":
        h = kernel_uniform(k)
    elif family == "gaussian":
        h = kernel_gaussian(k, k / 6.0)
    else:
        h = kernel_motion(k, float(k), g.uniform(0, math.pi))
    x = synth_image(g, H, W, grf_scale=32.0)
    m = valid_mask(H, W, l)
    y = observe(g, x, h, m, sigma)
    J = levels if reg == "frame" else 0
    md = Problem(y=y, mask=m, kernel=h, lam=lam, mu1=mu, mu2=mu, x_true=x, reg=reg, levels=J)
    y_obs = y[l:H - l, l:W - l].copy()
    ones = np.ones_like(y_obs, dtype=np.uint8)
    bc = Problem(y=y_obs, mask=ones, kernel=h, lam=lam, mu1=mu, mu2=mu, reg=reg, levels=J)
    et = Problem(y=edge_taper(y_obs, h), mask=ones, kernel=h, lam=lam, mu1=mu, mu2=mu, reg=reg, levels=J)
    return md, bc, et, x[l:H - l, l:W - l].copy(), y_obs


COMPARISON_BLURS = ("out-of-focus", "linear motion", "uniform", "Gaussian")


def comparison_problem(index, reg="tv", bsnr=40.0, size=256, levels=3):
    """The MD-vs-CG comparison setting of Sec. V: a size x size unknown image
    (the paper's cameraman is 256 x 256), one of four 19 x 19 blurs
    (COMPARISON_BLURS[index]: disk of radius 9, 19-px motion at a random angle,
    uniform, Gaussian sigma 3), observed on the valid region only (the
    (size - 18)^2 pixels free of the boundary), white noise at the given BSNR
    (variance of the valid blurred image over sigma^2, in dB), lambda 2e-4,
    penalties by the rule of Sec. V (mu2 = 10 lambda, mu1 = min(1, 5000 mu2)).
    reg: "tv" or "frame" (undecimated Haar, ``levels`` levels)."""
    g = rng(1000 * 7 + 10 * index + int(bsnr))
    H = W = size
    x = synth_image(g, H, W, grf_scale=16.0)
    k = 19
    if index == 0:
        h = kernel_disk(9.0, k)
    elif index == 1:
        h = kernel_motion(k, 19.0, g.uniform(0, math.pi))
    elif index == 2:
        h = kernel_uniform(k)
    else:
        h = kernel_gaussian(k, 3.0)
    m = valid_mask(H, W, k // 2)
    blurred = _blur_periodic(x, h)
    sigma = math.sqrt(float(np.var(blurred[m > 0])) / 10.0 ** (bsnr / 10.0))
    y = np.where(m > 0, blurred + sigma * g.standard_normal((H, W)), 0.0)
    lam = 2e-4
    mu2 = 10.0 * lam
    return Problem(y=y, mask=m, kernel=h, lam=lam, mu1=min(1.0, 5000.0 * mu2), mu2=mu2, x_true=x,
                   reg=reg, levels=levels if reg == "frame" else 0)
