"""Float64 reference for the warm-start network's layers (test infrastructure only).

The warm-start CNN is not part of the paper; it is a learned initialiser whose
output only sets u_0, d_0 (which Theorem 1 lets be arbitrary). This module
writes out the plain definitions of its layers:

* 3x3 convolution with dilation d, stride 1, zero padding d, NHWC activations
  x[n, r, c, ci], weights w[ky, kx, ci, co], bias b[co]:
      y[n, r, c, co] = b[co] + sum_{ky,kx,ci} x[n, r+(ky-1)d, c+(kx-1)d, ci] w[ky, kx, ci, co]
  (cross-correlation, the deep-learning convention), and its two gradients
  with respect to x (dgrad) and to w, b (wgrad);
* ReLU;
* one Adam step (Kingma & Ba, 2015, Algorithm 1) with bias correction.

Parity pins: tests/test_oracle_cnn.py (central finite differences of a scalar
loss, agreement with torch.nn.functional.conv2d on the CPU at dilations 1-3,
a dilated convolution against the plain one with a zero-stuffed kernel, Adam's closed-form
first step and agreement with torch.optim.Adam on the CPU).
"""

import numpy as np

__all__ = ["conv3x3_fwd", "conv3x3_dgrad", "conv3x3_wgrad", "relu", "adam_step"]


def _pad(x, p=1):
    return np.pad(np.asarray(x, dtype=np.float64), ((0, 0), (p, p), (p, p), (0, 0)))


def conv3x3_fwd(x, w, b=None, dil=1):
    """y = conv3x3_d(x, w) + b. x: (N, H, W, Ci), w: (3, 3, Ci, Co) -> (N, H, W, Co)."""
    N, H, W, _ = x.shape
    w = np.asarray(w, dtype=np.float64)
    d = dil
    xp = _pad(x, d)
    y = np.zeros((N, H, W, w.shape[3]))
    for ky in range(3):
        for kx in range(3):
            # x at (r + (ky - 1) d) is xp at (r + ky d)
            y += xp[:, ky * d:ky * d + H, kx * d:kx * d + W, :] @ w[ky, kx]
    if b is not None:
        y += np.asarray(b, dtype=np.float64)
    return y


def conv3x3_dgrad(dy, w, dil=1):
    """dL/dx given dL/dy: dx[n,r,c,ci] = sum_{ky,kx,co} dy[n, r-(ky-1)d, c-(kx-1)d, co] w[ky,kx,ci,co]."""
    N, H, W, _ = dy.shape
    w = np.asarray(w, dtype=np.float64)
    d = dil
    dyp = _pad(dy, d)
    dx = np.zeros((N, H, W, w.shape[2]))
    for ky in range(3):
        for kx in range(3):
            # dy at (r - (ky - 1) d) is dyp at (r + (2 - ky) d)
            dx += dyp[:, (2 - ky) * d:(2 - ky) * d + H, (2 - kx) * d:(2 - kx) * d + W, :] @ w[ky, kx].T
    return dx


def conv3x3_wgrad(x, dy, dil=1):
    """(dL/dw, dL/db): dw[ky,kx,ci,co] = sum_{n,r,c} x[n, r+(ky-1)d, c+(kx-1)d, ci] dy[n,r,c,co]."""
    N, H, W, Ci = x.shape
    dy = np.asarray(dy, dtype=np.float64)
    d = dil
    xp = _pad(x, d)
    dw = np.zeros((3, 3, Ci, dy.shape[3]))
    for ky in range(3):
        for kx in range(3):
            xs = xp[:, ky * d:ky * d + H, kx * d:kx * d + W, :].reshape(-1, Ci)
            dw[ky, kx] = xs.T @ dy.reshape(-1, dy.shape[3])
    return dw, dy.sum(axis=(0, 1, 2))


def relu(x):
    return np.maximum(np.asarray(x, dtype=np.float64), 0.0)


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1. Returns (p_new, m_new, v_new)."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
