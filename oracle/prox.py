"""Proximity operators used by the ADMM splittings (float64, closed forms).

Test infrastructure only (see ``oracle/__init__``).

* ``mask_prox``: prox of g1(v) = 1/2 ||y - M v||^2 / mu1, i.e.
  (M^T M + mu1 I)^{-1} (M^T y + mu1 v)                      (Sec. IV-B, eq. (40)).
  M^T M is the diagonal of the 0/1 mask m and M^T y is y zero-filled where
  m = 0, so the operator is per pixel. With m = 1 everywhere it reduces to
  the periodic-boundary prox (y + mu1 v) / (1 + mu1) of eq. (15).
* ``vsoft``: prox of lambda ||v||_2 / mu2 on 2-vectors (vector soft
  threshold, Sec. III-C) with the convention 0 / ||0|| = 0.
* ``soft``: prox of lambda ||v||_1 / mu2, the component-wise soft threshold of
  eq. (8) with threshold lambda / mu2 (eq. (16)); sign(0) = 0.

Parity pins: tests/test_oracle_prox.py (first-order optimality, brute-force
scalar and radial scans, special cases m = 0 and m = 1).
"""

import numpy as np

__all__ = ["mask_prox", "vsoft", "soft"]


def mask_prox(v, y, m, mu1):
    """u = (m * y + mu1 * v) / (m + mu1), elementwise, m in {0, 1}."""
    v = np.asarray(v, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    My = m * np.asarray(y, dtype=np.float64)      # M^T y: zero-filled outside the mask
    return (My + mu1 * v) / (m + mu1)


def vsoft(vh, vv, tau):
    """Vector soft threshold of the 2-vectors (vh[i], vv[i]) by tau.

    u = v / ||v|| * max(||v|| - tau, 0), and u = 0 where ||v|| <= tau
    (which also covers v = 0, the 0/0 convention of Sec. III-C).
    """
    vh = np.asarray(vh, dtype=np.float64)
    vv = np.asarray(vv, dtype=np.float64)
    rho = np.sqrt(vh * vh + vv * vv)
    keep = rho > tau
    scale = np.zeros_like(rho)
    scale[keep] = (rho[keep] - tau) / rho[keep]
    return vh * scale, vv * scale


def soft(v, tau):
    """soft(v, tau) = sign(v) * max(|v| - tau, 0), elementwise (eq. (8))."""
    v = np.asarray(v, dtype=np.float64)
    return np.sign(v) * np.maximum(np.abs(v) - tau, 0.0)
