"""TV-CG and FA-CG: the Reeves-Sorel alternative to mask decoupling (float64).

Test infrastructure only (see ``oracle/__init__``).

Instead of splitting the mask off the data term (MD), these variants keep
H1 = M A, the observed rows of the blur (Sec. IV-C, eq. (45); Sec. IV-D), so
the data prox is the periodic one of eq. (15) applied to the observed pixels
only, and the z-step matrix of Alg. 2 line 4 is no longer circulant. With B
the rows of A that M removes (so that A^T A = A^T M^T M A + B^T B) and C the
circulant inverse

    TV:  C = (A^T A + gamma (D^h)^T D^h + gamma (D^v)^T D^v)^{-1},
    FA:  C = (A^T A + gamma I)^{-1},                  gamma = mu2 / mu1,

the Sherman-Morrison-Woodbury identity gives (eqs. (43), (47), (51))

    (A^T M^T M A + gamma R^T R)^{-1} = C - C B^T (B C B^T - I)^{-1} B C
                                     = C + C B^T (I - B C B^T)^{-1} B C,

with R = D (TV) or R = I (FA; P^T P = I). The boundary system
(I - B C B^T) v = B C r, of the size of the unobserved pixels, is symmetric
positive definite; the paper solves it approximately with one conjugate
gradient iteration started from the previous outer iteration's estimate, so
that the method carries that estimate v from one iteration to the next.

One iteration (TV-CG: Alg. 3 with A -> M A; FA-CG: Alg. 2 with H1 = M A,
H2 = P):

    zeta = u + d
    r    = mu1 A^T M^T zeta1 + mu2 D^T (u_TV + d_TV)         (TV)
           A^T M^T zeta1 + gamma P^T zeta2                  (FA)
    t    = C r
    v    = cg(I - B C B^T, B t, start = v)   (cg_iters iterations; the paper: 1)
    z    = (t + C B^T v) / mu1                                (TV; FA without / mu1)
    u1   = (y + mu1 (M A z - d1)) / (1 + mu1)    on the observed pixels
    d1   = d1 - (M A z - u1)
    regulariser step as in TV-MD / FA-MD.

u1 and d1 live on the observed pixels; they are stored as full planes that
are zero elsewhere, as is v on the observed pixels.

Readings (the paper does not spell them out): "one CG iteration initialized
with the estimate of the previous outer iteration" is one iteration of a
fresh CG run from that estimate, i.e. a steepest-descent step
v <- v + a res, res = b - S v, a = res^T res / res^T S res (a = 0 when
res = 0); the cold start has v = 0.

Parity pins: tests/test_oracle_cg.py (dense 8x8 matrices: the identity above,
the exact z-step with the boundary system solved to convergence, one CG step
written out on the dense matrices; the limit equals the MD limit, which is
pinned to brute-force minimisers) and the golden trajectories of tests/golden
(tv_cg_5x6, fa_cg_4x6_J2: dense exact / 60-digit arithmetic).
"""

from dataclasses import dataclass

import numpy as np

from .operators import (
    conv_A, conv_At, diff_h, diff_v, diff_ht, diff_vt, dft2, idft2, kernel_spectrum, diff_spectra,
    haar_analysis, haar_synthesis,
)
from .prox import vsoft, soft

__all__ = ["TVCGState", "FACGState", "tv_cg_step", "tv_cg_run", "fa_cg_step", "fa_cg_run",
           "boundary_cg", "cg_zsolve"]


@dataclass
class TVCGState:
    """u = (u1, uh, uv), d = (d1, dh, dv), v: the boundary-system estimate."""
    u1: np.ndarray
    d1: np.ndarray
    uh: np.ndarray
    uv: np.ndarray
    dh: np.ndarray
    dv: np.ndarray
    v: np.ndarray

    @classmethod
    def zeros(cls, H, W):
        z = lambda: np.zeros((H, W))
        return cls(z(), z(), z(), z(), z(), z(), z())

    def copy(self):
        return TVCGState(*(np.array(a, dtype=np.float64) for a in
                           (self.u1, self.d1, self.uh, self.uv, self.dh, self.dv, self.v)))


@dataclass
class FACGState:
    u1: np.ndarray
    d1: np.ndarray
    u2: np.ndarray
    d2: np.ndarray
    v: np.ndarray

    @classmethod
    def zeros(cls, H, W, J):
        nb = 3 * J + 1
        return cls(np.zeros((H, W)), np.zeros((H, W)), np.zeros((nb, H, W)), np.zeros((nb, H, W)),
                   np.zeros((H, W)))

    def copy(self):
        return FACGState(*(np.array(a, dtype=np.float64) for a in (self.u1, self.d1, self.u2, self.d2, self.v)))


def boundary_cg(b, v0, S, iters=1):
    """`iters` conjugate-gradient iterations on S v = b started at v0."""
    v = np.array(v0, dtype=np.float64)
    res = b - S(v)
    p = res.copy()
    rr = float(np.sum(res * res))
    for _ in range(iters):
        if rr == 0.0:
            break
        q = S(p)
        pq = float(np.sum(p * q))
        if pq <= 0.0:
            break
        a = rr / pq
        v = v + a * p
        res = res - a * q
        rr_new = float(np.sum(res * res))
        p = res + (rr_new / rr) * p
        rr = rr_new
    return v


def _circulant_inverse(den):
    return lambda x: np.real(idft2(dft2(x) / den))


def cg_zsolve(r, v0, m, h, den, cg_iters=1):
    """z-step of the Reeves-Sorel variants without the final 1 / mu1 of TV:
    C r + C B^T v, v from cg_iters CG iterations on (I - B C B^T) v = B C r
    started at v0. den: the diagonal of C^{-1} in the DFT domain. Returns (z, v)."""
    C = _circulant_inverse(den)
    mb = 1.0 - m
    B = lambda x: mb * conv_A(x, h)          # the rows of A that M removes (as a zero-filled plane)
    Bt = lambda w: conv_At(mb * w, h)
    S = lambda w: w - B(C(Bt(w)))
    t = C(r)
    v = boundary_cg(B(t), v0, S, cg_iters)
    return t + C(Bt(v)), v


def tv_cg_step(st, y, m, h, lam, mu1, mu2, spectra, cg_iters=1):
    """One TV-CG iteration. Returns (new_state, z_{k+1}, (M A z, D^h z, D^v z))."""
    Lam, Dh, Dv = spectra
    gamma = mu2 / mu1
    den = np.abs(Lam) ** 2 + gamma * (np.abs(Dh) ** 2 + np.abs(Dv) ** 2)
    zeta1 = st.u1 + st.d1
    r = mu1 * conv_At(m * zeta1, h) + mu2 * diff_ht(st.uh + st.dh) + mu2 * diff_vt(st.uv + st.dv)
    w, v = cg_zsolve(r, st.v, m, h, den, cg_iters)
    z = w / mu1
    MAz = m * conv_A(z, h)
    u1 = m * (y + mu1 * (MAz - st.d1)) / (1.0 + mu1)
    d1 = st.d1 - (MAz - u1)
    zh, zv = diff_h(z), diff_v(z)
    uh, uv = vsoft(zh - st.dh, zv - st.dv, lam / mu2)
    dh = st.dh - (zh - uh)
    dv = st.dv - (zv - uv)
    return TVCGState(u1, d1, uh, uv, dh, dv, v), z, (MAz, zh, zv)


def fa_cg_step(st, y, m, h, lam, mu1, mu2, J, Lam, cg_iters=1):
    """One FA-CG iteration. Returns (new_state, z_{k+1}, (M A z, P z))."""
    gamma = mu2 / mu1
    den = np.abs(Lam) ** 2 + gamma
    zeta1 = st.u1 + st.d1
    r = conv_At(m * zeta1, h) + gamma * haar_synthesis(st.u2 + st.d2, J)
    z, v = cg_zsolve(r, st.v, m, h, den, cg_iters)
    MAz = m * conv_A(z, h)
    u1 = m * (y + mu1 * (MAz - st.d1)) / (1.0 + mu1)
    d1 = st.d1 - (MAz - u1)
    Pz = haar_analysis(z, J)
    u2 = soft(Pz - st.d2, lam / mu2)
    d2 = st.d2 - (Pz - u2)
    return FACGState(u1, d1, u2, d2, v), z, (MAz, Pz)


def _run(step, st, iters, record):
    zs, z = {}, None
    for k in range(1, iters + 1):
        st, z, _ = step(st)
        if k in record:
            zs[k] = z.copy()
    return dict(z=z, state=st, iters=iters, zs=zs)


def tv_cg_run(y, m, h, lam, mu1, mu2, iters, state0=None, record=(), cg_iters=1):
    """Run TV-CG for ``iters`` iterations from ``state0`` (cold start: zeros)."""
    y = np.asarray(y, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    H, W = y.shape
    spectra = (kernel_spectrum(h, H, W), *diff_spectra(H, W))
    st = TVCGState.zeros(H, W) if state0 is None else state0.copy()
    return _run(lambda s: tv_cg_step(s, y, m, h, lam, mu1, mu2, spectra, cg_iters), st, iters, set(record))


def fa_cg_run(y, m, h, lam, mu1, mu2, J, iters, state0=None, record=(), cg_iters=1):
    """Run FA-CG for ``iters`` iterations from ``state0`` (cold start: zeros)."""
    y = np.asarray(y, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    H, W = y.shape
    Lam = kernel_spectrum(h, H, W)
    st = FACGState.zeros(H, W, J) if state0 is None else state0.copy()
    return _run(lambda s: fa_cg_step(s, y, m, h, lam, mu1, mu2, J, Lam, cg_iters), st, iters, set(record))
