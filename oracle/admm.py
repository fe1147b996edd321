"""TV-MD and FA-MD iterations, objectives, residuals and warm-start state (float64).

Test infrastructure only (see ``oracle/__init__``).

TV-MD (Sec. IV-D): Alg. 3 (ADMM-TV) with the data-term update replaced by
eq. (49). One iteration, in the paper's notation (u, d partitioned as
u = (u^(1), u_TV), d the negated scaled dual of Alg. 1):

    zeta        = u_k + d_k                                   (Alg. 2/3)
    delta^h,v   = horizontal / vertical components of zeta_TV
    z_{k+1}     = K (mu1 A^T zeta^(1) + mu2 (D^h)^T delta^h + mu2 (D^v)^T delta^v)
                  with K = U^*(mu1|Lambda|^2 + mu2|Delta^h|^2 + mu2|Delta^v|^2)^{-1} U
                                                              (eq. (33))
    u^(1)_{k+1} = (M^T M + mu1 I)^{-1}(M^T y + mu1 (A z_{k+1} - d^(1)_k))   (eq. (49))
    d^(1)_{k+1} = d^(1)_k - (A z_{k+1} - u^(1)_{k+1})
    u_TV,i      = vsoft(D_i z_{k+1} - d_TV,i, lambda / mu2)
    d_TV,i      = d_TV,i - (D_i z_{k+1} - u_TV,i)

FA-MD (Sec. IV-C): Alg. 2 with H1 = A, H2 = P (Parseval frame), the z-step
of eqs. (24)-(25) with gamma = mu2 / mu1, the data prox of eq. (40) and the
soft threshold of eq. (16) on every frame coefficient (reading: the
objective penalises all of P x, eq. (44), so the coarse band is included).

Residuals (reading; the paper stops on the relative change of the objective,
Sec. V): with G the stacked operator of eq. (3) and Upsilon = diag(mu1 on the
data block, mu2 on the regulariser block) of eq. (5),

    r_pri  = ||G z_k - u_k|| / max(||G z_k||, ||u_k||)
    r_dual = ||Upsilon (u_k - u_{k-1})|| / max(||Upsilon d_k||, 1e-30).

Warm start (not in the paper; Theorem 1 allows any u_0, d_0): from a guess
x0 and a dual field p0 (projected to ||p0_i|| <= 1) the state is set to the
values the ADMM fixed point takes (KKT conditions of the two prox steps):
u^(1) = A x0, d^(1) = M^T (y - M A x0) / mu1, u_TV = D x0, d_TV = -(lambda/mu2) p0.

Parity pins: tests/test_oracle_admm.py (closed-form first two iterations, the
dense 8x8 z-solve, brute-force minimisers of the smoothed objective on 8x8
problems, lambda-large closed forms, mu- and initialisation-independence of
the limit, the M = I special case, the d^(1) = 0 off-mask invariant) and
tests/test_oracle_golden.py (iterates, objectives and both residuals of tiny
TV-MD and FA-MD problems against dense exact / 60-digit computations, with
planted mistakes in the residuals: a dropped block, mu in place of mu^2,
d_{k-1} in place of d_k, a band left out).
"""

from dataclasses import dataclass, field

import numpy as np

from .operators import (
    conv_A, conv_At, diff_h, diff_v, diff_ht, diff_vt,
    dft2, idft2, kernel_spectrum, diff_spectra, haar_analysis, haar_synthesis,
)
from .prox import mask_prox, vsoft, soft

__all__ = [
    "TVState", "FAState", "tv_md_step", "tv_md_run", "fa_md_step", "fa_md_run",
    "tv_objective", "fa_objective", "tv_residuals", "fa_residuals",
    "warm_start_state", "zsolve_tv", "zsolve_fa", "default_mu",
]


def default_mu(lam):
    """Penalty heuristic of Sec. V: mu2 = 10 lambda, mu1 = min(1, 5000 mu2).

    Reading: the printed rule sets mu1 from itself; the second mu1 is read as
    mu2. The choice affects convergence speed only, never the minimiser.
    """
    mu2 = 10.0 * lam
    mu1 = min(1.0, 5000.0 * mu2)
    return mu1, mu2


@dataclass
class TVState:
    """u = (u1, uh, uv), d = (d1, dh, dv); every block is an H x W float64 plane."""
    u1: np.ndarray
    d1: np.ndarray
    uh: np.ndarray
    uv: np.ndarray
    dh: np.ndarray
    dv: np.ndarray

    @classmethod
    def zeros(cls, H, W):
        z = lambda: np.zeros((H, W))
        return cls(z(), z(), z(), z(), z(), z())

    def copy(self):
        return TVState(*(np.array(a, dtype=np.float64) for a in
                         (self.u1, self.d1, self.uh, self.uv, self.dh, self.dv)))


@dataclass
class FAState:
    """u = (u1, u2), d = (d1, d2); u2, d2 hold the 3J+1 frame bands."""
    u1: np.ndarray
    d1: np.ndarray
    u2: np.ndarray
    d2: np.ndarray

    @classmethod
    def zeros(cls, H, W, J):
        nb = 3 * J + 1
        return cls(np.zeros((H, W)), np.zeros((H, W)),
                   np.zeros((nb, H, W)), np.zeros((nb, H, W)))

    def copy(self):
        return FAState(*(np.array(a, dtype=np.float64) for a in
                         (self.u1, self.d1, self.u2, self.d2)))


def _spectra(h, H, W):
    Lam = kernel_spectrum(h, H, W)
    Dh, Dv = diff_spectra(H, W)
    return Lam, Dh, Dv


def zsolve_tv(rhs, Lam, Dh, Dv, mu1, mu2):
    """z = K rhs, K = U^*(mu1|Lambda|^2 + mu2|Delta^h|^2 + mu2|Delta^v|^2)^{-1} U  (eq. (33))."""
    denom = mu1 * np.abs(Lam) ** 2 + mu2 * np.abs(Dh) ** 2 + mu2 * np.abs(Dv) ** 2
    return np.real(idft2(dft2(rhs) / denom))


def zsolve_fa(rhs, Lam, gamma):
    """z = U^*(|Lambda|^2 + gamma)^{-1} U rhs  (eq. (25))."""
    return np.real(idft2(dft2(rhs) / (np.abs(Lam) ** 2 + gamma)))


def tv_md_step(st, y, m, h, lam, mu1, mu2, spectra):
    """One TV-MD iteration. Returns (new_state, z_{k+1}, (A z, D^h z, D^v z))."""
    Lam, Dh, Dv = spectra
    zeta1 = st.u1 + st.d1
    delta_h = st.uh + st.dh
    delta_v = st.uv + st.dv
    rhs = mu1 * conv_At(zeta1, h) + mu2 * diff_ht(delta_h) + mu2 * diff_vt(delta_v)
    z = zsolve_tv(rhs, Lam, Dh, Dv, mu1, mu2)
    Az = conv_A(z, h)
    u1 = mask_prox(Az - st.d1, y, m, mu1)
    d1 = st.d1 - (Az - u1)
    zh, zv = diff_h(z), diff_v(z)
    uh, uv = vsoft(zh - st.dh, zv - st.dv, lam / mu2)
    dh = st.dh - (zh - uh)
    dv = st.dv - (zv - uv)
    return TVState(u1, d1, uh, uv, dh, dv), z, (Az, zh, zv)


def tv_objective(x, y, m, h, lam):
    """F(x) = 1/2 ||y - M A x||^2 + lambda sum_i ||D_i x||_2  (eq. (48))."""
    r = np.asarray(m, dtype=np.float64) * (np.asarray(y, dtype=np.float64) - conv_A(x, h))
    return 0.5 * np.sum(r * r) + lam * np.sum(np.sqrt(diff_h(x) ** 2 + diff_v(x) ** 2))


def tv_residuals(aux, st, st_prev, mu1, mu2):
    """(r_pri, r_dual) of the TV splitting (see module header)."""
    Az, zh, zv = aux
    pri = np.sqrt(np.sum((Az - st.u1) ** 2) + np.sum((zh - st.uh) ** 2) + np.sum((zv - st.uv) ** 2))
    gz = np.sqrt(np.sum(Az ** 2) + np.sum(zh ** 2) + np.sum(zv ** 2))
    un = np.sqrt(np.sum(st.u1 ** 2) + np.sum(st.uh ** 2) + np.sum(st.uv ** 2))
    dual = np.sqrt(mu1 ** 2 * np.sum((st.u1 - st_prev.u1) ** 2)
                   + mu2 ** 2 * (np.sum((st.uh - st_prev.uh) ** 2) + np.sum((st.uv - st_prev.uv) ** 2)))
    dn = np.sqrt(mu1 ** 2 * np.sum(st.d1 ** 2) + mu2 ** 2 * (np.sum(st.dh ** 2) + np.sum(st.dv ** 2)))
    return pri / max(gz, un, 1e-30), dual / max(dn, 1e-30)


def _run(step, objective, residuals, st, iters, record, tol, check_every, obj_tol):
    zs = {}
    history = []
    z = None
    k = 0
    converged = False
    f_prev = None
    for k in range(1, iters + 1):
        st_new, z, aux = step(st)
        if k in record:
            zs[k] = z.copy()
        stop = False
        if tol is not None and k % check_every == 0:
            rp, rd = residuals(aux, st_new, st)
            history.append((k, rp, rd))
            stop = rp <= tol and rd <= tol
        if obj_tol is not None:
            f = objective(z)
            if f_prev is not None and abs(f - f_prev) <= obj_tol * abs(f_prev):
                stop = True
            f_prev = f
        st = st_new
        if stop:
            converged = True
            break
    return dict(z=z, state=st, iters=k, zs=zs, history=history, converged=converged)


def tv_md_run(y, m, h, lam, mu1, mu2, iters, state0=None, record=(), tol=None,
              check_every=1, obj_tol=None):
    """Run TV-MD for up to ``iters`` iterations from ``state0`` (cold start: zeros).

    ``tol``: stop at the first iteration k with k % check_every == 0 where both
    residuals are <= tol. ``obj_tol``: the paper's rule, stop when the relative
    change of the objective falls below it (Sec. V).
    """
    y = np.asarray(y, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    H, W = y.shape
    spectra = _spectra(h, H, W)
    st = TVState.zeros(H, W) if state0 is None else state0.copy()
    step = lambda s: tv_md_step(s, y, m, h, lam, mu1, mu2, spectra)
    obj = lambda x: tv_objective(x, y, m, h, lam)
    res = lambda aux, s, sp: tv_residuals(aux, s, sp, mu1, mu2)
    return _run(step, obj, res, st, iters, set(record), tol, check_every, obj_tol)


def fa_md_step(st, y, m, h, lam, mu1, mu2, J, Lam):
    """One FA-MD iteration. Returns (new_state, z_{k+1}, (A z, P z))."""
    gamma = mu2 / mu1
    zeta1 = st.u1 + st.d1
    zeta2 = st.u2 + st.d2
    z = zsolve_fa(conv_At(zeta1, h) + gamma * haar_synthesis(zeta2, J), Lam, gamma)
    Az = conv_A(z, h)
    u1 = mask_prox(Az - st.d1, y, m, mu1)
    d1 = st.d1 - (Az - u1)
    Pz = haar_analysis(z, J)
    u2 = soft(Pz - st.d2, lam / mu2)
    d2 = st.d2 - (Pz - u2)
    return FAState(u1, d1, u2, d2), z, (Az, Pz)


def fa_objective(x, y, m, h, lam, J):
    """F(x) = 1/2 ||y - M A x||^2 + lambda ||P x||_1  (eq. (44))."""
    r = np.asarray(m, dtype=np.float64) * (np.asarray(y, dtype=np.float64) - conv_A(x, h))
    return 0.5 * np.sum(r * r) + lam * np.sum(np.abs(haar_analysis(x, J)))


def fa_residuals(aux, st, st_prev, mu1, mu2):
    Az, Pz = aux
    pri = np.sqrt(np.sum((Az - st.u1) ** 2) + np.sum((Pz - st.u2) ** 2))
    gz = np.sqrt(np.sum(Az ** 2) + np.sum(Pz ** 2))
    un = np.sqrt(np.sum(st.u1 ** 2) + np.sum(st.u2 ** 2))
    dual = np.sqrt(mu1 ** 2 * np.sum((st.u1 - st_prev.u1) ** 2)
                   + mu2 ** 2 * np.sum((st.u2 - st_prev.u2) ** 2))
    dn = np.sqrt(mu1 ** 2 * np.sum(st.d1 ** 2) + mu2 ** 2 * np.sum(st.d2 ** 2))
    return pri / max(gz, un, 1e-30), dual / max(dn, 1e-30)


def fa_md_run(y, m, h, lam, mu1, mu2, J, iters, state0=None, record=(), tol=None,
              check_every=1, obj_tol=None):
    """Run FA-MD (see ``tv_md_run`` for the stopping arguments)."""
    y = np.asarray(y, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    H, W = y.shape
    Lam = kernel_spectrum(h, H, W)
    st = FAState.zeros(H, W, J) if state0 is None else state0.copy()
    step = lambda s: fa_md_step(s, y, m, h, lam, mu1, mu2, J, Lam)
    obj = lambda x: fa_objective(x, y, m, h, lam, J)
    res = lambda aux, s, sp: fa_residuals(aux, s, sp, mu1, mu2)
    return _run(step, obj, res, st, iters, set(record), tol, check_every, obj_tol)


def warm_start_state(x0, p0h, p0v, y, m, h, lam, mu1, mu2):
    """TV state that is an ADMM fixed point when (x0, p0) solve the KKT system."""
    x0 = np.asarray(x0, dtype=np.float64)
    p0h = np.asarray(p0h, dtype=np.float64)
    p0v = np.asarray(p0v, dtype=np.float64)
    nrm = np.maximum(1.0, np.sqrt(p0h ** 2 + p0v ** 2))
    ph, pv = p0h / nrm, p0v / nrm
    Ax = conv_A(x0, h)
    m = np.asarray(m, dtype=np.float64)
    d1 = m * (np.asarray(y, dtype=np.float64) - Ax) / mu1
    return TVState(u1=Ax, d1=d1, uh=diff_h(x0), uv=diff_v(x0),
                   dh=-(lam / mu2) * ph, dv=-(lam / mu2) * pv)
