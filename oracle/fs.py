"""FS-MD: frame-synthesis deconvolution with mask decoupling (float64).

Test infrastructure only (see ``oracle/__init__``).

Problem (Sec. IV-C, eq. (35)): frame coefficients z of the image x = W z,

    min_z  1/2 ||y - M A W z||^2 + lambda ||z||_1,

with W the synthesis operator of a Parseval frame (W W^T = I). Here W = P^T,
the adjoint of the undecimated Haar analysis P used by FA-MD (P^T P = I), so
z has 3J+1 bands of H x W coefficients.

FS-MD is Alg. 2 with H1 = A W (eq. (13)), H2 = I (eq. (14)), g1 the
mask-decoupled data term of eq. (38) with the prox of eq. (40), and
g2 = lambda ||.||_1 with the soft threshold of eq. (16). One iteration, in
the paper's order (gamma = mu2 / mu1):

    zeta = u_k + d_k
    r    = W^T A^T zeta1 + gamma zeta2                       (right side of eq. (17))
    z    = (1 / gamma) (r - W^T F W r)                        (eq. (17) by eq. (18))
           F = A^T (A A^T + gamma I)^{-1} A = U^* Lambda^* (|Lambda|^2 + gamma)^{-1} Lambda U
                                                              (eq. (20))
    u1   = (M^T M + mu1 I)^{-1} (M^T y + mu1 (A W z - d1))    (eq. (40))
    u2   = soft(z - d2, lambda / mu2)                         (eq. (16))
    d1  <- d1 - (A W z - u1),  d2 <- d2 - (z - u2)

The image estimate is x = W z.

Residuals (the same reading as the other solvers): G = (A W; I), so the
primal blocks are A W z - u1 and z - u2, and the dual residual weighs the
changes of u1, u2 by mu1, mu2.

Parity pins: tests/test_oracle_fs.py (the identity of eq. (18) and the
spectral F of eq. (20) against dense inverses; the z-step against the dense
normal equations; the limit against a proximal-gradient minimiser of
eq. (35); the M = I case) and the golden trajectory of tests/golden
(fs_md_4x6_J2: dense matrices, exact rational arithmetic, the z-step as a
dense solve of the normal equations, no identity of eq. (18) assumed).
"""

from dataclasses import dataclass

import numpy as np

from .operators import conv_A, conv_At, dft2, idft2, kernel_spectrum, haar_analysis, haar_synthesis
from .prox import mask_prox, soft

__all__ = ["FSState", "fs_zsolve", "fs_md_step", "fs_md_run", "fs_objective", "fs_residuals"]


@dataclass
class FSState:
    """u = (u1, u2), d = (d1, d2); u2, d2 hold 3J+1 coefficient bands."""
    u1: np.ndarray
    d1: np.ndarray
    u2: np.ndarray
    d2: np.ndarray

    @classmethod
    def zeros(cls, H, W, J):
        nb = 3 * J + 1
        return cls(np.zeros((H, W)), np.zeros((H, W)), np.zeros((nb, H, W)), np.zeros((nb, H, W)))

    def copy(self):
        return FSState(*(np.array(a, dtype=np.float64) for a in (self.u1, self.d1, self.u2, self.d2)))


def fs_zsolve(zeta1, zeta2, h, Lam, gamma, J):
    """z = (W^T A^T A W + gamma I)^{-1} (W^T A^T zeta1 + gamma zeta2) by eqs. (18) and (20)."""
    W = lambda c: haar_synthesis(c, J)
    Wt = lambda x: haar_analysis(x, J)
    F = lambda x: np.real(idft2(np.conj(Lam) * Lam * dft2(x) / (np.abs(Lam) ** 2 + gamma)))
    r = Wt(conv_At(zeta1, h)) + gamma * zeta2
    return (r - Wt(F(W(r)))) / gamma


def fs_md_step(st, y, m, h, lam, mu1, mu2, J, Lam):
    """One FS-MD iteration. Returns (new_state, z_{k+1} (coefficients), (A W z, z))."""
    gamma = mu2 / mu1
    zeta1 = st.u1 + st.d1
    zeta2 = st.u2 + st.d2
    z = fs_zsolve(zeta1, zeta2, h, Lam, gamma, J)
    AWz = conv_A(haar_synthesis(z, J), h)
    u1 = mask_prox(AWz - st.d1, y, m, mu1)
    d1 = st.d1 - (AWz - u1)
    u2 = soft(z - st.d2, lam / mu2)
    d2 = st.d2 - (z - u2)
    return FSState(u1, d1, u2, d2), z, (AWz, z)


def fs_objective(z, y, m, h, lam, J):
    """F(z) = 1/2 ||y - M A W z||^2 + lambda ||z||_1  (eq. (35))."""
    r = np.asarray(m, dtype=np.float64) * (np.asarray(y, dtype=np.float64) - conv_A(haar_synthesis(z, J), h))
    return 0.5 * np.sum(r * r) + lam * np.sum(np.abs(z))


def fs_residuals(aux, st, st_prev, mu1, mu2):
    AWz, z = aux
    pri = np.sqrt(np.sum((AWz - st.u1) ** 2) + np.sum((z - st.u2) ** 2))
    gz = np.sqrt(np.sum(AWz ** 2) + np.sum(z ** 2))
    un = np.sqrt(np.sum(st.u1 ** 2) + np.sum(st.u2 ** 2))
    dual = np.sqrt(mu1 ** 2 * np.sum((st.u1 - st_prev.u1) ** 2) + mu2 ** 2 * np.sum((st.u2 - st_prev.u2) ** 2))
    dn = np.sqrt(mu1 ** 2 * np.sum(st.d1 ** 2) + mu2 ** 2 * np.sum(st.d2 ** 2))
    return pri / max(gz, un, 1e-30), dual / max(dn, 1e-30)


def fs_md_run(y, m, h, lam, mu1, mu2, J, iters, state0=None, record=(), tol=None, check_every=1, obj_tol=None):
    """Run FS-MD for up to ``iters`` iterations from ``state0`` (cold start: zeros).

    Returns dict(z = the last coefficients, x = W z, zs = {k: W z_k} for k in
    record, state, iters, history = [(k, r_pri, r_dual)], converged); the
    stopping rules are those of ``tv_md_run``.
    """
    y = np.asarray(y, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    H, W = y.shape
    Lam = kernel_spectrum(h, H, W)
    st = FSState.zeros(H, W, J) if state0 is None else state0.copy()
    record = set(record)
    xs, history = {}, []
    z, k, converged, f_prev = None, 0, False, None
    for k in range(1, iters + 1):
        new, z, aux = fs_md_step(st, y, m, h, lam, mu1, mu2, J, Lam)
        if k in record:
            xs[k] = haar_synthesis(z, J)
        stop = False
        if tol is not None and k % check_every == 0:
            rp, rd = fs_residuals(aux, new, st, mu1, mu2)
            history.append((k, rp, rd))
            stop = rp <= tol and rd <= tol
        if obj_tol is not None:
            f = fs_objective(z, y, m, h, lam, J)
            if f_prev is not None and abs(f - f_prev) <= obj_tol * abs(f_prev):
                stop = True
            f_prev = f
        st = new
        if stop:
            converged = True
            break
    return dict(z=z, x=haar_synthesis(z, J), zs=xs, state=st, iters=k, history=history, converged=converged)
