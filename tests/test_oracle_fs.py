"""Pins of the FP64 oracle's FS-MD (frame synthesis with mask decoupling, Sec. IV-C).

* eq. (18) (the Sherman-Morrison-Woodbury form of the z-step matrix of
  eq. (17)) and the spectral F of eq. (20) against dense inverses;
* the oracle's z-step against the dense normal equations on random inputs,
  and the image it implies, W z, against the circulant solve of the
  analysis formulation (a consequence of W W^T = I that the GPU path uses);
* the whole trajectory against tests/golden/fs_md_4x6_J2 (dense matrices,
  exact rational arithmetic, the z-step as a dense solve), with planted
  mistakes;
* the limit: the objective of eq. (35) at the FS-MD limit equals the minimum
  that accelerated proximal gradient (FISTA, a different algorithm) reaches
  on the same dense problem.
"""

import numpy as np
import pytest

import oracle as O
import oracle.fs as ofs
from golden_fixtures import FS_NAMES, load
from test_oracle_admm import dense_conv, small_problem

TOL = 1e-12


def _dense_W(H, W, J):
    """The synthesis operator W = P^T as an n x d matrix."""
    nb = 3 * J + 1
    n = H * W
    Wm = np.zeros((n, nb * n))
    for i in range(nb * n):
        c = np.zeros(nb * n)
        c[i] = 1.0
        Wm[:, i] = O.haar_synthesis(c.reshape(nb, H, W), J).ravel()
    return Wm


@pytest.mark.parametrize("J", [1, 2])
def test_eq18_and_the_spectral_F_equal_dense_inverses(J):
    H = W = 8
    y, m, h = small_problem(3, H=H, W=W, k=3)
    A = dense_conv(h, H, W)
    Wm = _dense_W(H, W, J)
    assert np.allclose(Wm @ Wm.T, np.eye(H * W), atol=1e-13)           # Parseval: W W^T = I
    gamma = 0.3
    F = A.T @ np.linalg.solve(A @ A.T + gamma * np.eye(H * W), A)
    d = Wm.shape[1]
    lhs = np.linalg.inv(Wm.T @ A.T @ A @ Wm + gamma * np.eye(d))
    rhs = (np.eye(d) - Wm.T @ F @ Wm) / gamma
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-10 * np.abs(lhs).max())
    # eq. (20): F through the kernel spectrum, on a random image
    Lam = O.kernel_spectrum(h, H, W)
    x = np.random.default_rng(1).standard_normal((H, W))
    Fx = np.real(O.idft2(np.conj(Lam) * Lam * O.dft2(x) / (np.abs(Lam) ** 2 + gamma)))
    np.testing.assert_allclose(Fx.ravel(), F @ x.ravel(), rtol=0, atol=1e-12)


@pytest.mark.parametrize("J", [1, 3])
def test_zstep_is_the_dense_normal_equations(J):
    H, W = 8, 8
    y, m, h = small_problem(5, H=H, W=W, k=5)
    A = dense_conv(h, H, W)
    Wm = _dense_W(H, W, J)
    gamma = 0.7
    g = np.random.default_rng(J)
    zeta1 = g.standard_normal((H, W))
    zeta2 = g.standard_normal((3 * J + 1, H, W))
    Lam = O.kernel_spectrum(h, H, W)
    z = O.fs_zsolve(zeta1, zeta2, h, Lam, gamma, J)
    AW = A @ Wm
    exact = np.linalg.solve(AW.T @ AW + gamma * np.eye(AW.shape[1]), AW.T @ zeta1.ravel() + gamma * zeta2.ravel())
    np.testing.assert_allclose(z.ravel(), exact, rtol=0, atol=1e-10 * np.abs(exact).max())
    # the image W z is the circulant solve (A^T A + gamma I)^{-1} (A^T zeta1 + gamma W zeta2)
    x = O.zsolve_fa(O.conv_At(zeta1, h) + gamma * O.haar_synthesis(zeta2, J), Lam, gamma)
    np.testing.assert_allclose(O.haar_synthesis(z, J), x, rtol=0, atol=1e-10 * np.abs(x).max())


def _fs_run(g, record=()):
    return O.fs_md_run(g["y"], g["mask"], g["kernel"], g["lambda"], g["mu1"], g["mu2"], g["levels"],
                       iters=g["iters"], record=record)


def _history(g):
    y, m, h = g["y"], g["mask"].astype(np.float64), g["kernel"]
    H, W = g["shape"]
    Lam = O.kernel_spectrum(h, H, W)
    st = O.FSState.zeros(H, W, g["levels"])
    out = {}
    for k in range(1, g["iters"] + 1):
        new, z, aux = O.fs_md_step(st, y, m, h, g["lambda"], g["mu1"], g["mu2"], g["levels"], Lam)
        out[k] = O.fs_residuals(aux, new, st, g["mu1"], g["mu2"])
        st = new
    return out


@pytest.mark.parametrize("name", FS_NAMES)
def test_fs_oracle_matches_exact_trajectory(name):
    g = load(name)
    assert g["method"] == "fs"
    res = _fs_run(g, record=tuple(g["zs"]))
    for k, xk in g["zs"].items():
        err = np.max(np.abs(res["zs"][k] - xk))
        assert err <= TOL * max(1.0, np.max(np.abs(xk))), (name, k, err)
    f = O.fs_objective(res["z"], g["y"], g["mask"], g["kernel"], g["lambda"], g["levels"])
    assert abs(f - g["objective"][1]) <= TOL * abs(g["objective"][1])
    hist = _history(g)
    for k, (rp, rd) in g["residuals"].items():
        assert abs(hist[k][0] - rp) <= TOL * rp and abs(hist[k][1] - rd) <= TOL * rd, (name, k)


_zsolve = ofs.fs_zsolve


@pytest.mark.parametrize("mutation", ["gamma_inverted", "no_F_term", "lambda_not_over_mu2", "no_adjoint_W"])
def test_planted_fs_mistake_is_caught(mutation, monkeypatch):
    if mutation == "gamma_inverted":          # eq. (18) with mu2/mu1 in place of mu1/mu2 as the factor
        monkeypatch.setattr(ofs, "fs_zsolve", lambda z1, z2, h, L, g, J: _zsolve(z1, z2, h, L, g, J) * g * g)
    elif mutation == "no_F_term":           # the identity part of eq. (18) alone
        monkeypatch.setattr(ofs, "fs_zsolve",
                            lambda z1, z2, h, L, g, J: (O.haar_analysis(O.conv_At(z1, h), J) + g * z2) / g)
    elif mutation == "lambda_not_over_mu2":  # soft threshold by lambda instead of lambda / mu2
        real_soft = ofs.soft
        monkeypatch.setattr(ofs, "soft", lambda v, t: real_soft(v, t * 0.25))
    else:                                   # W in place of W^T on the data term (a transposed operand)
        monkeypatch.setattr(ofs, "fs_zsolve",
                            lambda z1, z2, h, L, g, J: _zsolve(O.conv_A(z1, h), z2, h, L, g, J))
    for name in FS_NAMES:
        g = load(name)
        res = _fs_run(g, record=tuple(g["zs"]))
        err = max(np.max(np.abs(res["zs"][k] - xk)) for k, xk in g["zs"].items())
        assert err > 1e-6, (mutation, name, err)


def test_fs_limit_is_the_minimum_of_eq35():
    # FISTA (Beck-Teboulle) on the dense lasso of eq. (35) reaches the same
    # minimum as FS-MD run to convergence
    H, W, J = 8, 8, 1
    y, m, h = small_problem(11, H=H, W=W, k=3, p_missing=0.2)
    lam, mu1, mu2 = 0.01, 0.05, 0.05
    run = O.fs_md_run(y, m, h, lam, mu1, mu2, J, iters=4000)
    F = lambda z: O.fs_objective(z, y, m, h, lam, J)
    f_admm = F(run["z"])
    B = np.diag(m.ravel().astype(np.float64)) @ dense_conv(h, H, W) @ _dense_W(H, W, J)
    L = np.linalg.norm(B, 2) ** 2
    z = np.zeros(B.shape[1])
    w, t = z.copy(), 1.0
    yv = (m * y).ravel()
    for _ in range(20000):
        zn = O.soft(w - B.T @ (B @ w - yv) / L, lam / L)
        tn = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        w = zn + ((t - 1.0) / tn) * (zn - z)
        z, t = zn, tn
    f_fista = F(z.reshape(3 * J + 1, H, W))
    assert abs(f_admm - f_fista) <= 1e-11 * f_fista, (f_admm, f_fista)
