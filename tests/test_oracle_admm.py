"""Pins for oracle/admm.py.

Each check rests on something other than the oracle itself: closed forms of
the first iterations (via numpy.fft), dense-matrix solves built with
scipy.signal.convolve2d, certified brute-force minimisers of the smoothed
objective, lambda-large closed forms derived from the optimality conditions,
and properties Theorem 1 fixes (limit independent of mu and of u_0, d_0).
"""

import numpy as np
import pytest
from scipy import signal

import oracle as O
from oracle import admm as oadmm


# ---------------------------------------------------------------- helpers

def dense_conv(h, H, W):
    n = H * W
    A = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = signal.convolve2d(e.reshape(H, W), h, mode="same", boundary="wrap").ravel()
    return A


def dense_diffs(H, W):
    n = H * W
    Dh = np.zeros((n, n))
    Dv = np.zeros((n, n))
    for r in range(H):
        for c in range(W):
            i = r * W + c
            Dh[i, i] -= 1.0
            Dh[i, r * W + (c + 1) % W] += 1.0
            Dv[i, i] -= 1.0
            Dv[i, ((r + 1) % H) * W + c] += 1.0
    return Dh, Dv


def small_problem(seed, H=8, W=8, k=3, p_missing=0.0):
    g = np.random.default_rng(seed)
    h = np.abs(g.standard_normal((k, k))) + 0.1
    h /= h.sum()
    l = k // 2
    m = np.zeros((H, W))
    m[l:H - l, l:W - l] = 1.0
    if p_missing:
        m *= (g.uniform(size=(H, W)) >= p_missing)
    x = (g.uniform(size=(H, W)) > 0.5).astype(float)
    y = m * (signal.convolve2d(x, h, mode="same", boundary="wrap") + 0.02 * g.standard_normal((H, W)))
    return y, m, h


def newton_min(fgh, x0, eps_list=tuple(10.0 ** -e for e in range(2, 11))):
    """Damped Newton with backtracking on each smoothed objective, with continuation."""
    x = x0.copy()
    for eps in eps_list:
        for _ in range(300):
            f, g, Hs = fgh(x, eps)
            step = np.linalg.solve(Hs + 1e-13 * np.eye(len(x)), -g)
            dec = -g @ step
            if dec < 1e-24:
                break
            t = 1.0
            while fgh(x + t * step, eps, only_f=True) > f - 0.25 * t * dec and t > 1e-12:
                t *= 0.5
            x = x + t * step
    return x


def tv_smoothed(A, Dh, Dv, m, y, lam):
    def fgh(x, eps, only_f=False):
        p, q = Dh @ x, Dv @ x
        s = np.sqrt(p * p + q * q + eps * eps)
        r = m * (A @ x) - y
        f = 0.5 * r @ r + lam * s.sum()
        if only_f:
            return f
        g = A.T @ (m * r) + lam * (Dh.T @ (p / s) + Dv.T @ (q / s))
        G = p[:, None] * Dh + q[:, None] * Dv
        Hs = (A.T @ (m[:, None] * A)
              + lam * (Dh.T @ ((1 / s)[:, None] * Dh) + Dv.T @ ((1 / s)[:, None] * Dv)
                       - G.T @ ((1 / s ** 3)[:, None] * G)))
        return f, g, Hs
    return fgh


def fa_smoothed(A, P, m, y, lam):
    def fgh(x, eps, only_f=False):
        c = P @ x
        s = np.sqrt(c * c + eps * eps)
        r = m * (A @ x) - y
        f = 0.5 * r @ r + lam * s.sum()
        if only_f:
            return f
        g = A.T @ (m * r) + lam * P.T @ (c / s)
        Hs = A.T @ (m[:, None] * A) + lam * P.T @ ((eps * eps / s ** 3)[:, None] * P)
        return f, g, Hs
    return fgh


# ------------------------------------------------------- closed forms

def test_first_two_iterations_closed_form():
    y, m, h = small_problem(1, H=12, W=10, k=5, p_missing=0.2)
    mu1, mu2, lam = 0.3, 0.2, 0.05
    out = O.tv_md_run(y, m, h, lam, mu1, mu2, iters=2, record=(1, 2))
    assert np.all(out["zs"][1] == 0.0)                       # z_1 = 0 from a cold start
    one = O.tv_md_run(y, m, h, lam, mu1, mu2, iters=1)["state"]
    u1 = m * y / (m + mu1)
    np.testing.assert_allclose(one.u1, u1, atol=1e-15)
    np.testing.assert_allclose(one.d1, u1, atol=1e-15)
    assert np.all(one.uh == 0) and np.all(one.dv == 0)
    # z_2 = (2 mu1 / (1 + mu1)) IDFT(Khat conj(Lam) DFT(m y)), with numpy.fft
    H, W = y.shape
    hp = np.zeros((H, W))
    l = h.shape[0] // 2
    for a in range(-l, l + 1):
        for b in range(-l, l + 1):
            hp[a % H, b % W] += h[a + l, b + l]
    Lam = np.fft.fft2(hp)
    k1 = np.arange(H)[:, None]
    k2 = np.arange(W)[None, :]
    dd = (2 - 2 * np.cos(2 * np.pi * k1 / H)) + (2 - 2 * np.cos(2 * np.pi * k2 / W))
    Khat = 1.0 / (mu1 * np.abs(Lam) ** 2 + mu2 * dd)
    z2 = (2 * mu1 / (1 + mu1)) * np.real(np.fft.ifft2(Khat * np.conj(Lam) * np.fft.fft2(m * y)))
    np.testing.assert_allclose(out["zs"][2], z2, rtol=0, atol=1e-12 * np.abs(z2).max())


def test_first_iteration_residuals_are_one():
    y, m, h = small_problem(2, k=3)
    out = O.tv_md_run(y, m, h, 0.05, 0.3, 0.2, iters=1, tol=1e-30, check_every=1)
    k, rp, rd = out["history"][0]
    assert k == 1 and abs(rp - 1.0) < 1e-14 and abs(rd - 1.0) < 1e-14


@pytest.mark.parametrize("k", [3, 5])
def test_zsolve_matches_dense_inverse(k):
    H, W = 8, 8
    g = np.random.default_rng(k)
    h = g.standard_normal((k, k))
    rhs = g.standard_normal((H, W))
    mu1, mu2 = 0.7, 0.3
    A = dense_conv(h, H, W)
    Dh, Dv = dense_diffs(H, W)
    Lam = O.kernel_spectrum(h, H, W)
    Sh, Sv = O.diff_spectra(H, W)
    Mtv = mu1 * A.T @ A + mu2 * (Dh.T @ Dh + Dv.T @ Dv)
    np.testing.assert_allclose(O.zsolve_tv(rhs, Lam, Sh, Sv, mu1, mu2).ravel(),
                               np.linalg.solve(Mtv, rhs.ravel()), atol=1e-10)
    gamma = mu2 / mu1
    np.testing.assert_allclose(O.zsolve_fa(rhs, Lam, gamma).ravel(),
                               np.linalg.solve(A.T @ A + gamma * np.eye(H * W), rhs.ravel()), atol=1e-10)


def test_zsolve_recovers_rhs_at_larger_size():
    H, W = 24, 30
    g = np.random.default_rng(3)
    h = np.abs(g.standard_normal((7, 7)))
    h /= h.sum()
    rhs = g.standard_normal((H, W))
    mu1, mu2 = 1e-3, 1e-3
    Lam = O.kernel_spectrum(h, H, W)
    Sh, Sv = O.diff_spectra(H, W)
    z = O.zsolve_tv(rhs, Lam, Sh, Sv, mu1, mu2)
    back = mu1 * O.conv_At(O.conv_A(z, h), h) + mu2 * (O.diff_ht(O.diff_h(z)) + O.diff_vt(O.diff_v(z)))
    np.testing.assert_allclose(back, rhs, atol=1e-10 * np.abs(rhs).max())


# ------------------------------------------------ brute-force minimisers

@pytest.mark.parametrize("k,p_missing,seed", [(3, 0.0, 10), (5, 0.0, 11), (3, 0.3, 12)])
def test_tv_md_reaches_bruteforce_minimum(k, p_missing, seed):
    H = W = 8
    y, m, h = small_problem(seed, H, W, k, p_missing)
    lam = 0.02
    A = dense_conv(h, H, W)
    Dh, Dv = dense_diffs(H, W)
    xe = newton_min(tv_smoothed(A, Dh, Dv, m.ravel(), y.ravel(), lam), np.zeros(H * W))
    F_eps = O.tv_objective(xe.reshape(H, W), y, m, h, lam)
    bound = lam * H * W * 1e-10             # 0 <= F(x_eps) - F* <= lam * n * eps
    out = O.tv_md_run(y, m, h, lam, 0.2, 0.1, iters=20000, tol=1e-13, check_every=50)
    F_admm = O.tv_objective(out["z"], y, m, h, lam)
    assert F_admm >= F_eps - bound - 1e-12 * F_eps
    assert F_admm - F_eps <= 1e-9 * F_eps + bound


@pytest.mark.parametrize("J,k,seed", [(1, 3, 20), (2, 3, 21)])
def test_fa_md_reaches_bruteforce_minimum(J, k, seed):
    H = W = 8
    y, m, h = small_problem(seed, H, W, k, 0.2)
    lam = 0.01
    A = dense_conv(h, H, W)
    n = H * W
    P = np.zeros(((3 * J + 1) * n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        P[:, j] = O.haar_analysis(e.reshape(H, W), J).ravel()
    xe = newton_min(fa_smoothed(A, P, m.ravel(), y.ravel(), lam), np.zeros(n))
    F_eps = O.fa_objective(xe.reshape(H, W), y, m, h, lam, J)
    bound = lam * P.shape[0] * 1e-10
    out = O.fa_md_run(y, m, h, lam, 0.2, 0.05, J, iters=20000, tol=1e-13, check_every=50)
    F_admm = O.fa_objective(out["z"], y, m, h, lam, J)
    assert F_admm >= F_eps - bound - 1e-12 * F_eps
    assert F_admm - F_eps <= 1e-9 * F_eps + bound


# ------------------------------------------------ lambda-large closed forms

def _lap_pinv(H, W):
    Dh, Dv = dense_diffs(H, W)
    return Dh, Dv, np.linalg.pinv(Dh.T @ Dh + Dv.T @ Dv)


def test_tv_large_lambda_gives_constant_and_small_lambda_does_not():
    H = W = 12
    y, m, h = small_problem(30, H, W, k=3, p_missing=0.2)
    beta = h.sum()
    c = y[m > 0].sum() / (beta * (m > 0).sum())
    g = O.conv_At(m * (y - beta * c), h).ravel()      # 1^T g = 0
    Dh, Dv, L = _lap_pinv(H, W)
    w = L @ g
    p = np.stack([Dh @ w, Dv @ w])
    lam_bar = np.sqrt((p ** 2).sum(axis=0)).max()      # sufficient: p / lam feasible
    const = np.full((H, W), c)
    # lambda above lam_bar: the constant image c 1 is the minimiser
    lam = 1.5 * lam_bar
    out = O.tv_md_run(y, m, h, lam, 0.5, 0.5, iters=6000)
    F_c = O.tv_objective(const, y, m, h, lam)
    assert abs(O.tv_objective(out["z"], y, m, h, lam) - F_c) <= 1e-9 * F_c
    assert np.abs(out["z"] - c).max() < 1e-4
    # necessary condition <g, w> <= lam TV(w) violated -> strictly better than c 1
    tvw = np.sqrt((Dh @ w) ** 2 + (Dv @ w) ** 2).sum()
    lam = 0.5 * (g @ w) / tvw
    out = O.tv_md_run(y, m, h, lam, 0.5, 0.5, iters=6000)
    F_c = O.tv_objective(const, y, m, h, lam)
    assert O.tv_objective(out["z"], y, m, h, lam) < F_c * (1 - 1e-3)


def test_fa_large_lambda_gives_zero_and_small_lambda_does_not():
    H = W = 8
    J = 2
    y, m, h = small_problem(31, H, W, k=3, p_missing=0.2)
    g = O.conv_At(m * y, h)
    lam_bar = np.abs(O.haar_analysis(g, J)).max()
    F0 = 0.5 * np.sum(y * y)
    lam = 1.5 * lam_bar
    out = O.fa_md_run(y, m, h, lam, 0.5, 0.5, J, iters=4000)
    assert np.abs(out["z"]).max() < 1e-6
    lam = 0.5 * np.sum(g * g) / np.abs(O.haar_analysis(g, J)).sum()
    out = O.fa_md_run(y, m, h, lam, 0.5, 0.5, J, iters=4000)
    assert O.fa_objective(out["z"], y, m, h, lam, J) < F0 * (1 - 1e-3)


# ------------------------------------------------ properties from Theorem 1

def test_limit_independent_of_mu_and_initialisation():
    H = W = 10
    y, m, h = small_problem(40, H, W, k=3, p_missing=0.1)
    lam = 0.02
    a = O.tv_md_run(y, m, h, lam, 0.2, 0.1, iters=20000, tol=1e-13, check_every=50)
    g = np.random.default_rng(41)
    st0 = O.TVState(*(g.standard_normal((H, W)) for _ in range(6)))
    b = O.tv_md_run(y, m, h, lam, 0.05, 0.3, iters=40000, state0=st0, tol=1e-13, check_every=50)
    Fa = O.tv_objective(a["z"], y, m, h, lam)
    Fb = O.tv_objective(b["z"], y, m, h, lam)
    assert abs(Fa - Fb) <= 1e-8 * Fa


def test_warm_start_at_the_solution_is_a_fixed_point():
    H = W = 10
    y, m, h = small_problem(42, H, W, k=3, p_missing=0.1)
    lam, mu1, mu2 = 0.02, 0.2, 0.1
    sol = O.tv_md_run(y, m, h, lam, mu1, mu2, iters=20000, tol=1e-14, check_every=50)
    st = sol["state"]
    ph, pv = -(mu2 / lam) * st.dh, -(mu2 / lam) * st.dv
    ws = O.warm_start_state(sol["z"], ph, pv, y, m, h, lam, mu1, mu2)
    nxt = O.tv_md_run(y, m, h, lam, mu1, mu2, iters=1, state0=ws)
    np.testing.assert_allclose(nxt["z"], sol["z"], atol=1e-8)


def test_off_mask_data_dual_vanishes():
    y, m, h = small_problem(43, 16, 16, k=5, p_missing=0.3)
    out = O.tv_md_run(y, m, h, 0.02, 0.1, 0.1, iters=7)
    d1 = out["state"].d1
    assert np.abs(d1[m == 0]).max() <= 1e-12 * np.abs(d1).max()


def test_default_mu_rule():
    assert O.default_mu(2e-4) == (1.0, 2e-3)
    mu1, mu2 = O.default_mu(1e-6)
    assert mu2 == pytest.approx(1e-5) and mu1 == pytest.approx(0.05)


# ------------------------------------------- pins catch planted mistakes

@pytest.mark.parametrize("mutation", ["dual_sign", "threshold", "prox_mu"])
def test_planted_mistake_is_caught_by_minimiser_pin(mutation, monkeypatch):
    H = W = 8
    y, m, h = small_problem(10, H, W, 3, 0.0)
    lam = 0.02
    A = dense_conv(h, H, W)
    Dh, Dv = dense_diffs(H, W)
    xe = newton_min(tv_smoothed(A, Dh, Dv, m.ravel(), y.ravel(), lam), np.zeros(H * W))
    F_eps = O.tv_objective(xe.reshape(H, W), y, m, h, lam)
    if mutation == "threshold":
        real = oadmm.vsoft
        monkeypatch.setattr(oadmm, "vsoft", lambda a, b, t: real(a, b, 3.0 * t))
    elif mutation == "prox_mu":
        real = oadmm.mask_prox
        monkeypatch.setattr(oadmm, "mask_prox", lambda v, yy, mm, mu: real(v, yy, mm, 2.0 * mu))
    else:
        def bad_step(st, y_, m_, h_, lam_, mu1, mu2, spectra):
            new, z, aux = _orig_step(st, y_, m_, h_, lam_, mu1, mu2, spectra)
            Az = aux[0]
            new.d1 = st.d1 + (Az - new.u1)       # wrong sign of the dual update
            return new, z, aux
        monkeypatch.setattr(oadmm, "tv_md_step", bad_step)
    with np.errstate(invalid="ignore", over="ignore"):   # the wrong dual sign diverges
        out = oadmm.tv_md_run(y, m, h, lam, 0.2, 0.1, iters=3000)
    F_bad = O.tv_objective(out["z"], y, m, h, lam) if np.all(np.isfinite(out["z"])) else np.inf
    assert not (F_bad - F_eps <= 1e-9 * F_eps + lam * H * W * 1e-10)


_orig_step = oadmm.tv_md_step
