"""Pins of the FP64 oracle's TV-CG and FA-CG (the Reeves-Sorel variants, Sec. IV-B..IV-D).

* the Sherman-Morrison-Woodbury split of eqs. (43), (47), (51) against a
  dense inverse on 8 x 8 problems;
* the z-step with the boundary system solved to convergence against the
  dense solve of the non-circulant system, and one CG iteration written out
  on the dense matrices;
* whole trajectories against tests/golden (dense matrices, exact rational
  FA-CG and 60-digit TV-CG, no FFT), with planted mistakes;
* the limit: TV-CG / FA-CG minimise the same objective as TV-MD / FA-MD, so
  run to convergence they reach the same objective value (the MD limit is
  pinned to brute-force minimisers in tests/test_oracle_admm.py).
"""

import numpy as np
import pytest

import oracle as O
import oracle.cg as ocg
from golden_fixtures import CG_NAMES, load
from test_oracle_admm import dense_conv, dense_diffs, small_problem

TOL = 1e-12


def _dense_haar(H, W, J):
    n = H * W
    P = np.zeros(((3 * J + 1) * n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        P[:, i] = O.haar_analysis(e.reshape(H, W), J).ravel()
    return P


def _dense_setup(seed, reg, k=3, p_missing=0.25):
    H = W = 8
    y, m, h = small_problem(seed, H=H, W=W, k=k, p_missing=p_missing)
    A = dense_conv(h, H, W)
    mb = (1.0 - m).ravel()
    B = A[mb > 0]                                   # rows of A at the unobserved pixels
    if reg == "tv":
        Dh, Dv = dense_diffs(H, W)
        R2 = Dh.T @ Dh + Dv.T @ Dv
        spectra = (O.kernel_spectrum(h, H, W), *O.diff_spectra(H, W))
        den = lambda g: np.abs(spectra[0]) ** 2 + g * (np.abs(spectra[1]) ** 2 + np.abs(spectra[2]) ** 2)
    else:
        R2 = np.eye(H * W)                         # P^T P = I
        Lam = O.kernel_spectrum(h, H, W)
        den = lambda g: np.abs(Lam) ** 2 + g
    return y, m, h, A, B, R2, den


@pytest.mark.parametrize("reg", ["tv", "fa"])
def test_smw_split_equals_the_dense_inverse(reg):
    y, m, h, A, B, R2, _ = _dense_setup(3, reg)
    gamma = 0.4
    C = np.linalg.inv(A.T @ A + gamma * R2)
    I = np.eye(B.shape[0])
    K = C - C @ B.T @ np.linalg.solve(B @ C @ B.T - I, B @ C)
    Mv = np.diag(m.ravel())
    direct = np.linalg.inv(A.T @ Mv @ A + gamma * R2)
    np.testing.assert_allclose(K, direct, rtol=0, atol=1e-9 * np.abs(direct).max())
    # the boundary system I - B C B^T is symmetric positive definite
    S = I - B @ C @ B.T
    assert np.allclose(S, S.T) and np.linalg.eigvalsh(S).min() > 0


@pytest.mark.parametrize("reg", ["tv", "fa"])
def test_zstep_with_converged_cg_is_the_dense_solve(reg):
    y, m, h, A, B, R2, den = _dense_setup(5, reg, k=5, p_missing=0.3)
    gamma = 0.7
    g = np.random.default_rng(5)
    r = g.standard_normal((8, 8))
    v0 = (1.0 - m) * g.standard_normal((8, 8))
    z, v = O.cg_zsolve(r, v0, m, h, den(gamma), cg_iters=400)
    Mv = np.diag(m.ravel())
    exact = np.linalg.solve(A.T @ Mv @ A + gamma * R2, r.ravel())
    np.testing.assert_allclose(z.ravel(), exact, rtol=0, atol=1e-9 * np.abs(exact).max())
    assert np.all(v[m > 0] == 0.0)


@pytest.mark.parametrize("reg", ["tv", "fa"])
def test_one_cg_step_on_the_dense_matrices(reg):
    y, m, h, A, B, R2, den = _dense_setup(7, reg)
    gamma = 0.3
    g = np.random.default_rng(7)
    r = g.standard_normal((8, 8))
    obs = (1.0 - m).ravel() > 0
    v0 = np.zeros(64)
    v0[obs] = g.standard_normal(obs.sum())
    z, v = O.cg_zsolve(r, v0.reshape(8, 8), m, h, den(gamma), cg_iters=1)
    C = np.linalg.inv(A.T @ A + gamma * R2)
    S = np.eye(B.shape[0]) - B @ C @ B.T
    t = C @ r.ravel()
    w0 = v0[obs]
    res = B @ t - S @ w0
    a = (res @ res) / (res @ S @ res)
    w1 = w0 + a * res
    np.testing.assert_allclose(v.ravel()[obs], w1, rtol=0, atol=1e-11 * np.abs(w1).max())
    np.testing.assert_allclose(z.ravel(), t + C @ B.T @ w1, rtol=0, atol=1e-11 * np.abs(t).max())


def _cg_run(g, record=(), iters=None, step=None):
    kw = dict(iters=iters or g["iters"], record=record)
    if g["reg"] == "tv":
        return O.tv_cg_run(g["y"], g["mask"], g["kernel"], g["lambda"], g["mu1"], g["mu2"], **kw)
    return O.fa_cg_run(g["y"], g["mask"], g["kernel"], g["lambda"], g["mu1"], g["mu2"], g["levels"], **kw)


def _residual_history(g):
    """(r_pri, r_dual) with the data block M A z - u1, by the oracle's residual
    functions (which take the data block's forward image as given)."""
    y, m, h, lam, mu1, mu2 = g["y"], g["mask"].astype(np.float64), g["kernel"], g["lambda"], g["mu1"], g["mu2"]
    H, W = g["shape"]
    out = {}
    if g["reg"] == "tv":
        spectra = (O.kernel_spectrum(h, H, W), *O.diff_spectra(H, W))
        st = O.TVCGState.zeros(H, W)
        for k in range(1, g["iters"] + 1):
            new, z, aux = O.tv_cg_step(st, y, m, h, lam, mu1, mu2, spectra)
            out[k] = O.tv_residuals(aux, new, st, mu1, mu2)
            st = new
    else:
        Lam = O.kernel_spectrum(h, H, W)
        st = O.FACGState.zeros(H, W, g["levels"])
        for k in range(1, g["iters"] + 1):
            new, z, aux = O.fa_cg_step(st, y, m, h, lam, mu1, mu2, g["levels"], Lam)
            out[k] = O.fa_residuals(aux, new, st, mu1, mu2)
            st = new
    return out


@pytest.mark.parametrize("name", CG_NAMES)
def test_cg_oracle_matches_exact_trajectory(name):
    g = load(name)
    assert g["method"] == "cg"
    res = _cg_run(g, record=tuple(g["zs"]))
    assert np.all(res["zs"][1] == 0.0)
    for k, zk in g["zs"].items():
        err = np.max(np.abs(res["zs"][k] - zk))
        assert err <= TOL * max(1.0, np.max(np.abs(zk))), (name, k, err)
    f = (O.tv_objective(res["z"], g["y"], g["mask"], g["kernel"], g["lambda"]) if g["reg"] == "tv" else
         O.fa_objective(res["z"], g["y"], g["mask"], g["kernel"], g["lambda"], g["levels"]))
    assert abs(f - g["objective"][1]) <= TOL * abs(g["objective"][1])
    hist = _residual_history(g)
    for k, (rp, rd) in g["residuals"].items():
        assert abs(hist[k][0] - rp) <= TOL * rp and abs(hist[k][1] - rd) <= TOL * rd, (name, k)


_cg_zsolve = ocg.cg_zsolve


@pytest.mark.parametrize("mutation", ["no_warm_start", "plus_identity", "no_boundary_term", "mu_scale"])
def test_planted_cg_mistake_is_caught(mutation, monkeypatch):
    if mutation == "no_warm_start":          # every CG run from zero instead of the previous estimate
        monkeypatch.setattr(ocg, "cg_zsolve", lambda r, v0, m, h, den, it=1: _cg_zsolve(r, 0 * v0, m, h, den, it))
    elif mutation == "plus_identity":       # (B C B^T + I) in place of (B C B^T - I)
        def wrong(r, v0, m, h, den, it=1):
            C = ocg._circulant_inverse(den)
            mb = 1.0 - m
            B = lambda x: mb * O.conv_A(x, h)
            Bt = lambda w: O.conv_At(mb * w, h)
            t = C(r)
            v = ocg.boundary_cg(B(t), v0, lambda w: w + B(C(Bt(w))), it)
            return t - C(Bt(v)), v
        monkeypatch.setattr(ocg, "cg_zsolve", wrong)
    elif mutation == "no_boundary_term":    # the circulant C alone (the periodic model's z-step)
        monkeypatch.setattr(ocg, "cg_zsolve", lambda r, v0, m, h, den, it=1: (ocg._circulant_inverse(den)(r), v0))
    else:                                   # TV without the 1 / mu1 of eq. (51): only caught on TV
        monkeypatch.setattr(ocg, "cg_zsolve", lambda r, v0, m, h, den, it=1: _cg_zsolve(r * 2.0, v0, m, h, den, it))
    for name in CG_NAMES:
        g = load(name)
        res = _cg_run(g, record=tuple(g["zs"]))
        err = max(np.max(np.abs(res["zs"][k] - zk)) for k, zk in g["zs"].items())
        assert err > 1e-6, (mutation, name, err)


@pytest.mark.parametrize("reg", ["tv", "fa"])
def test_cg_limit_is_the_md_limit(reg):
    # same objective (eqs. (44), (48)): run to convergence, equal objective values
    y, m, h = small_problem(11, H=12, W=10, k=3, p_missing=0.2)
    lam, mu1, mu2 = 0.02, 0.5, 0.25
    K = 6000
    if reg == "tv":
        cg = O.tv_cg_run(y, m, h, lam, mu1, mu2, iters=K)["z"]
        md = O.tv_md_run(y, m, h, lam, mu1, mu2, iters=K)["z"]
        F = lambda x: O.tv_objective(x, y, m, h, lam)
    else:
        cg = O.fa_cg_run(y, m, h, lam, mu1, mu2, 2, iters=K)["z"]
        md = O.fa_md_run(y, m, h, lam, mu1, mu2, 2, iters=K)["z"]
        F = lambda x: O.fa_objective(x, y, m, h, lam, 2)
    assert abs(F(cg) - F(md)) <= 1e-9 * F(md), (F(cg), F(md))
