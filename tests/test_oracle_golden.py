"""The oracle against exact / 60-digit trajectories of tiny TV-MD and FA-MD problems.

The fixtures in tests/golden were written by tests/golden/make_golden.py from
dense explicit operator matrices and dense linear solves, in exact rational
(FA-MD) or 60-digit decimal (TV-MD) arithmetic: none of the oracle's code, no
FFT, no spectral diagonalisation and no use of the frame's Parseval property.
Agreement of every recorded iterate to ~1e-12 pins the oracle's whole
iteration (right-hand side, z-step, data step, both proximity operators and
both dual updates, in order) and its objective, not only its fixed point.
"""

import importlib.util
import os

import numpy as np
import pytest

import oracle as O
import oracle.admm as oadmm
from golden_fixtures import GOLDEN, NAMES, load

TOL = 1e-12


def _oracle_run(g, record):
    if g["reg"] == "tv":
        return O.tv_md_run(g["y"], g["mask"], g["kernel"], g["lambda"], g["mu1"], g["mu2"],
                           iters=g["iters"], record=record)
    return O.fa_md_run(g["y"], g["mask"], g["kernel"], g["lambda"], g["mu1"], g["mu2"], g["levels"],
                       iters=g["iters"], record=record)


@pytest.mark.parametrize("name", NAMES)
def test_oracle_iterates_match_exact_trajectory(name):
    g = load(name)
    res = _oracle_run(g, tuple(g["zs"]))
    for k, zk in g["zs"].items():
        err = np.max(np.abs(res["zs"][k] - zk))
        assert err <= TOL * max(1.0, np.max(np.abs(zk))), (name, k, err)
    k_obj, f_ref = g["objective"]
    assert k_obj == g["iters"]
    if g["reg"] == "tv":
        f = O.tv_objective(res["z"], g["y"], g["mask"], g["kernel"], g["lambda"])
    else:
        f = O.fa_objective(res["z"], g["y"], g["mask"], g["kernel"], g["lambda"], g["levels"])
    assert abs(f - f_ref) <= TOL * abs(f_ref)


def test_fixtures_exercise_both_threshold_branches():
    # a pin is only as strong as the branches it visits: along every fixture's
    # trajectory some coefficients are shrunk to zero and others survive, with
    # margins far above FP64 rounding (so both sides take the same branches)
    for name in NAMES:
        g = load(name)
        y, m, h, lam, mu1, mu2 = g["y"], g["mask"], g["kernel"], g["lambda"], g["mu1"], g["mu2"]
        H, W = g["shape"]
        tau = lam / mu2
        shrunk = kept = 0
        margin = np.inf
        if g["reg"] == "tv":
            spectra = (O.kernel_spectrum(h, H, W), *O.diff_spectra(H, W))
            st = O.TVState.zeros(H, W)
            for _ in range(g["iters"]):
                new, z, (_, zh, zv) = O.tv_md_step(st, y, m, h, lam, mu1, mu2, spectra)
                rho = np.hypot(zh - st.dh, zv - st.dv)
                st = new
                shrunk, kept = shrunk + np.sum(rho <= tau), kept + np.sum(rho > tau)
                margin = min(margin, np.min(np.abs(rho - tau)))
        else:
            Lam = O.kernel_spectrum(h, H, W)
            st = O.FAState.zeros(H, W, g["levels"])
            for _ in range(g["iters"]):
                new, z, (_, Pz) = O.fa_md_step(st, y, m, h, lam, mu1, mu2, g["levels"], Lam)
                v = np.abs(Pz - st.d2)
                st = new
                shrunk, kept = shrunk + np.sum(v <= tau), kept + np.sum(v > tau)
                margin = min(margin, np.min(np.abs(v - tau)))
        assert shrunk > 0 and kept > 0, name
        assert margin > 1e-6, (name, margin)


def test_small_fixtures_regenerate_identically():
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(GOLDEN, "make_golden.py"))
    G = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(G)
    for make in (G._tv_problem, G._fa_problem):
        pb = make()
        zs, obj, res = G.run(pb)
        g = load(pb["name"])
        assert sorted(zs) == sorted(g["zs"])
        for k in zs:
            fresh = np.array([float(G._dec(v)) for v in zs[k]]).reshape(g["shape"])
            assert np.array_equal(fresh, g["zs"][k])
        assert float(G._dec(obj)) == g["objective"][1]
        assert sorted(res) == sorted(g["residuals"])
        for k, (rp, rd) in res.items():
            assert (float(G._dec(rp)), float(G._dec(rd))) == g["residuals"][k]


# ------------------------------------------- the residuals of the stopping rule

def _oracle_history(g):
    """(r_pri, r_dual) of every iteration (a negative tolerance never stops the run)."""
    if g["reg"] == "tv":
        out = O.tv_md_run(g["y"], g["mask"], g["kernel"], g["lambda"], g["mu1"], g["mu2"],
                          iters=g["iters"], tol=-1.0, check_every=1)
    else:
        out = O.fa_md_run(g["y"], g["mask"], g["kernel"], g["lambda"], g["mu1"], g["mu2"], g["levels"],
                          iters=g["iters"], tol=-1.0, check_every=1)
    return {k: (rp, rd) for k, rp, rd in out["history"]}


def _residual_err(g):
    hist = _oracle_history(g)
    return max(max(abs(hist[k][0] - rp) / rp, abs(hist[k][1] - rd) / rd)
               for k, (rp, rd) in g["residuals"].items())


@pytest.mark.parametrize("name", NAMES)
def test_oracle_residuals_match_exact_values(name):
    # tv_residuals / fa_residuals against r_pri and r_dual computed from their
    # definitions on the exact state (u_k, u_{k-1}, d_k, G z_k) at k = 2, 3, 5, 8
    g = load(name)
    assert sorted(g["residuals"]) == [2, 3, 5, 8]
    assert _residual_err(g) <= TOL


_tv_res = oadmm.tv_residuals
_fa_res = oadmm.fa_residuals


def _tv_res_dropped_block(aux, st, sp, mu1, mu2):
    # primal residual without the TV block
    Az, zh, zv = aux
    rp, rd = _tv_res(aux, st, sp, mu1, mu2)
    pri = np.sqrt(np.sum((Az - st.u1) ** 2))
    den = max(np.sqrt(np.sum(Az ** 2) + np.sum(zh ** 2) + np.sum(zv ** 2)),
              np.sqrt(np.sum(st.u1 ** 2) + np.sum(st.uh ** 2) + np.sum(st.uv ** 2)))
    return pri / den, rd


def _mu_not_squared(res):
    # Upsilon applied as sqrt(Upsilon): the dual residual weighs the blocks by mu, not mu^2
    return lambda aux, st, sp, mu1, mu2: (res(aux, st, sp, mu1, mu2)[0],
                                          res(aux, st, sp, np.sqrt(mu1), np.sqrt(mu2))[1])


def _tv_res_previous_dual(aux, st, sp, mu1, mu2):
    # the dual residual normalised by d_{k-1} instead of d_k
    rp, rd = _tv_res(aux, st, sp, mu1, mu2)
    dn_k = np.sqrt(mu1 ** 2 * np.sum(st.d1 ** 2) + mu2 ** 2 * (np.sum(st.dh ** 2) + np.sum(st.dv ** 2)))
    dn_p = np.sqrt(mu1 ** 2 * np.sum(sp.d1 ** 2) + mu2 ** 2 * (np.sum(sp.dh ** 2) + np.sum(sp.dv ** 2)))
    return rp, rd * dn_k / max(dn_p, 1e-30)


def _fa_res_dropped_frame(aux, st, sp, mu1, mu2):
    Az, Pz = aux
    rp, rd = _fa_res(aux, st, sp, mu1, mu2)
    pri = np.sqrt(np.sum((Az - st.u1) ** 2))
    den = max(np.sqrt(np.sum(Az ** 2) + np.sum(Pz ** 2)), np.sqrt(np.sum(st.u1 ** 2) + np.sum(st.u2 ** 2)))
    return pri / den, rd


def _fa_res_no_coarse_band(aux, st, sp, mu1, mu2):
    # the coarsest band left out of the dual residual
    Az, Pz = aux
    rp, _ = _fa_res(aux, st, sp, mu1, mu2)
    dual = np.sqrt(mu1 ** 2 * np.sum((st.u1 - sp.u1) ** 2) + mu2 ** 2 * np.sum((st.u2[:-1] - sp.u2[:-1]) ** 2))
    dn = np.sqrt(mu1 ** 2 * np.sum(st.d1 ** 2) + mu2 ** 2 * np.sum(st.d2 ** 2))
    return rp, dual / dn


@pytest.mark.parametrize("mutation", ["tv_dropped_block", "tv_mu_not_squared", "tv_previous_dual",
                                      "fa_dropped_frame", "fa_mu_not_squared", "fa_no_coarse_band"])
def test_planted_residual_mistake_is_caught(mutation, monkeypatch):
    if mutation.startswith("tv"):
        fn = {"tv_dropped_block": _tv_res_dropped_block, "tv_mu_not_squared": _mu_not_squared(_tv_res),
              "tv_previous_dual": _tv_res_previous_dual}[mutation]
        monkeypatch.setattr(oadmm, "tv_residuals", fn)
        names = ("tv_md_5x6", "tv_md_8x10")
    else:
        fn = {"fa_dropped_frame": _fa_res_dropped_frame, "fa_mu_not_squared": _mu_not_squared(_fa_res),
              "fa_no_coarse_band": _fa_res_no_coarse_band}[mutation]
        monkeypatch.setattr(oadmm, "fa_residuals", fn)
        names = ("fa_md_4x6_J2", "fa_md_8x8_J3")
    assert all(_residual_err(load(n)) > 1e-4 for n in names)


# ------------------------------------------- the pins catch planted mistakes

_tv_step = oadmm.tv_md_step
_soft = oadmm.soft
_zsolve_fa = oadmm.zsolve_fa


def _max_err(g, kernel=None):
    if kernel is not None:
        g = dict(g, kernel=kernel)
    res = _oracle_run(g, tuple(g["zs"]))
    return max(np.max(np.abs(res["zs"][k] - zk)) for k, zk in g["zs"].items())


@pytest.mark.parametrize("mutation", ["relaxed_dual", "transposed_kernel_tv", "transposed_kernel_fa",
                                      "coarse_band_unthresholded", "zstep_gamma"])
def test_planted_mistake_is_caught_by_golden_trajectory(mutation, monkeypatch):
    # relaxed_dual keeps the fixed point (an over-relaxed dual step of the same
    # ADMM converges to the same minimiser), so only a trajectory pin sees it
    kernel = None
    if mutation == "relaxed_dual":
        g = load("tv_md_5x6")

        def step(st, *a):
            new, z, aux = _tv_step(st, *a)
            new.d1 = st.d1 - 1.5 * (aux[0] - new.u1)
            return new, z, aux
        monkeypatch.setattr(oadmm, "tv_md_step", step)
    elif mutation == "transposed_kernel_tv":
        g = load("tv_md_8x10")
        kernel = g["kernel"].T.copy()
    elif mutation == "transposed_kernel_fa":
        g = load("fa_md_8x8_J3")
        kernel = g["kernel"].T.copy()
    elif mutation == "coarse_band_unthresholded":
        g = load("fa_md_4x6_J2")
        monkeypatch.setattr(oadmm, "soft", lambda v, t: np.concatenate([_soft(v[:-1], t), v[-1:]]))
    else:
        g = load("fa_md_8x8_J3")
        monkeypatch.setattr(oadmm, "zsolve_fa", lambda rhs, Lam, gm: _zsolve_fa(rhs, Lam, 1.0 / gm))
    assert _max_err(g, kernel) > 1e-6
