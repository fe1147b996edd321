"""GPU parity of TV-CG and FA-CG (the Reeves-Sorel variants, Sec. IV-B..IV-D)
against the FP64 oracle (oracle/cg.py, pinned in tests/test_oracle_cg.py).

Bar, as for the MD solvers: per-iterate relative L2 error and largest element
error (over max |z|) of z_k <= 1e-4 after a fixed number of iterations from
the same cold start; residuals at check iterations within 1e-3 relative; the
device objective within 1e-4 of the FP64 objective of the FP32 iterate.
"""

import numpy as np
import pytest

import oracle as O
from paper_1210_2687_amd import admm as A
from paper_1210_2687_amd import workloads as WL
from gpu_util import dev, host, announce, check_iterate, full_problem, fast_tv_problem

pytestmark = pytest.mark.gpu

ITER_TOL = 1e-4
RES_TOL = 1e-3


def _oracle(p, ks):
    """z_k and (r_pri, r_dual) at the iterations ks of the oracle's CG run."""
    y, m, h = np.asarray(p.y, np.float64), p.mask.astype(np.float64), p.kernel
    H, W = y.shape
    ks = set(ks)
    zs, res = {}, {}
    if p.reg == "frame":
        Lam = O.kernel_spectrum(h, H, W)
        st = O.FACGState.zeros(H, W, p.levels)
        step = lambda s: O.fa_cg_step(s, y, m, h, p.lam, p.mu1, p.mu2, p.levels, Lam)
        resid = O.fa_residuals
    else:
        spectra = (O.kernel_spectrum(h, H, W), *O.diff_spectra(H, W))
        st = O.TVCGState.zeros(H, W)
        step = lambda s: O.tv_cg_step(s, y, m, h, p.lam, p.mu1, p.mu2, spectra)
        resid = O.tv_residuals
    for k in range(1, max(ks) + 1):
        new, z, aux = step(st)
        if k in ks:
            zs[k] = z
            res[k] = resid(aux, new, st, p.mu1, p.mu2)
        st = new
    return zs, res


def _objective(p, z):
    if p.reg == "frame":
        return O.fa_objective(z, p.y, p.mask, p.kernel, p.lam, p.levels)
    return O.tv_objective(z, p.y, p.mask, p.kernel, p.lam)


def _solve(plan, p, K, graph=False, tol=0.0, check_every=None):
    import torch
    y = dev(p.y)
    x = torch.zeros_like(y)
    info = plan.solve(y, x, None, max_iters=K, tol=tol, check_every=check_every or K, graph=graph)
    return host(x), info


def _check_run(p, ks, tiles=None):
    zs, res = _oracle(p, ks)
    with A.Plan([p], method=A.ADMM_METHOD_CG, tiles=tiles) as plan:
        for k in sorted(ks):
            z, info = _solve(plan, p, k)
            assert info["iters"] == k
            if k == 1:
                assert np.all(z == 0.0)          # u = d = v = 0: the first right-hand side vanishes
                continue
            check_iterate(z, zs[k], ITER_TOL, f"k={k}")
            rp, rd = res[k]
            ep, ed = abs(info["r_pri"] - rp) / rp, abs(info["r_dual"] - rd) / rd
            announce(f"  k={k}: r_pri {info['r_pri']:.4e} vs {rp:.4e}, r_dual {info['r_dual']:.4e} vs {rd:.4e}")
            assert ep <= RES_TOL and ed <= RES_TOL, (k, ep, ed)
            F = _objective(p, z)
            assert abs(info["objective"] - F) <= 1e-4 * F


@pytest.mark.parametrize("shape,k,family", [((96, 160), 7, "gaussian"), ((135, 189), 9, "motion"),
                                            ((125, 98), 5, "uniform")])
def test_tv_cg_parity(shape, k, family):
    announce(f"tv-cg parity {shape} k={k} {family}")
    p = full_problem(500 + k, *shape, k, family, missing=0.3, lam=2e-4, mu=0.01)
    _check_run(p, [1, 2, 10, 60])


@pytest.mark.parametrize("shape,J", [((96, 160), 2), ((120, 84), 3), ((64, 72), 1), ((48, 64), 4)])
def test_fa_cg_parity(shape, J):
    announce(f"fa-cg parity {shape} J={J}")
    p = full_problem(600 + J, *shape, 7, reg="frame", levels=J, mu=0.02)
    _check_run(p, [1, 2, 10, 60])


def test_tv_cg_parity_large_ragged_rows():
    # a middle size class of the row pass, several row and column tiles with
    # ragged tails (600 = 8 x 75 rows, 1000 columns: 501 half-spectrum columns)
    announce("tv-cg parity 600 x 1000")
    p = full_problem(511, 600, 1000, 13, missing=0.4, lam=2e-4, mu=0.01)
    _check_run(p, [2, 8])


@pytest.mark.parametrize("shape,reg", [((16384, 24), "tv"), ((24, 12000), "frame")])
def test_cg_parity_long_sides(shape, reg):
    # TV-CG with columns of 16384 (both circulant solves through the split
    # column transform) and FA-CG with rows of 12000 (the sixth row class in
    # both inverse row modes)
    announce(f"{reg}-cg parity {shape}")
    p = full_problem(512, *shape, 5, reg=reg, levels=2 if reg == "frame" else 0, missing=0.3, mu=0.02)
    _check_run(p, [2, 4])


def test_cg_tile_shapes_do_not_change_iterates():
    # the CG step length sums per row block in a fixed order: another tiling
    # changes the rounding of the sums, within the parity bar
    announce("tv-cg tile shapes")
    p = full_problem(512, 96, 128, 9)
    zs, _ = _oracle(p, [30])
    for tiles in ({"cols_per_block": 1, "rows_per_block": 2}, {"cols_per_block": 4, "rows_per_block": 8}):
        with A.Plan([p], method=A.ADMM_METHOD_CG, tiles=tiles) as plan:
            z, _ = _solve(plan, p, 30)
        check_iterate(z, zs[30], ITER_TOL, str(tiles))


def test_cg_ragged_batch_matches_oracle():
    # TV and FA problems of several sizes in one plan, each against its own oracle run
    import torch
    announce("cg ragged batch")
    probs = [full_problem(520, 96, 160, 7), full_problem(521, 64, 64, 5, "uniform"),
             full_problem(522, 80, 120, 7, reg="frame", levels=2, mu=0.02),
             full_problem(523, 135, 100, 9, "motion", missing=0.5)]
    K = 25
    with A.Plan(probs, method=A.ADMM_METHOD_CG) as plan:
        ys = [dev(p.y) for p in probs]
        xs = [torch.zeros_like(y) for y in ys]
        infos = plan.batch(ys, xs, max_iters=K, check_every=K)
        for i, p in enumerate(probs):
            zs, res = _oracle(p, [K])
            check_iterate(host(xs[i]), zs[K], ITER_TOL, f"member {i}")
            assert infos[i]["iters"] == K
            assert abs(infos[i]["r_pri"] - res[K][0]) <= RES_TOL * res[K][0]


def test_cg_graph_replay_matches_eager_launches():
    import torch
    announce("cg graph replay vs eager")
    p = full_problem(530, 96, 96, 9)
    q = full_problem(531, 64, 80, 5, reg="frame", levels=2, mu=0.02)
    for prob in (p, q):
        with A.Plan([prob], method=A.ADMM_METHOD_CG) as plan:
            z0, i0 = _solve(plan, prob, 90, check_every=10)
            for rep in range(3):
                torch.cuda.synchronize()
                zg, ig = _solve(plan, prob, 90, graph=True, check_every=10)
                assert np.array_equal(zg, z0), rep
                assert ig["objective"] == i0["objective"]


def test_cg_reaches_the_md_objective():
    # TV-CG and TV-MD minimise the same objective (eq. (48)); run to a tight
    # tolerance, both reach the same value
    announce("cg and md objectives at convergence")
    p = fast_tv_problem(9, 64, 80, 5)
    F = lambda z: O.tv_objective(z, p.y, p.mask, p.kernel, p.lam)
    with A.Plan([p]) as plan:
        zm, im = _solve(plan, p, 6000, tol=1e-5, check_every=10)
    with A.Plan([p], method=A.ADMM_METHOD_CG) as plan:
        zc, ic = _solve(plan, p, 6000, tol=1e-5, check_every=10)
    announce(f"  md iters {im['iters']} F {F(zm):.8e}; cg iters {ic['iters']} F {F(zc):.8e}")
    assert im["converged"] and ic["converged"]
    assert abs(F(zc) - F(zm)) <= 2e-5 * F(zm)


def test_cg_static_entry_point_matches_the_plan():
    import torch
    announce("cg static entry")
    p = full_problem(540, 96, 128, 7)
    with A.Plan([p], method=A.ADMM_METHOD_CG) as plan:
        z0, i0 = _solve(plan, p, 40)
    cp = A.make_problem(p.kernel, p.mask, p.lam, p.mu1, p.mu2, method=A.ADMM_METHOD_CG)
    y = dev(p.y)
    x = torch.zeros_like(y)
    info = A.admm_deconv_solve_static(cp, y, x, max_iters=40, check_every=40)
    torch.cuda.synchronize()
    assert np.array_equal(host(x), z0)
    assert info["objective"] == i0["objective"]


def test_cg_rejects_state_and_mixed_methods():
    announce("cg error paths")
    p = full_problem(550, 64, 64, 5)
    H, W = p.shape
    with A.Plan([p], method=A.ADMM_METHOD_CG) as plan:
        st = A.alloc_state(H, W)
        import torch
        y = dev(p.y)
        x = torch.zeros_like(y)
        with pytest.raises(A.AdmmError) as e:
            plan.solve(y, x, st, max_iters=5)
        assert e.value.status == A.ADMM_E_UNSUPPORTED
    a = A.make_problem(p.kernel, p.mask, p.lam, p.mu1, p.mu2, method=A.ADMM_METHOD_MD)
    b = A.make_problem(p.kernel, p.mask, p.lam, p.mu1, p.mu2, method=A.ADMM_METHOD_CG)
    with pytest.raises(A.AdmmError) as e:
        A.admm_deconv_plan([a, b])
    assert e.value.status == A.ADMM_E_UNSUPPORTED
