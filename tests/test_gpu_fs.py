"""GPU parity of FS-MD (frame synthesis with mask decoupling, Sec. IV-C)
against the FP64 oracle (oracle/fs.py, pinned in tests/test_oracle_fs.py).

The library returns the image x_k = W z_k; the bar is the MD solvers' one:
relative L2 error and largest element error (over max |x|) <= 1e-4 after a
fixed number of iterations from the same start, residuals within 1e-3
relative, the device objective of eq. (35) within 1e-4 of the oracle's.
"""

import numpy as np
import pytest

import oracle as O
from paper_1210_2687_amd import admm as A
from gpu_util import dev, host, announce, check_iterate, full_problem, gpu_solve

pytestmark = pytest.mark.gpu

ITER_TOL = 1e-4
RES_TOL = 1e-3


def _fs_problem(seed, H, W, J, k=7, **kw):
    p = full_problem(seed, H, W, k, reg="frame", levels=J, **kw)
    p.reg = "synthesis"
    return p


def _oracle(p, ks):
    """x_k = W z_k, (r_pri, r_dual) and F(z_k) at the iterations ks."""
    y, m, h = np.asarray(p.y, np.float64), p.mask.astype(np.float64), p.kernel
    H, W = y.shape
    Lam = O.kernel_spectrum(h, H, W)
    st = O.FSState.zeros(H, W, p.levels)
    xs, res, obj = {}, {}, {}
    for k in range(1, max(ks) + 1):
        new, z, aux = O.fs_md_step(st, y, m, h, p.lam, p.mu1, p.mu2, p.levels, Lam)
        if k in ks:
            xs[k] = O.haar_synthesis(z, p.levels)
            res[k] = O.fs_residuals(aux, new, st, p.mu1, p.mu2)
            obj[k] = O.fs_objective(z, p.y, p.mask, p.kernel, p.lam, p.levels)
        st = new
    return xs, res, obj, st


def _check(p, ks):
    xs, res, obj, _ = _oracle(p, set(ks))
    with A.Plan([p]) as plan:
        for k in sorted(ks):
            x, info = gpu_solve(plan, p, k, check_every=k)
            assert info["iters"] == k
            if k == 1:
                assert np.all(x == 0.0)          # zeta = 0: the first z and x vanish
                continue
            check_iterate(x, xs[k], ITER_TOL, f"k={k}")
            rp, rd = res[k]
            ep, ed = abs(info["r_pri"] - rp) / rp, abs(info["r_dual"] - rd) / rd
            announce(f"  k={k}: r_pri {info['r_pri']:.4e} vs {rp:.4e}, r_dual {info['r_dual']:.4e} vs {rd:.4e}, "
                     f"F {info['objective']:.6e} vs {obj[k]:.6e}")
            assert ep <= RES_TOL and ed <= RES_TOL, (k, ep, ed)
            assert abs(info["objective"] - obj[k]) <= 1e-4 * obj[k]


@pytest.mark.parametrize("shape,J", [((96, 160), 2), ((120, 84), 3), ((64, 72), 1), ((48, 64), 4), ((40, 36), 3)])
def test_fs_parity(shape, J):
    announce(f"fs parity {shape} J={J}")
    _check(_fs_problem(700 + J, *shape, J, mu=0.02), [1, 2, 10, 60])


def test_fs_parity_large():
    # several row and column tiles with ragged tails, a middle row size class
    announce("fs parity 600 x 1000 J=3")
    _check(_fs_problem(711, 600, 1000, 3, k=13, missing=0.4, mu=0.01), [2, 6])


@pytest.mark.parametrize("shape", [(24, 6000), (10125, 24)])
def test_fs_parity_long_sides(shape):
    # rows of 6000 (the fifth row class, stage table read through the caches)
    # and columns of 10125 (split into three sub-transforms of 3375 around a
    # radix-3 pass through HBM)
    announce(f"fs parity {shape} J=2")
    _check(_fs_problem(712, *shape, 2, k=5, mu=0.02), [2, 5])


def test_fs_state_export_and_bitwise_resume():
    import torch
    announce("fs state export / resume")
    p = _fs_problem(720, 64, 80, 2, mu=0.02)
    H, W = p.shape
    nb = 3 * p.levels + 1
    with A.Plan([p]) as plan:
        s1 = A.alloc_state(H, W, nreg=nb)
        x30, _ = gpu_solve(plan, p, 30, state=s1)
        s2 = A.alloc_state(H, W, nreg=nb)
        gpu_solve(plan, p, 12, state=s2)
        x30b, _ = gpu_solve(plan, p, 18, state=s2)
    assert np.array_equal(x30, x30b)
    for key in ("u1", "d1", "ureg", "dreg"):
        assert torch.equal(s1[key], s2[key]), key
    _, _, _, ref = _oracle(p, {30})
    for key, val in (("u1", ref.u1), ("d1", ref.d1), ("ureg", ref.u2), ("dreg", ref.d2)):
        e = np.linalg.norm(host(s1[key]) - val) / np.linalg.norm(val)
        announce(f"  state {key}: rel {e:.2e}")
        assert e <= 1e-3, key


def test_fs_graph_replay_and_tolerance_stop():
    import torch
    announce("fs graph replay and residual stop")
    p = _fs_problem(730, 64, 64, 2, k=5, mu=0.005, lam=2e-3, missing=0.2)   # converges in about 1500 iterations
    tol, c = 1e-4, 10
    ref = O.fs_md_run(p.y, p.mask, p.kernel, p.lam, p.mu1, p.mu2, p.levels, iters=4000, tol=tol, check_every=c)
    assert ref["converged"]
    with A.Plan([p]) as plan:
        x0, i0 = gpu_solve(plan, p, 4000, tol=tol, check_every=c)
        for rep in range(2):
            torch.cuda.synchronize()
            x1, i1 = gpu_solve(plan, p, 4000, tol=tol, check_every=c, graph=True)
            assert i1["iters"] == i0["iters"] and np.array_equal(x0, x1), rep
    announce(f"  gpu stops at {i0['iters']}, oracle at {ref['iters']}")
    assert i0["converged"] == 1 and abs(i0["iters"] - ref["iters"]) <= c
    # the converged images agree closely (the coefficient minimiser need not be unique)
    check_iterate(x0, ref["x"], 2e-3, "converged image")


def test_fs_in_a_mixed_batch():
    # TV, FA and FS problems in one plan, each against its own oracle
    import torch
    announce("mixed TV / FA / FS batch")
    tv = full_problem(740, 96, 128, 7)
    fa = full_problem(741, 80, 120, 7, reg="frame", levels=2, mu=0.02)
    fs = _fs_problem(742, 72, 96, 3, mu=0.02)
    K = 20
    with A.Plan([tv, fa, fs]) as plan:
        ys = [dev(p.y) for p in (tv, fa, fs)]
        xs = [torch.zeros_like(y) for y in ys]
        infos = plan.batch(ys, xs, max_iters=K, check_every=K)
    ref_tv = O.tv_md_run(tv.y, tv.mask, tv.kernel, tv.lam, tv.mu1, tv.mu2, iters=K)["z"]
    ref_fa = O.fa_md_run(fa.y, fa.mask, fa.kernel, fa.lam, fa.mu1, fa.mu2, fa.levels, iters=K)["z"]
    ref_fs, _, obj, _ = _oracle(fs, {K})
    check_iterate(host(xs[0]), ref_tv, ITER_TOL, "tv member")
    check_iterate(host(xs[1]), ref_fa, ITER_TOL, "fa member")
    check_iterate(host(xs[2]), ref_fs[K], ITER_TOL, "fs member")
    assert abs(infos[2]["objective"] - obj[K]) <= 1e-4 * obj[K]


def test_fs_static_entry_point_matches_the_plan():
    import torch
    announce("fs static entry")
    p = _fs_problem(750, 64, 96, 2, mu=0.02)
    with A.Plan([p]) as plan:
        x0, i0 = gpu_solve(plan, p, 25, check_every=25)
    cp = A.make_problem(p.kernel, p.mask, p.lam, p.mu1, p.mu2, reg=A.ADMM_REG_FRAME_SYNTHESIS, levels=p.levels)
    y = dev(p.y)
    x = torch.zeros_like(y)
    info = A.admm_deconv_solve_static(cp, y, x, max_iters=25, check_every=25, nreg=3 * p.levels + 1)
    torch.cuda.synchronize()
    assert np.array_equal(host(x), x0)
    assert info["objective"] == i0["objective"]
