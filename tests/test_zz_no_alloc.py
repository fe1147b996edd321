"""The allocation-free solve against the planned solve, through the C ABI.

admm_deconv_solve_static plans one problem into the library's static device
workspace and solves it there. It runs the same kernels on the same tile
choices as admm_deconv_plan + admm_deconv_solve, so its iterates, infos and
states must equal theirs bit for bit, also when a call follows a larger one
whose contents the shared workspace still holds.
"""

import numpy as np
import pytest

from paper_1210_2687_amd import admm as A
from gpu_util import dev, host, announce, full_problem, fast_tv_problem

pytestmark = pytest.mark.gpu


def _cprob(p):
    reg = A.ADMM_REG_FRAME if p.reg == "frame" else A.ADMM_REG_TV
    return A.make_problem(p.kernel, p.mask, p.lam, p.mu1, p.mu2, reg, p.levels)


def _nreg(p):
    return 3 * p.levels + 1 if p.reg == "frame" else 2


def _planned(p, K, tol=0.0, c=10, state=None):
    import torch
    with A.Plan([p]) as plan:
        y = dev(p.y)
        x = torch.zeros_like(y)
        info = plan.solve(y, x, state, max_iters=K, tol=tol, check_every=c)
    return host(x), info


def _static(p, K, tol=0.0, c=10, state=None):
    import torch
    y = dev(p.y)
    x = torch.full_like(y, float("nan"))      # every output element must be written
    info = A.admm_deconv_solve_static(_cprob(p), y, x, state, max_iters=K, tol=tol, check_every=c,
                                      nreg=_nreg(p))
    torch.cuda.synchronize()
    return host(x), info


@pytest.mark.parametrize("reg", ["tv", "frame"])
def test_static_solve_equals_the_planned_solve_on_consecutive_calls(reg):
    # a larger problem, then a smaller one in the same workspace
    if reg == "tv":
        cases = [full_problem(501, 384, 320, 13), full_problem(502, 96, 80, 7, "motion")]
    else:
        cases = [full_problem(503, 256, 192, 9, reg="frame", levels=3),
                 full_problem(504, 64, 72, 5, "uniform", reg="frame", levels=2)]
    for p in cases:
        announce(f"static solve {reg} {p.shape}, 40 iterations")
        xs, i_s = _static(p, 40)
        xr, i_r = _planned(p, 40)
        assert np.array_equal(xs, xr)
        assert i_s == i_r


def test_static_tolerance_solve_and_resume():
    import torch
    p = fast_tv_problem(505, 72, 64, 7)
    announce("static solve to tolerance 1e-4, then 30 + 30 iterations through a state")
    xs, i_s = _static(p, 3000, tol=1e-4, c=10)
    xr, i_r = _planned(p, 3000, tol=1e-4, c=10)
    assert i_s["converged"] == 1 and i_s == i_r and np.array_equal(xs, xr)
    H, W = p.shape
    s_static, s_plan = A.alloc_state(H, W), A.alloc_state(H, W)
    _static(p, 30, state=s_static)
    x2s, _ = _static(p, 30, state=s_static)
    _planned(p, 30, state=s_plan)
    x2r, _ = _planned(p, 30, state=s_plan)
    assert np.array_equal(x2s, x2r)
    for key in s_static:
        assert torch.equal(s_static[key], s_plan[key]), key


def test_static_solve_rejects_a_problem_beyond_its_workspace():
    import torch
    p = fast_tv_problem(506, 1024, 1024, 7)          # about 64 MB of workspace
    y = dev(p.y)
    x = torch.zeros_like(y)
    with pytest.raises(A.AdmmError) as e:
        A.admm_deconv_solve_static(_cprob(p), y, x, max_iters=5)
    assert e.value.status == A.ADMM_E_UNSUPPORTED
    assert "at most" in str(e.value)
    # and the next call in range still works
    q = full_problem(507, 64, 64, 5)
    xs, _ = _static(q, 12)
    xr, _ = _planned(q, 12)
    assert np.array_equal(xs, xr)
