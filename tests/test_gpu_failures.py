"""Failure detection on the GPU path: divergence, allocation failure, budgets.

By Theorem 1 the iterates stay bounded whenever a solution exists, so a
non-finite value can only come from non-finite inputs; the library flags it
per problem (info.diverged) at the next check iteration and returns
ADMM_E_DIVERGED, while the other problems of the batch run on unaffected.
NaN arithmetic is ordinary arithmetic on the GPU: no kernel indexes memory
with a value it computes, so these tests drive no out-of-bounds access.
"""

import numpy as np
import pytest

from paper_1210_2687_amd import admm as A
from gpu_util import dev, host, announce, fast_tv_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("graph", [False, True])
def test_nan_state_diverges_alone(graph):
    import torch
    announce(f"NaN initial state in one problem of a batch (graph={graph})")
    probs = [fast_tv_problem(s, 64, 64 + 8 * s, 7) for s in range(3)]
    with A.Plan(probs) as plan:
        ys = [dev(p.y) for p in probs]

        def run(bad):
            xs = [torch.zeros_like(y) for y in ys]
            sts = [A.alloc_state(*p.shape) for p in probs]
            if bad is not None:
                sts[bad]["u1"][3, 5] = float("nan")
            infos = plan.batch(ys, xs, sts, max_iters=2000, tol=1e-4, check_every=10, graph=graph,
                               raise_on_diverged=False)
            torch.cuda.synchronize()
            return [host(x) for x in xs], infos

        x0, i0 = run(None)
        assert all(i["converged"] == 1 and i["diverged"] == 0 for i in i0)
        x1, i1 = run(1)
        announce(f"  infos: {[(i['iters'], i['converged'], i['diverged']) for i in i1]}")
        assert i1[1]["diverged"] == 1 and i1[1]["converged"] == 0 and i1[1]["iters"] == 10
        for j in (0, 2):
            assert i1[j] == i0[j]
            assert np.array_equal(x1[j], x0[j])
        # the status of the call says so
        with pytest.raises(A.AdmmError) as e:
            xs = [torch.zeros_like(y) for y in ys]
            sts = [A.alloc_state(*p.shape) for p in probs]
            sts[1]["dreg"][0, 1, 1] = float("inf")
            plan.batch(ys, xs, sts, max_iters=40, tol=1e-4, check_every=10, graph=graph)
        assert e.value.status == A.ADMM_E_DIVERGED


def test_nan_observation_without_tolerance_is_caught_at_the_last_iteration():
    import torch
    announce("NaN in an observed pixel, fixed iteration count")
    p = fast_tv_problem(11)
    y = p.y.copy()
    r, c = np.argwhere(p.mask == 1)[7]
    y[r, c] = np.nan
    with A.Plan([p]) as plan:
        yd = dev(y)
        x = torch.zeros_like(yd)
        with pytest.raises(A.AdmmError) as e:
            plan.solve(yd, x, max_iters=25)
        assert e.value.status == A.ADMM_E_DIVERGED
        # the same plan still solves a finite problem afterwards
        info = plan.solve(dev(p.y), x, max_iters=25)
        assert info["diverged"] == 0 and np.all(np.isfinite(host(x)))


def test_allocation_failure_reports_nomem_and_leaves_the_library_usable():
    import torch
    free, total = torch.cuda.mem_get_info()
    # a 2048^2 TV problem needs about 256 MB of plan memory; ask for 1.5 x the device
    p = fast_tv_problem(12, 2048, 2048, 7)
    cp = A.make_problem(p.kernel, p.mask, p.lam, p.mu1, p.mu2)
    count = int(1.5 * total / 250e6) + 1
    announce(f"plan of {count} x 2048^2 problems on a device of {total / 2**30:.0f} GiB")
    with pytest.raises(A.AdmmError) as e:
        A.admm_deconv_plan([cp] * count)
    assert e.value.status == A.ADMM_E_NOMEM
    assert "allocation" in str(e.value)
    q = fast_tv_problem(13)
    with A.Plan([q]) as plan:
        yd = dev(q.y)
        x = torch.zeros_like(yd)
        info = plan.solve(yd, x, max_iters=5)
    assert info["iters"] == 5


def test_budget_exhausted_is_not_an_error():
    import torch
    announce("max_iters below the iterations to tolerance")
    p = fast_tv_problem(14)
    with A.Plan([p]) as plan:
        yd = dev(p.y)
        x = torch.zeros_like(yd)
        for graph in (False, True):
            info = plan.solve(yd, x, max_iters=30, tol=1e-6, check_every=10, graph=graph)
            assert info["iters"] == 30 and info["converged"] == 0 and info["diverged"] == 0
            assert info["r_pri"] > 1e-6
