"""The HIP path against the golden trajectories (exact / 60-digit, tests/golden).

The fixtures come from dense explicit-matrix evaluations of the iterations
(tests/golden/make_golden.py), independent of both the oracle and the
library. Bar: relative error of every recorded FP32 iterate <= 1e-4, z_1 = 0
exactly on the cold start, and the objective of the last iterate within 1e-5.
The library needs sides >= 8, so the two fixtures of that size are used; both
batch members run in one plan (a TV and an FA problem in the same launches).
"""

import numpy as np
import pytest

import oracle as O
from paper_1210_2687_amd import admm as A
from paper_1210_2687_amd import workloads as WL
from gpu_util import dev, host, rel, announce
from golden_fixtures import load

pytestmark = pytest.mark.gpu

ITER_TOL = 1e-4
OBJ_TOL = 1e-5
NAMES = ("tv_md_8x10", "fa_md_8x8_J3")


def _problem(g):
    reg = "tv" if g["reg"] == "tv" else "frame"
    return WL.Problem(y=g["y"], mask=g["mask"], kernel=g["kernel"], lam=g["lambda"], mu1=g["mu1"],
                      mu2=g["mu2"], reg=reg, levels=g["levels"])


@pytest.mark.parametrize("graph", [False, True])
def test_iterates_match_golden_trajectories(graph):
    import torch
    gs = [load(n) for n in NAMES]
    probs = [_problem(g) for g in gs]
    ks = sorted(set(gs[0]["zs"]) & set(gs[1]["zs"]))
    with A.Plan(probs) as plan:
        for k in ks:
            announce(f"golden batch k={k} graph={graph}")
            ys = [dev(p.y) for p in probs]
            xs = [torch.zeros_like(y) for y in ys]
            infos = plan.batch(ys, xs, max_iters=k, graph=graph)
            for g, p, x, info in zip(gs, probs, xs, infos):
                z = host(x)
                assert info["iters"] == k
                if k == 1:
                    assert np.all(z == 0.0)
                    continue
                e = rel(z, g["zs"][k])
                announce(f"  {p.reg} {p.shape} k={k} rel err {e:.3e}")
                assert e <= ITER_TOL
                if k == g["iters"]:
                    if g["reg"] == "tv":
                        f = O.tv_objective(z, g["y"], g["mask"], g["kernel"], g["lambda"])
                    else:
                        f = O.fa_objective(z, g["y"], g["mask"], g["kernel"], g["lambda"], g["levels"])
                    f_ref = g["objective"][1]
                    assert abs(f - f_ref) <= OBJ_TOL * abs(f_ref)
