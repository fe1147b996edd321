"""GPU checks of the FFT autotuner: it plans, caches its choice, reuses the
cache, and the iterates do not depend on the tile shape it picks."""

import json

import numpy as np
import pytest

from paper_1210_2687_amd import admm as A
from paper_1210_2687_amd import workloads as WL
from gpu_util import announce, dev, fast_tv_problem, host

pytestmark = pytest.mark.gpu


def _batch():
    probs = [fast_tv_problem(51, 96, 128, 7), fast_tv_problem(52, 64, 64, 5), WL.config3(size=64, levels=2)]
    return probs


def _run(plan, probs, iters=30):
    import torch
    ys = [dev(p.y) for p in probs]
    xs = [torch.zeros_like(y) for y in ys]
    plan.batch(ys, xs, max_iters=iters)
    torch.cuda.synchronize()
    return [host(x) for x in xs]


def _cprobs(probs):
    return [A.make_problem(p.kernel, p.mask, p.lam, p.mu1, p.mu2,
                           A.ADMM_REG_FRAME if p.reg == "frame" else A.ADMM_REG_TV, p.levels) for p in probs]


def _arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def test_tuned_plan_writes_and_reuses_its_cache(tmp_path):
    probs = _batch()
    path = str(tmp_path / "tune.json")
    announce("autotune: measuring")
    with A.Plan(probs, tune=True, cache_path=path) as plan:
        tiles = [plan.tiles(i) for i in range(len(probs))]
    data = json.load(open(path))
    assert len(data) == 1
    key = A.admm_tune_key(_cprobs(probs), _arch())
    entry = data[key]
    announce(f"  {key}: {entry}")
    assert 1 <= entry["tc"] <= 4 and entry["rows"] >= 1 and entry["col_us"] > 0 and entry["row_us"] > 0
    assert all(1 <= tc <= entry["tc"] and 1 <= b <= entry["rows"] for tc, b in tiles)
    # a forced entry is used as written, without measuring
    A.admm_tune_cache_store(path, key, 1, 2)
    with A.Plan(probs, tune=True, cache_path=path) as plan:
        assert all(plan.tiles(i) == (1, 2) for i in range(len(probs)))


@pytest.mark.parametrize("tc,rows", [(1, 2), (2, 5), (4, 8), (3, 16)])
def test_iterates_do_not_depend_on_the_tile_shape(tmp_path, tc, rows):
    probs = _batch()
    with A.Plan(probs) as plan:
        ref = _run(plan, probs)
    path = str(tmp_path / "tune.json")
    A.admm_tune_cache_store(path, A.admm_tune_key(_cprobs(probs), _arch()), tc, rows)
    with A.Plan(probs, tune=True, cache_path=path) as plan:
        used = [plan.tiles(i) for i in range(len(probs))]
        got = _run(plan, probs)
    announce(f"tiles {used}")
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_pass_timing_entry_point():
    import torch
    probs = _batch()
    with A.Plan(probs) as plan:
        _run(plan, probs, iters=5)
        for k in ("col", "row_tv", "frame", "row_inv", "row_fwd"):
            ms = plan.time_pass(k, reps=5)
            assert 0.0 < ms < 100.0, k
        with pytest.raises(A.AdmmError):
            plan.time_pass("nonsense", reps=5)
        # a solve after the timing launches starts over from its own initial state
        ref = _run(plan, probs)
    with A.Plan(probs) as plan2:
        again = _run(plan2, probs)
    for a, b in zip(ref, again):
        assert np.array_equal(a, b)
