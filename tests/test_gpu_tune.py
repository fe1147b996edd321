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
        # one size class alone: columns of 64 (radix-8 ends) and 96 (general), TV rows <= 512
        for k in ("col:0", "col:1", "row_tv:0"):
            ms = plan.time_pass(k, reps=5)
            assert 0.0 < ms < 100.0, k
        for k in ("col:4", "row_tv:2", "col:9", "row_tv:3", "col:", "col:x", "frame:0"):
            with pytest.raises(A.AdmmError):
                plan.time_pass(k, reps=5)
        # a solve after the timing launches starts over from its own initial state
        ref = _run(plan, probs)
    with A.Plan(probs) as plan2:
        again = _run(plan2, probs)
    for a, b in zip(ref, again):
        assert np.array_equal(a, b)


# ------------------------------------------- radix schedules (the tuner's radix dimension)
def _oracle_z(p, K):
    import oracle as O
    if p.reg == "frame":
        return O.fa_md_run(p.y, p.mask, p.kernel, p.lam, p.mu1, p.mu2, p.levels, iters=K)["z"]
    return O.tv_md_run(p.y, p.mask, p.kernel, p.lam, p.mu1, p.mu2, iters=K)["z"]


def _sched_batch():
    # lengths with each kind of factorisation: powers of two (512, 256, 64),
    # mixed (96 = 2^5 3, 160 = 2^5 5, 448 = 2^6 7, 120 = 2^3 15, 1000 = 2^3 5^3)
    from gpu_util import full_problem
    return [full_problem(601, 96, 160, 7), full_problem(602, 512, 448, 9, "motion"),
            full_problem(603, 120, 1000, 5, "uniform"), full_problem(604, 256, 64, 7),
            full_problem(605, 64, 96, 5, reg="frame", levels=2)]


@pytest.mark.parametrize("rsched,csched", [(0, 0), (1, 0), (2, 0), (3, 0), (0, 1), (0, 2), (3, 2), (1, 1)])
def test_every_radix_schedule_matches_the_oracle(rsched, csched):
    # a schedule changes the rounding of the transforms only: each variant is
    # held to the per-iterate bar against the FP64 oracle (not bitwise)
    from gpu_util import check_iterate
    import torch
    probs = _sched_batch()
    K = 12
    with A.Plan(probs, tiles={"row_schedule": rsched, "col_schedule": csched}) as plan:
        used = [plan.schedules(i) for i in range(len(probs))]
        ys = [dev(p.y) for p in probs]
        xs = [torch.zeros_like(y) for y in ys]
        plan.batch(ys, xs, max_iters=K)
        got = [host(x) for x in xs]
    announce(f"schedules requested ({rsched}, {csched}), used {used}")
    for p, (rv, cv) in zip(probs, used):
        H, W = p.shape
        # the variant is used unless it gives the length the default schedule
        same_r = A.admm_fft_schedule(W, rsched) == A.admm_fft_schedule(W, 0)
        same_c = A.admm_fft_schedule(H, csched) == A.admm_fft_schedule(H, 0)
        assert rv == (0 if same_r else rsched) and cv == (0 if same_c else csched)
    for p, z in zip(probs, got):
        check_iterate(z, _oracle_z(p, K), what=f"{p.shape} schedules ({rsched}, {csched})")


def test_tuner_records_and_reuses_radix_schedules(tmp_path):
    probs = _sched_batch()[:3]
    path = str(tmp_path / "tune.json")
    with A.Plan(probs, tune=True, cache_path=path) as plan:
        chosen = [plan.schedules(i) for i in range(len(probs))]
    entry = json.load(open(path))[A.admm_tune_key(_cprobs(probs), _arch())]
    announce(f"tuned entry {entry}, schedules {chosen}")
    assert 0 <= entry.get("rsched", 0) <= 3 and 0 <= entry.get("csched", 0) <= 2
    # planning again from the cache reproduces the schedules without measuring
    with A.Plan(probs, tune=True, cache_path=path) as plan:
        assert [plan.schedules(i) for i in range(len(probs))] == chosen
