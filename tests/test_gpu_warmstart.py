"""GPU checks of the learned warm start: the state mapping against the oracle,
the fixed-point property, the cold-start fallback, the network's gradients
against an FP64 backpropagation, and what a trained network gains."""

import numpy as np
import pytest

import oracle as O
from paper_1210_2687_amd import admm as A
from paper_1210_2687_amd import warmstart as WS
from paper_1210_2687_amd import workloads as WL
from gpu_util import announce, dev, fast_tv_problem, host, rel

pytestmark = pytest.mark.gpu


def test_warmstart_map_matches_oracle():
    p = fast_tv_problem(61, 72, 96, 9)
    g = np.random.default_rng(61)
    H, W = p.shape
    x0 = g.uniform(0, 1, (H, W))
    p0 = g.standard_normal((2, H, W)) * 0.8            # about a third of the pixels have |p0| > 1
    st = A.alloc_state(H, W)
    with A.Plan([p]) as plan:
        plan.warmstart_map(0, dev(x0), dev(p0), dev(p.y), st)
    ref = O.warm_start_state(x0, p0[0], p0[1], p.y, p.mask, p.kernel, p.lam, p.mu1, p.mu2)
    errs = {"u1": rel(host(st["u1"]), ref.u1), "d1": rel(host(st["d1"]), ref.d1),
            "uh": rel(host(st["ureg"])[0], ref.uh), "uv": rel(host(st["ureg"])[1], ref.uv),
            "dh": rel(host(st["dreg"])[0], ref.dh), "dv": rel(host(st["dreg"])[1], ref.dv)}
    announce(f"map errors {errs}")
    assert max(errs.values()) <= 1e-5


def test_mapped_solution_is_a_fixed_point():
    import torch
    p = fast_tv_problem(62, 64, 64, 7)
    H, W = p.shape
    y = dev(p.y)
    with A.Plan([p]) as plan:
        st = A.alloc_state(H, W)
        x = torch.zeros_like(y)
        info = plan.solve(y, x, st, max_iters=20000, tol=2e-6, check_every=50)
        assert info["converged"] == 1
        pstar = -(p.mu2 / p.lam) * st["dreg"]
        st2 = A.alloc_state(H, W)
        plan.warmstart_map(0, x, pstar.contiguous(), y, st2)
        x2 = torch.zeros_like(y)
        info2 = plan.solve(y, x2, st2, max_iters=1000, tol=1e-4, check_every=10)
    announce(f"cold {info['iters']} iterations to 2e-6; from the mapped solution {info2['iters']} to 1e-4")
    assert info2["converged"] == 1 and info2["iters"] <= 20
    assert abs(info2["objective"] - info["objective"]) <= 1e-6 * abs(info["objective"])


def test_non_finite_prediction_falls_back_to_a_cold_start():
    import torch
    p = fast_tv_problem(63, 64, 64, 7)
    net = WS.WarmStartNet(seed=1)
    net.w[-1].fill_(float("nan"))
    net.pack()
    y, m, e = WS.to_device([p])
    with A.Plan([p]) as plan:
        _, ic, _ = WS.solve_cold(plan, y[0], 1e-4, 5000, 10)
        xw, iw, _, used = WS.solve_warm(plan, net, y[0], m[0], e[0], 1e-4, 5000, 10)
    assert not used
    assert iw["iters"] == ic["iters"] and iw["objective"] == ic["objective"]
    assert torch.isfinite(xw).all()


def _bf16(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32).to(torch.bfloat16).to(torch.float32).double().numpy()


def _oracle_backprop(net, y, m, e, xt, pt):
    """FP64 forward and backward of the same network, with activations and
    back-propagated gradients rounded to bf16 where the device stores them."""
    N, H, W = y.shape
    a = np.zeros((N, H, W, 8))
    a[..., 0] = m * y
    a[..., 1] = m
    a[..., 2:6] = e[:, None, None, :]
    acts = [_bf16(a)]
    ws = []
    nl = len(net.w)
    for li in range(nl):
        w = host(net.w[li])                                      # [9][cout][cin]
        cout, cin = w.shape[1], w.shape[2]
        wo = _bf16(w).reshape(3, 3, cout, cin).transpose(0, 1, 3, 2)
        ws.append(wo)
        z = O.conv3x3_fwd(acts[-1], wo, host(net.b[li]), dil=net.dil[li])
        acts.append(_bf16(O.relu(z) if li < nl - 1 else z))
    out = acts[-1]
    npx = N * H * W
    g = np.zeros_like(out)
    g[..., 0] = 2.0 * (m * y + out[..., 0] - xt) / npx
    g[..., 1] = 2.0 * net.alpha * (out[..., 1] - pt[:, 0]) / npx
    g[..., 2] = 2.0 * net.alpha * (out[..., 2] - pt[:, 1]) / npx
    dy = _bf16(g)
    dws, dbs = [None] * nl, [None] * nl
    for li in range(nl - 1, -1, -1):
        dw, db = O.conv3x3_wgrad(acts[li], dy, dil=net.dil[li])
        dws[li] = dw.transpose(0, 1, 3, 2).reshape(9, dw.shape[3], dw.shape[2])
        dbs[li] = db
        if li > 0:
            dy = _bf16(O.conv3x3_dgrad(dy, ws[li], dil=net.dil[li]) * (acts[li] > 0))
    return dws, dbs


def test_network_gradients_match_fp64_backpropagation():
    import torch
    g = np.random.default_rng(64)
    N, H, W = 2, 12, 20
    y = g.uniform(0, 1, (N, H, W))
    m = (g.uniform(size=(N, H, W)) > 0.3).astype(np.uint8)
    e = g.uniform(0, 0.5, (N, 4))
    xt = g.uniform(0, 1, (N, H, W))
    pt = g.uniform(-1, 1, (N, 2, H, W))
    net = WS.WarmStartNet(seed=2)
    f32 = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda").contiguous()
    _, dws, dbs = net.gradients(f32(y), torch.tensor(m, device="cuda"), f32(e), f32(xt), f32(pt))
    torch.cuda.synchronize()
    rdw, rdb = _oracle_backprop(net, host(f32(y)), m, host(f32(e)), host(f32(xt)), host(f32(pt)))
    for li in range(len(dws)):
        ew, eb = rel(host(dws[li]), rdw[li]), rel(host(dbs[li]), rdb[li])
        announce(f"layer {li}: dw rel {ew:.2e} db rel {eb:.2e}")
        assert ew <= 1e-2 and eb <= 1e-2


def test_training_lowers_the_loss_and_the_warm_start_cuts_iterations():
    announce("targets")
    data = WS.targets(WS.problems(0, 64, 128))
    net = WS.WarmStartNet(seed=0)
    hist = WS.train(net, data, steps=400, batch=8)
    first, last = np.mean(hist[:10]), np.mean(hist[-10:])
    announce(f"loss {first:.3e} -> {last:.3e}")
    assert last < 0.7 * first
    rows = WS.evaluate(net, WS.problems(10 ** 6, 6, 128))
    s = WS.summary(rows)
    announce(str(s))
    assert s["all_converged"]
    assert all(r["warm_used"] for r in rows)
    assert s["p50_warm_iters"] < 0.9 * s["p50_cold_iters"]
    assert s["max_rel_objective_gap_final"] <= 1e-5
