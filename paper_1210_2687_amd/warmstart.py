"""Learned warm start for TV-MD (not part of the paper's method).

A 6-layer 3x3 CNN reads the observation and predicts an initial image x0 and
a TV dual field p0; ``admm_warmstart_map`` turns them into the ADMM state
u1 = A x0, d1 = M^T (y - M A x0) / mu1, u_TV = D x0, d_TV = -(lambda/mu2) p0
(|p0| clipped to 1). These are the KKT forms of the optimal state, so a
perfect prediction is a fixed point, and by Theorem 1 of the paper any
prediction still converges to a minimiser: the network changes the iteration
count, never the answer. A non-finite prediction falls back to a cold start.

Network: layers 8 -> 32 -> 32 -> 32 -> 32 -> 32 -> 16 channels, 3x3 kernels
dilated 1, 2, 4, 8, 4, 1 (a 41 x 41 receptive field), ReLU after all but the last; input [m y, m, e0..e3, 0, 0] with a 4-number kernel embedding e;
outputs 0..2 give x0 = m y + out0 and p0 = (out1, out2). Activations are
NHWC bf16, weights FP32 masters with bf16 copies, accumulation FP32, all in
the library's BF16 MFMA kernels; the loss is mean over pixels of
(x0 - x*)^2 + alpha |p0 - p*|^2 with targets from the GPU ADMM itself, and
the optimiser is Adam. This module only orchestrates: every step of the
forward pass, the backward pass and the update runs in the library.
"""

import math
import time

import numpy as np

from . import admm as A
from . import workloads as WL

CHANNELS = (8, 32, 32, 32, 32, 32, 16)
DILATIONS = (1, 2, 4, 8, 4, 1)    # per layer: a 41 x 41 receptive field (13 x 13 undilated)


def kernel_embedding(h):
    """Four numbers describing a blur kernel: its second moments about the
    centre (rows, columns, cross; in units of 16 px^2) and sqrt(sum h^2)."""
    h = np.asarray(h, dtype=np.float64)
    k = h.shape[0]
    o = np.arange(k) - k // 2
    r, c = np.meshgrid(o, o, indexing="ij")
    s = h.sum()
    return np.array([(h * r * r).sum() / s / 16.0, (h * c * c).sum() / s / 16.0,
                     (h * r * c).sum() / s / 16.0, math.sqrt((h * h).sum())], dtype=np.float32)


class WarmStartNet:
    """Weights, Adam state and scratch of the warm-start CNN (device tensors)."""

    def __init__(self, seed=0, alpha=0.25, dilations=DILATIONS):
        import torch
        self.alpha = alpha
        self.dil = tuple(int(d) for d in dilations)
        assert len(self.dil) == len(CHANNELS) - 1
        g = np.random.default_rng(seed)
        self.w, self.b, self.mw, self.vw, self.mb, self.vb = [], [], [], [], [], []
        self.wf, self.wb = [], []
        for li in range(len(CHANNELS) - 1):
            cin, cout = CHANNELS[li], CHANNELS[li + 1]
            # He initialisation for the ReLU layers; the output layer starts small so
            # that the first prediction is close to x0 = m y, p0 = 0
            fan_in = 9 * (cin if li > 0 else 6)
            std = math.sqrt(2.0 / fan_in) * (0.1 if li == len(CHANNELS) - 2 else 1.0)
            w = (std * g.standard_normal((9, cout, cin))).astype(np.float32)
            if li == 0:
                w[:, :, 6:] = 0.0          # the two spare input channels
            f32 = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda").contiguous()
            self.w.append(f32(w))
            self.b.append(torch.zeros(cout, dtype=torch.float32, device="cuda"))
            self.mw.append(torch.zeros_like(self.w[-1]))
            self.vw.append(torch.zeros_like(self.w[-1]))
            self.mb.append(torch.zeros_like(self.b[-1]))
            self.vb.append(torch.zeros_like(self.b[-1]))
            self.wf.append(torch.zeros(9 * 32 * 32, dtype=torch.bfloat16, device="cuda"))
            self.wb.append(torch.zeros(9 * 32 * 32, dtype=torch.bfloat16, device="cuda"))
        self.t = 0
        self._ws = {}
        self.pack()

    @property
    def nparams(self):
        return sum(w.numel() + b.numel() for w, b in zip(self.w, self.b))

    def pack(self):
        for li in range(len(self.w)):
            A.admm_conv3x3_pack_weights(self.w[li], CHANNELS[li], CHANNELS[li + 1], self.wf[li], self.wb[li])

    def _buf(self, name, shape, dtype):
        import torch
        t = self._ws.get(name)
        if t is None or t.shape != torch.Size(shape) or t.dtype != dtype:
            t = torch.empty(shape, dtype=dtype, device="cuda")
            self._ws[name] = t
        return t

    def forward(self, y, mask, emb, keep=False):
        """y [N,H,W] f32, mask [N,H,W] u8, emb [N,4] f32 -> output [N,H,W,16] bf16
        (and the list of layer inputs when keep is set, for the backward pass)."""
        import torch
        N, H, W = y.shape
        a = self._buf("in", (N, H, W, 8), torch.bfloat16)
        A.admm_ws_input(y, mask, emb, N, H, W, a)
        acts = [a]
        nl = len(self.w)
        for li in range(nl):
            cout = CHANNELS[li + 1]
            # every layer input is kept for the backward pass; inference ping-pongs
            o = self._buf(f"a{li + 1}" if keep else f"p{li % 2}_{cout}", (N, H, W, cout), torch.bfloat16)
            A.admm_conv3x3_bf16_fwd(acts[-1], N, H, W, CHANNELS[li], self.wf[li], self.b[li], cout,
                                    1 if li < nl - 1 else 0, None, o, dil=self.dil[li])
            acts.append(o)
        return (acts[-1], acts) if keep else acts[-1]

    def gradients(self, y, mask, emb, xt, pt):
        """Loss and its gradients (lists dw [9][cout][cin], db [cout], FP32,
        device buffers reused by the next call) on a minibatch."""
        import torch
        N, H, W = y.shape
        out, acts = self.forward(y, mask, emb, keep=True)
        npx = N * H * W
        dout = self._buf("dout", (N, H, W, 16), torch.bfloat16)
        lpart = self._buf("lpart", ((npx + 255) // 256,), torch.float32)
        A.admm_ws_loss(out, y, mask, xt, pt, N, H, W, self.alpha, dout, lpart)
        chunk = 1024
        dy = dout
        nl = len(self.w)
        dws, dbs = [None] * nl, [None] * nl
        for li in range(nl - 1, -1, -1):
            cin, cout = CHANNELS[li], CHANNELS[li + 1]
            wsb = A.admm_conv3x3_bf16_wgrad_workspace(N, H, W, cin, cout, chunk)
            ws = self._buf(f"ws{li}", (wsb // 4 + 1,), torch.float32)
            dws[li] = self._buf(f"dw{li}", (9, cout, cin), torch.float32)
            dbs[li] = self._buf(f"db{li}", (cout,), torch.float32)
            A.admm_conv3x3_bf16_wgrad(acts[li], dy, N, H, W, cin, cout, chunk, ws, dws[li], dbs[li], dil=self.dil[li])
            if li > 0:
                # dL/d(input of layer li) through the ReLU that produced it
                dx = self._buf(f"dx{li % 2}_{cin}", (N, H, W, cin), torch.bfloat16)
                A.admm_conv3x3_bf16_fwd(dy, N, H, W, cout, self.wb[li], None, cin, 0, acts[li], dx, dil=self.dil[li])
                dy = dx
        return lpart, dws, dbs

    def train_step(self, y, mask, emb, xt, pt, lr, want_loss=True):
        """One Adam step on a minibatch; returns the loss (host float) if asked."""
        lpart, dws, dbs = self.gradients(y, mask, emb, xt, pt)
        self.t += 1
        for li in range(len(self.w)):
            A.admm_adam_step(self.w[li], dws[li], self.mw[li], self.vw[li], lr, self.t)
            A.admm_adam_step(self.b[li], dbs[li], self.mb[li], self.vb[li], lr, self.t)
        self.pack()
        return float(lpart.sum().item()) if want_loss else None

    def predict(self, y, mask, emb):
        """Warm-start guess (x0 [N,H,W], p0 [N,2,H,W]) for a batch."""
        import torch
        N, H, W = y.shape
        out = self.forward(y, mask, emb)
        x0 = torch.empty((N, H, W), dtype=torch.float32, device="cuda")
        p0 = torch.empty((N, 2, H, W), dtype=torch.float32, device="cuda")
        A.admm_ws_output(out, y, mask, N, H, W, x0, p0)
        return x0, p0


# ----------------------------------------------------------------- data
def problems(first, count, size):
    return [WL.config5_problem(first + i, size=size) for i in range(count)]


def light_problem(index, size):
    """``WL.config5_problem`` without the true image and with a float32
    observation (what the solver and the network read; a quarter of the host
    memory, for data sets of tens of thousands of problems)."""
    p = WL.config5_problem(index, size=size)
    return WL.Problem(y=p.y.astype(np.float32), mask=p.mask, kernel=p.kernel, lam=p.lam, mu1=p.mu1, mu2=p.mu2)


def to_device(probs):
    import torch
    y = torch.tensor(np.stack([p.y for p in probs]), dtype=torch.float32, device="cuda")
    m = torch.tensor(np.stack([p.mask for p in probs]), dtype=torch.uint8, device="cuda")
    e = torch.tensor(np.stack([kernel_embedding(p.kernel) for p in probs]), dtype=torch.float32, device="cuda")
    return y, m, e


def targets(probs, tol=1e-6, max_iters=8000, check_every=20):
    """Training targets from the GPU ADMM itself, all problems in one batch:
    x* and the dual field p* = -(mu2 / lambda) d_TV* (admm_warmstart_dual).
    Returns (y, m, e, xt, pt, infos); a target whose solve stopped at
    max_iters before tol is kept (it is an iterate of the same convergent
    method) and counted as unconverged in its info."""
    import torch
    y, m, e = to_device(probs)
    N = len(probs)
    H, W = probs[0].shape
    xt = torch.zeros((N, H, W), dtype=torch.float32, device="cuda")
    pt = torch.empty((N, 2, H, W), dtype=torch.float32, device="cuda")
    with A.Plan(probs) as plan:
        states = [A.alloc_state(H, W) for _ in probs]
        infos = plan.batch([y[i] for i in range(N)], [xt[i] for i in range(N)], states, max_iters=max_iters,
                           tol=tol, check_every=check_every, graph=True)
        for i, st in enumerate(states):
            plan.warmstart_dual(i, st["dreg"], pt[i])
    return y, m, e, xt, pt, infos


def train(net, data, steps, batch=8, lr=2e-3, seed=0, log=None):
    """Adam on random minibatches of the data tuple (y, m, e, xt, pt); returns the loss history."""
    y, m, e, xt, pt = data[:5]
    g = np.random.default_rng(seed)
    hist = []
    for s in range(steps):
        idx = g.choice(y.shape[0], size=batch, replace=False)
        import torch
        ii = torch.tensor(idx, device="cuda")
        lr_s = lr * 0.5 * (1.0 + math.cos(math.pi * s / max(steps, 1)))   # cosine decay
        loss = net.train_step(y[ii].contiguous(), m[ii].contiguous(), e[ii].contiguous(), xt[ii].contiguous(),
                              pt[ii].contiguous(), lr_s)
        hist.append(loss)
        if log and (s % max(1, steps // 10) == 0 or s == steps - 1):
            log(f"step {s}: loss {loss:.4e}")
    return hist


# ----------------------------------------------------------------- time to tolerance
def solve_cold(plan, y, tol, max_iters, check_every):
    import torch
    x = torch.zeros_like(y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = plan.solve(y, x, None, max_iters=max_iters, tol=tol, check_every=check_every, graph=True)
    torch.cuda.synchronize()
    return x, info, time.perf_counter() - t0


def solve_warm(plan, net, y, m, e, tol, max_iters, check_every):
    """Network inference + state mapping + solve, timed together; cold start if
    the prediction is not finite."""
    import torch
    H, W = y.shape
    x = torch.zeros_like(y)
    st = A.alloc_state(H, W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x0, p0 = net.predict(y[None], m[None], e[None])
    ok = bool(torch.isfinite(x0).all().item() and torch.isfinite(p0).all().item())
    if ok:
        plan.warmstart_map(0, x0[0].contiguous(), p0[0].contiguous(), y, st)
    info = plan.solve(y, x, st if ok else None, max_iters=max_iters, tol=tol, check_every=check_every, graph=True)
    torch.cuda.synchronize()
    return x, info, time.perf_counter() - t0, ok


def final_objectives(net, probs, y, m, e, tol, max_iters, check_every=50, batch=64):
    """Objectives of cold and warm runs to a tight tolerance, problems in
    batches of ``batch`` (throughput mode: only the values are compared)."""
    import torch
    out = []
    for b in range(0, len(probs), batch):
        chunk = probs[b:b + batch]
        n = len(chunk)
        ys = [y[b + i] for i in range(n)]
        with A.Plan(chunk) as plan:
            xs = [torch.zeros_like(t) for t in ys]
            ic = plan.batch(ys, xs, None, max_iters=max_iters, tol=tol, check_every=check_every, graph=True)
            x0, p0 = net.predict(y[b:b + n], m[b:b + n], e[b:b + n])
            ok = [bool(torch.isfinite(x0[i]).all().item() and torch.isfinite(p0[i]).all().item()) for i in range(n)]
            sts = [A.alloc_state(*p.shape) for p in chunk]
            for i in range(n):
                if ok[i]:
                    plan.warmstart_map(i, x0[i].contiguous(), p0[i].contiguous(), ys[i], sts[i])
            xs = [torch.zeros_like(t) for t in ys]
            iw = plan.batch(ys, xs, sts, max_iters=max_iters, tol=tol, check_every=check_every, graph=True)
        out += list(zip(ic, iw))
    return out


def evaluate(net, probs, tol=1e-4, max_iters=8000, check_every=10, final_tol=5e-6, final_iters=40000,
             final_batch=64, log=None):
    """Per-problem cold and warm time-to-tolerance (seconds, warm including the
    network and the state mapping), iterations, and the objectives F of cold
    and warm runs continued to final_tol (the minimiser's F is unique; at tol
    both are still up to about tol away from it). Each problem gets its own
    plan; the graphs of both paths are captured by short untimed runs before
    the timed solves."""
    y, m, e = to_device(probs)
    rows = []
    warm_k = 4 * check_every + 1      # long enough to capture the period graphs the timed runs replay
    for i, p in enumerate(probs):
        with A.Plan([p]) as plan:
            solve_cold(plan, y[i], tol, warm_k, check_every)
            solve_warm(plan, net, y[i], m[i], e[i], tol, warm_k, check_every)
            _, ic, tc = solve_cold(plan, y[i], tol, max_iters, check_every)
            _, iw, tw, ok = solve_warm(plan, net, y[i], m[i], e[i], tol, max_iters, check_every)
        rows.append({"cold_s": tc, "warm_s": tw, "cold_iters": ic["iters"], "warm_iters": iw["iters"],
                     "cold_obj": ic["objective"], "warm_obj": iw["objective"], "cold_conv": ic["converged"],
                     "warm_conv": iw["converged"], "warm_used": ok})
        if log and (i + 1) % 64 == 0:
            log(f"  timed {i + 1}/{len(probs)} problems")
    if final_tol:
        fin = final_objectives(net, probs, y, m, e, final_tol, final_iters, batch=final_batch)
        for r, (fc, fw) in zip(rows, fin):
            r.update({"final_cold_obj": fc["objective"], "final_warm_obj": fw["objective"],
                      "final_conv": fc["converged"] and fw["converged"]})
    else:
        for r in rows:
            r.update({"final_cold_obj": r["cold_obj"], "final_warm_obj": r["warm_obj"],
                      "final_conv": r["cold_conv"] and r["warm_conv"]})
    return rows


def summary(rows):
    c = np.array([r["cold_s"] for r in rows]) * 1e3
    w = np.array([r["warm_s"] for r in rows]) * 1e3
    ci = np.array([r["cold_iters"] for r in rows])
    wi = np.array([r["warm_iters"] for r in rows])
    co = np.array([r["cold_obj"] for r in rows])
    wo = np.array([r["warm_obj"] for r in rows])
    return {"n": len(rows), "p50_cold_ms": float(np.median(c)), "p50_warm_ms": float(np.median(w)),
            "p90_cold_ms": float(np.percentile(c, 90)), "p90_warm_ms": float(np.percentile(w, 90)),
            "p50_speedup": float(np.median(c) / np.median(w)),
            "p50_cold_iters": float(np.median(ci)), "p50_warm_iters": float(np.median(wi)),
            "max_rel_objective_gap_at_tol": float(np.max(np.abs(wo - co) / np.abs(co))),
            "max_rel_objective_gap_final": float(np.max([abs(r["final_warm_obj"] - r["final_cold_obj"]) /
                                                         abs(r["final_cold_obj"]) for r in rows])),
            "final_converged": bool(all(r["final_conv"] for r in rows)),
            "all_converged": bool(all(r["cold_conv"] and r["warm_conv"] for r in rows))}
