#!/usr/bin/env python3
"""Benchmark of the batched mask-decoupled ADMM (TV-MD, FA-MD) on one MI355X.

Headline (the timed steps): 8 unknown 512x512 images (rectangles/ellipses
plus a smooth random field), images 0-3 blurred by a 19x19 Gaussian
(sigma 3), 4-7 by a 15-px linear motion blur, observed on the valid region
minus 40% i.i.d. missing pixels, sigma 2e-3, lambda 2e-4, mu1 = mu2 = 1e-3.
One step = one batched solve of 500 ADMM iterations from a cold start (plan,
y, x and all workspaces resident on the GPU before timing starts).

The same JSON line also carries, under "configs", the other workloads:
  c1          128^2 TV-MD, 9x9 uniform, 200 iterations (GPU time; the FP64
              oracle's wall time is in cpu_baseline)
  c3          FA-MD 1024^2, J = 3, 13x13 disk, 20% missing 8x8 blocks, time to
              residual tolerance 1e-4
  c3_fs       FS-MD (frame synthesis) on the c3 data, 400 iterations
  headline_cg TV-CG (Reeves-Sorel, one CG step per iteration) on the
              headline batch
  md_vs_cg    the paper's MD-vs-CG comparison (Tables 3 and 4): 256^2,
              four 19x19 blurs, TV and FA, MD to the paper's stopping rule,
              CG to the MD objective
  tv4096      TV-MD 4096^2, 100 iterations (sides above 2048: the block-level
              column pass and the three-pass TV row schedule)
  tv8192      (only with --quick --workload tv8192: its input takes over a
              minute of host work) TV-MD 8192^2, 20 iterations
  tv16384     (only with --quick --workload tv16384) TV-MD 16384^2, 10
              iterations, on the 4096^2 image tiled 4 x 4 (throughput does not
              depend on the data; the columns run the split transform)
  c4          ragged batch of 256 TV-MD problems (sides 128..1024, kernels
              5..31), 200 iterations
  beyond_cache  64 x 512^2 TV-MD, 500 iterations (working set ~0.9 GB, far
              beyond the 256 MB memory-side cache)
  c5          learned warm start: 20k training problems at 256^2 (targets from
              the GPU ADMM), 512 unseen 512^2 problems, p50 time to 1e-4 cold
              vs warm
with a roofline per workload: algorithmic bytes per iteration (this
schedule's two-launch TV iteration, the FA iteration's four launches) over
the measured time per iteration, and for the headline the dominant kernel's
launch duration as well. ``--quick`` runs the headline alone. The CPU
baseline (the FP64 oracle) also times 5 iterations of the c3 problem and 5
of four c4 problems when those workloads run.
"""

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor
from functools import partial

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel·ADMM-iters/s (batched) + p50 time-to-tol, warm-start vs cold-start"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "row_tv_tv8x512_traffic.txt")
KERNEL_SOURCES = ["paper_1210_2687_amd/csrc/admm_kernels.hip", "paper_1210_2687_amd/csrc/fft_lds.h",
                  "paper_1210_2687_amd/csrc/admm_internal.h"]


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def alg_bytes_per_launch(problems):
    """Algorithmic HBM bytes of one launch of each kernel class (plain iteration).

    col:     read the two transposed half spectra (16 B / entry) and Lambda
             (8 B / entry), write the two half spectra back: 40 B per entry of
             the H x (W/2+1) half spectrum.
    row_tv:  read the half spectra (16 B / entry), d1, d^h, d^v (12 B / px),
             y (4 B / px) and the mask (1 B / px); write d1, d^h, d^v
             (12 B / px) and the next half spectra (16 B / entry).
    row_inv: read the half spectra (16 B / entry), d1, y, mask (9 B / px);
             write d1, zeta1, z (12 B / px); the synthesis formulation also
             reads s (4 B / px).
    frame:   read z (4 B / px) and the 3J+1 frame duals, write the duals and
             q (4 B / px): 8 + 8 (3J+1) B / px (the synthesis formulation:
             x - W zeta2 and the coefficients u2, the same count).
    row_fwd: read zeta1 and q (8 B / px), write the half spectra (16 B / entry).
    TV rows longer than 2048 run the three-pass schedule: row_inv and row_fwd
    as for the frame, and the TV step (counted under row_tv): read z and the
    two duals, write the duals and s, 24 B / px.
    Halo re-reads are not counted (they are overhead, not algorithmic).
    """
    out = {"col": 0, "row_tv": 0, "row_inv": 0, "frame": 0, "row_fwd": 0}
    for p in problems:
        H, W = p.shape
        hp = H * (W // 2 + 1)
        n = H * W
        out["col"] += 40 * hp
        reg = getattr(p, "reg", "tv")
        if reg in ("frame", "synthesis"):
            out["row_inv"] += 16 * hp + (25 if reg == "synthesis" else 21) * n
            out["frame"] += (8 + 8 * (3 * p.levels + 1)) * n
            out["row_fwd"] += 8 * n + 16 * hp
        elif W > 2048:
            out["row_inv"] += 16 * hp + 21 * n
            out["row_tv"] += 24 * n
            out["row_fwd"] += 8 * n + 16 * hp
        else:
            out["row_tv"] += 32 * hp + 29 * n
    return out


def iteration_roofline(problems, us_per_iter):
    b = sum(alg_bytes_per_launch(problems).values())
    gbs = b / (us_per_iter * 1e-6) / 1e9
    return {"bound": "hbm", "alg_bytes_per_iter": int(b), "us_per_iter": round(us_per_iter, 3),
            "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}


def read_traffic(expected_hash):
    """HBM traffic per launch from committed rocprofv3 counters, if taken on this kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != expected_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ------------------------------------------------------------------ host data
def _c2_member(i, size):
    from paper_1210_2687_amd import workloads as WL
    return WL.config2(i % 8, size=size)


def host_data(args):
    """Every synthetic input, generated in a process pool before the GPU is touched."""
    from paper_1210_2687_amd import workloads as WL
    from paper_1210_2687_amd import warmstart as WS
    data = {}
    workers = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers) as ex:
        # the 4096^2 image (about 16 s of host work) is drawn beside the others
        big = ex.submit(_c2_member, 0, 4096) if (args.workload == "tv4096" or not args.quick) else None
        huge = ex.submit(_c2_member, 0, 8192) if args.workload == "tv8192" else None
        if args.workload == "tv16384" and big is None:
            big = ex.submit(_c2_member, 0, 4096)
        data["c2"] = list(ex.map(partial(_c2_member, size=args.size), range(args.batch)))
        if args.workload in ("fa1024", "fs1024") or not args.quick:
            data["c3"] = WL.config3(size=1024, levels=3)
            data["c3_fs"] = dataclasses.replace(data["c3"], reg="synthesis")
        if args.workload == "ragged256" or not args.quick:
            data["c4"] = list(ex.map(WL.config4, range(256), chunksize=4))
        if args.workload == "tv64x512" or not args.quick:
            data["c64"] = [data["c2"][i % len(data["c2"])] for i in range(64)]
        if args.workload == "tv4096" or not args.quick:
            data["c_big"] = [big.result()]
        if huge is not None:
            data["c_huge"] = [huge.result()]
        if args.workload == "tv16384":
            b = big.result()
            data["c_16k"] = [dataclasses.replace(b, y=np.tile(b.y, (4, 4)), mask=np.tile(b.mask, (4, 4)),
                                                 x_true=None)]
        if not args.quick:
            data["c1"] = WL.config1()
            if args.ws_train:
                data["c5_train"] = list(ex.map(partial(WS.light_problem, size=256), range(args.ws_train),
                                               chunksize=64))
                data["c5_eval"] = list(ex.map(partial(WS.light_problem, size=512),
                                              range(10 ** 6, 10 ** 6 + args.ws_eval), chunksize=8))
    log(f"host data generated in {time.perf_counter() - t0:.1f} s with {workers} processes")
    return data


# ------------------------------------------------------------------ GPU workloads
def timed_batch(probs, iters, steps, warmup, tune, graph=True, method=0):
    """Plan (autotuned tiles unless tune is False), warm up, time `steps` cold-start
    batched solves of `iters` iterations. Returns (plan, ys, xs, result dict)."""
    import torch
    from paper_1210_2687_amd import admm as A
    ys = [torch.tensor(p.y, dtype=torch.float32, device="cuda") for p in probs]
    xs = [torch.zeros_like(y) for y in ys]
    t0 = time.perf_counter()
    plan = A.Plan(probs, tune=tune, cache_path=os.environ.get("ADMM_TUNE_CACHE"), method=method)
    t_plan = time.perf_counter() - t0
    run = lambda: plan.batch(ys, xs, max_iters=iters, tol=0.0, graph=graph)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    px = sum(p.y.size for p in probs)
    tc, rows = plan.tiles(0)
    res = {"value": px * iters / dt / 1e6, "ms_per_step": dt * 1e3, "pixels": int(px), "iters": iters,
           "us_per_iter": dt * 1e6 / iters, "plan_s": round(t_plan, 2),
           "tiles": {"cols_per_block": tc, "rows_per_block": rows, "chosen_by": "autotuner" if tune else "heuristic"}}
    return plan, ys, xs, res


def kernel_breakdown(plan, ys, xs, iters):
    """Per-launch microseconds of each kernel class from an event-timed eager run."""
    plan.batch(ys, xs, max_iters=iters, tol=0.0, graph=False, profile=True)
    kt = plan.kernel_times()
    return {k: round(v[1] / v[0] * 1e3, 3) for k, v in kt.items() if v[0]}


def dominant_roofline(plan, probs, kt, reps=50):
    """The dominant pass kernel's launch duration: `reps` back-to-back launches
    between one pair of HIP events on the plan's stream."""
    alg = alg_bytes_per_launch(probs)
    dom = max((k for k in ("col", "row_tv", "row_inv", "frame", "row_fwd") if k in kt), key=lambda k: kt[k])
    avg_s = plan.time_pass(dom, reps) / 1e3
    achieved = alg[dom] / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": dom, "avg_launch_us": round(avg_s * 1e6, 3),
            "alg_bytes_per_launch": int(alg[dom]), "timing": f"{reps} back-to-back launches between one HIP event pair"}


COL_CLASS_NAMES = ["columns <= 512, radix-8 first and last stage", "columns <= 512, general schedule",
                   "columns 513..1024, radix-8 ends", "columns 513..1024, general", "columns 1025..2048, radix-8 ends",
                   "columns 1025..2048, general", "columns 2049..4096", "columns 4097..8192", "columns above 8192"]
ROW_CLASS_NAMES = ["TV rows <= 512", "TV rows 513..1024", "TV rows 1025..2048"]


def class_breakdown(plan, reps=20):
    """Microseconds per launch of each size class of the column and fused TV row
    passes that the plan has (`reps` back-to-back launches between one HIP event pair)."""
    from paper_1210_2687_amd import admm as A
    out = {}
    for kind, names in (("col", COL_CLASS_NAMES), ("row_tv", ROW_CLASS_NAMES)):
        for c, nm in enumerate(names):
            try:
                out[f"{kind}:{c} ({nm})"] = round(plan.time_pass(f"{kind}:{c}", reps) * 1e3, 2)
            except A.AdmmError:
                pass   # no problem of the batch in this class
    return out


def run_throughput(name, probs, iters, steps, warmup, tune, desc, method=0):
    log(f"{name}: {desc}")
    plan, ys, xs, r = timed_batch(probs, iters, steps, warmup, tune, method=method)
    kt = kernel_breakdown(plan, ys, xs, min(iters, 100))
    out = {"workload": desc, "value": round(r["value"], 1), "unit": "Mpx*iter/s", "ms_per_step": round(r["ms_per_step"], 3),
           "steps": steps, "problems": len(probs), "pixels": r["pixels"], "iters": iters, "tiles": r["tiles"],
           "plan_s": r["plan_s"], "us_per_iter": round(r["us_per_iter"], 3), "kernel_us_event_per_launch": kt}
    if name == "c4":   # the ragged batch: its size classes apart
        out["class_us_per_launch"] = class_breakdown(plan)
    if method == 0:   # the rooflines price the MD schedule's launches
        out["roofline_iteration"] = iteration_roofline(probs, r["us_per_iter"])
        out["roofline_dominant"] = dominant_roofline(plan, probs, kt)
        log(f"{name}: {out['value']:.1f} Mpx*iter/s, iteration at {out['roofline_iteration']['frac']:.3f} of HBM peak")
    else:
        log(f"{name}: {out['value']:.1f} Mpx*iter/s, {r['us_per_iter']:.2f} us per iteration")
    plan.close()
    return out


def _solve_ms(plan, y, x, reps=3, **kw):
    """Median wall time (ms) of `reps` solves on the plan's stream, and the last info."""
    import torch
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = plan.solve(y, x, graph=True, **kw)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(times)), info


def _us_per_iter(plan, y, x, K=400):
    """Microseconds per iteration: solves of K and 3K iterations, the difference
    over 2K (the per-solve work cancels)."""
    a, _ = _solve_ms(plan, y, x, max_iters=K, check_every=K)
    b, _ = _solve_ms(plan, y, x, max_iters=3 * K, check_every=3 * K)
    return (b - a) * 1e3 / (2 * K)


def run_md_vs_cg(obj_tol=1e-4, c=10, max_iters=20000):
    """The paper's MD-vs-CG comparison (Sec. V, Tables 3 and 4) on synthetic
    256 x 256 images with its four 19 x 19 blurs at 40 dB BSNR: each MD solve
    runs to the paper's stopping rule (relative change of the objective from
    one iteration to the next <= obj_tol), then the CG variant runs until its
    objective reaches the MD solve's final objective (the smallest multiple of
    c found by doubling and bisection over cold-start solves); both solves
    timed whole. Also the time per iteration of the four solvers (Table 4)."""
    import torch
    from paper_1210_2687_amd import admm as A
    from paper_1210_2687_amd import workloads as WL
    log("md_vs_cg: TV/FA MD vs CG on the four 19x19 blurs, 256^2, 40 dB")
    rows, per_iter = [], {}
    for reg in ("tv", "frame"):
        name = "TV" if reg == "tv" else "FA"
        for i, blur in enumerate(WL.COMPARISON_BLURS):
            p = WL.comparison_problem(i, reg)
            y = torch.tensor(p.y, dtype=torch.float32, device="cuda")
            x = torch.zeros_like(y)
            with A.Plan([p]) as md, A.Plan([p], method=A.ADMM_METHOD_CG) as cg:
                md.solve(y, x, max_iters=max_iters, obj_tol=obj_tol, check_every=1, graph=True)   # graphs captured
                t_md, info_md = _solve_ms(md, y, x, max_iters=max_iters, obj_tol=obj_tol, check_every=1)
                f_md = info_md["objective"]

                def f_cg(K):
                    return cg.solve(y, x, max_iters=K, check_every=K, graph=True)["objective"]

                K = c
                while K <= max_iters and f_cg(K) > f_md:
                    K *= 2
                k_cg, t_cg = None, None
                if K <= max_iters:
                    lo, hi = (K // 2 if K > c else 0), K
                    while hi - lo > c:
                        mid = (lo + hi) // 2 // c * c
                        if mid <= lo:
                            break
                        if f_cg(mid) <= f_md:
                            hi = mid
                        else:
                            lo = mid
                    k_cg = hi
                    t_cg, info_cg = _solve_ms(cg, y, x, max_iters=k_cg, check_every=k_cg)
                if i == 0:
                    per_iter[f"{name}-MD"] = round(_us_per_iter(md, y, x), 2)
                    per_iter[f"{name}-CG"] = round(_us_per_iter(cg, y, x), 2)
            rows.append({"solver": name, "blur": blur, "md_iters": info_md["iters"], "md_converged": info_md["converged"],
                         "md_ms": round(t_md, 3), "md_objective": f_md, "cg_iters": k_cg,
                         "cg_ms": None if t_cg is None else round(t_cg, 3),
                         "cg_over_md_time": None if t_cg is None else round(t_cg / t_md, 3)})
            log(f"md_vs_cg: {name} {blur}: MD {info_md['iters']} it {t_md:.2f} ms, CG {k_cg} it "
                f"{t_cg if t_cg is None else round(t_cg, 2)} ms")
    ratios = {}
    for name in ("TV", "FA"):
        r = [q["cg_over_md_time"] for q in rows if q["solver"] == name and q["cg_over_md_time"] is not None]
        ratios[name] = round(float(np.mean(r)), 3) if r else None
    return {"workload": "TV and FA (J = 3) MD vs CG: 256x256 synthetic images, 19x19 out-of-focus / motion / "
                        "uniform / Gaussian blurs, valid region only, 40 dB BSNR, lambda 2e-4, mu by the rule of "
                        "Sec. V; MD until the objective changes by <= 1e-4 (relative) in an iteration, CG until "
                        "its objective reaches the MD one",
            "rows": rows, "mean_cg_over_md_time": ratios, "us_per_iter": per_iter,
            "cg_over_md_per_iter": {n: round(per_iter[f"{n}-CG"] / per_iter[f"{n}-MD"], 3) for n in ("TV", "FA")},
            "paper_context": "Table 4 (MATLAB, Core i5 2.39 GHz): 0.033 / 0.058 / 0.059 / 0.096 s per iteration "
                             "(TV-MD, TV-CG, FA-MD, FA-CG); Table 3: CG 1.5-2x the MD time"}


def run_c1(p, steps=5):
    import torch
    from paper_1210_2687_amd import admm as A
    log("c1: 128^2 TV-MD, 200 iterations")
    y = torch.tensor(p.y, dtype=torch.float32, device="cuda")
    x = torch.zeros_like(y)
    with A.Plan([p]) as plan:
        plan.solve(y, x, max_iters=200, graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = plan.solve(y, x, max_iters=200, graph=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
    return {"workload": "TV-MD 128x128, 9x9 uniform, valid 120x120, 200 iterations, cold start",
            "gpu_ms": round(dt * 1e3, 3), "value": round(p.y.size * 200 / dt / 1e6, 1), "unit": "Mpx*iter/s",
            "objective": info["objective"], "oracle": "FP64 oracle wall time: cpu_baseline.config1_oracle_s"}


def run_c3(p, tol=1e-4, max_iters=5000, c=10):
    import torch
    from paper_1210_2687_amd import admm as A
    log("c3: FA-MD 1024^2 J=3, time to tolerance 1e-4")
    y = torch.tensor(p.y, dtype=torch.float32, device="cuda")
    x = torch.zeros_like(y)
    with A.Plan([p], tune=True, cache_path=os.environ.get("ADMM_TUNE_CACHE")) as plan:
        plan.solve(y, x, max_iters=4 * c + 1, tol=tol, check_every=c, graph=True)    # graphs captured, untimed
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = plan.solve(y, x, max_iters=max_iters, tol=tol, check_every=c, graph=True)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        dt = float(np.median(times))
        kt = kernel_breakdown(plan, [y], [x], 50)
        dom = dominant_roofline(plan, [p], kt)
        # throughput at a fixed iteration count (graph replay), for the iteration roofline
        K = 400
        plan.solve(y, x, max_iters=K, graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.solve(y, x, max_iters=K, graph=True)
        torch.cuda.synchronize()
        us_it = (time.perf_counter() - t0) * 1e6 / K
    it = info["iters"]
    out = {"workload": "FA-MD 1024x1024, undecimated Haar J = 3, 13x13 disk r = 6, valid region minus 20% of 8x8 "
                       "blocks, sigma 1e-3, lambda 2e-4, mu 1e-3, tolerance 1e-4 on both residuals (checked every 10)",
           "time_to_tol_ms": round(dt * 1e3, 2), "iters": it, "converged": info["converged"],
           "r_pri": info["r_pri"], "r_dual": info["r_dual"], "objective": info["objective"],
           "value": round(p.y.size * it / dt / 1e6, 1), "unit": "Mpx*iter/s",
           "roofline_iteration": iteration_roofline([p], us_it), "roofline_dominant": dom,
           "kernel_us_event_per_launch": kt}
    log(f"c3: {it} iterations in {dt * 1e3:.1f} ms, iteration at {out['roofline_iteration']['frac']:.3f} of HBM peak")
    return out


def cnn_flops_per_px(train=False):
    """Multiply-adds x 2 of the warm-start network per pixel (forward), and of
    one training step (forward, input gradients of layers 2..6, weight gradients)."""
    from paper_1210_2687_amd.warmstart import CHANNELS
    layers = [(CHANNELS[i], CHANNELS[i + 1]) for i in range(len(CHANNELS) - 1)]
    fwd = sum(2 * 9 * ci * co for ci, co in layers)
    if not train:
        return fwd
    dgrad = sum(2 * 9 * ci * co for ci, co in layers[1:])
    return 2 * fwd + dgrad


def run_c5(train_probs, eval_probs, steps, target_batch=500, target_iters=3000):
    """Train the warm-start network on GPU-generated targets, then time cold and
    warm solves to tolerance 1e-4 on unseen problems."""
    import torch
    from paper_1210_2687_amd import warmstart as WS
    n_train, n_eval = len(train_probs), len(eval_probs)
    log(f"c5: targets for {n_train} problems of 256^2 (tol 1e-6, at most {target_iters} iterations)")
    t0 = time.perf_counter()
    parts, conv = [], 0
    for b in range(0, n_train, target_batch):
        y, m, e, xt, pt, infos = WS.targets(train_probs[b:b + target_batch], tol=1e-6, max_iters=target_iters)
        parts.append((y, m, e, xt, pt))
        conv += sum(i["converged"] for i in infos)
        if (b // target_batch) % 8 == 7:
            log(f"c5: targets {b + target_batch}/{n_train}")
    data = tuple(torch.cat([d[k] for d in parts]) for k in range(5))
    del parts
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    log(f"c5: targets done in {t_data:.1f} s ({conv}/{n_train} reached 1e-6); training {steps} steps")
    net = WS.WarmStartNet(seed=0)
    t0 = time.perf_counter()
    hist = WS.train(net, data, steps=steps, batch=8)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"c5: trained in {t_train:.1f} s, loss {np.mean(hist[:10]):.3e} -> {np.mean(hist[-10:]):.3e}")
    # network throughput: inference on 4 unseen 512^2 problems, one training step on 8 x 256^2
    y, m, e = WS.to_device(eval_probs[:4])
    for _ in range(2):
        net.predict(y, m, e)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        net.predict(y, m, e)
    torch.cuda.synchronize()
    fwd_s = (time.perf_counter() - t0) / reps
    fwd_tf = cnn_flops_per_px() * y.numel() / fwd_s / 1e12
    ii = torch.arange(8, device="cuda")
    batch = [t[ii].contiguous() for t in data]
    net.train_step(*batch, lr=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.train_step(*batch, lr=0.0, want_loss=False)
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / reps
    step_tf = cnn_flops_per_px(train=True) * batch[0].numel() / step_s / 1e12
    del data, batch
    log(f"c5: timing cold and warm solves of {n_eval} unseen problems of 512^2")
    rows = WS.evaluate(net, eval_probs, log=log)
    s = WS.summary(rows)
    s.update({"workload": "learned warm start (6 conv3x3 layers, 32 channels, BF16 MFMA) vs cold start, TV-MD",
              "tol": 1e-4, "check_every": 10, "eval": f"{n_eval} unseen 512x512 problems, one at a time",
              "train": f"{n_train} problems 256x256, targets from the GPU ADMM (tol 1e-6, at most {target_iters} "
                       f"iterations; {conv} reached it), {steps} Adam steps of 8",
              "targets_s": round(t_data, 1), "train_s": round(t_train, 1),
              "final_objective_check": "cold and warm continued to tolerance 5e-6 (batches of 64)",
              "net_params": net.nparams, "loss_first_last": [float(np.mean(hist[:10])), float(np.mean(hist[-10:]))],
              "cnn_fwd_tflops": round(fwd_tf, 2), "cnn_train_step_tflops": round(step_tf, 2),
              "bf16_peak_tflops": 2500.0, "timing": "wall clock per problem; warm includes the network and the "
                                                    "state mapping; both solve on a hipGraph"})
    log(f"c5: p50 cold {s['p50_cold_ms']:.1f} ms, warm {s['p50_warm_ms']:.1f} ms ({s['p50_speedup']:.2f}x)")
    return s


# ------------------------------------------------------------------ CPU baseline (the oracle)
def cpu_baseline(iters, sample, c1=None, c3=None, c4=None):
    """The FP64 oracle on a bounded sample of the headline workload (and, if
    given, the whole 128^2 workload: its headline is the oracle's wall time; 5
    iterations of the FA-MD 1024^2 problem; 5 iterations of 4 problems of the
    ragged batch, extrapolated to the batch)."""
    import oracle as O
    try:
        import threadpoolctl
        cores = max(i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()) or os.cpu_count()
    except Exception:
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    log(f"cpu baseline: FP64 oracle on {len(sample)} images x {iters} iterations")
    t0 = time.perf_counter()
    for p in sample:
        O.tv_md_run(p.y, p.mask, p.kernel, p.lam, p.mu1, p.mu2, iters=iters)
    dt = time.perf_counter() - t0
    px_it = sum(p.y.size for p in sample) * iters
    shapes = ", ".join(f"{p.shape[0]}x{p.shape[1]}" for p in sample)
    out = {"value": px_it / dt / 1e6, "unit": "Mpx*iter/s", "cores": int(cores), "kind": "oracle",
           "sample": f"{len(sample)} of the 8 headline images (one 19x19 Gaussian, one 15-px motion) ({shapes}), "
                     f"{iters} iterations each, {dt:.1f} s"}
    if c1 is not None:
        t0 = time.perf_counter()
        O.tv_md_run(c1.y, c1.mask, c1.kernel, c1.lam, c1.mu1, c1.mu2, iters=200)
        out["config1_oracle_s"] = round(time.perf_counter() - t0, 3)
        out["config1"] = "TV-MD 128x128, 9x9 uniform, 200 iterations, the whole run"
    if c3 is not None:
        t0 = time.perf_counter()
        O.fa_md_run(c3.y, c3.mask, c3.kernel, c3.lam, c3.mu1, c3.mu2, c3.levels, iters=5)
        dt = time.perf_counter() - t0
        out["fa1024"] = {"value": round(c3.y.size * 5 / dt / 1e6, 3), "unit": "Mpx*iter/s",
                          "s_per_iter": round(dt / 5, 3),
                          "sample": f"FA-MD {c3.shape[0]}x{c3.shape[1]}, J = {c3.levels}, 5 iterations"}
    if c4:
        sub = c4[:4]
        t0 = time.perf_counter()
        for p in sub:
            O.tv_md_run(p.y, p.mask, p.kernel, p.lam, p.mu1, p.mu2, iters=5)
        dt = time.perf_counter() - t0
        rate = sum(p.y.size for p in sub) * 5 / dt
        out["ragged256"] = {"value": round(rate / 1e6, 3), "unit": "Mpx*iter/s",
                          "extrapolated_s_per_iter": round(sum(p.y.size for p in c4) / rate, 2),
                          "sample": "TV-MD, the first 4 of the 256 ragged problems ("
                                    + ", ".join(f"{p.shape[0]}x{p.shape[1]}" for p in sub)
                                    + "), 5 iterations each; the batch's time per iteration extrapolated by its "
                                      "pixel count"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tv8x512",
                    choices=["tv8x512", "tv64x512", "tv4096", "tv8192", "tv16384", "fa1024", "fs1024", "ragged256", "md_vs_cg",
                             "tv8x512_cg"],
                    help="the headline is tv8x512; with --quick, the others run alone (profiling)")
    ap.add_argument("--quick", action="store_true", help="only the chosen workload, no other configs")
    ap.add_argument("--iters", type=int, default=500, help="ADMM iterations per headline step")
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--cpu-iters", type=int, default=100, help="oracle iterations per sampled headline image")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ws-train", type=int, default=20000, help="warm-start training problems (256x256; 0: skip)")
    ap.add_argument("--ws-steps", type=int, default=8000, help="warm-start Adam steps of 8")
    ap.add_argument("--ws-eval", type=int, default=512, help="warm-start evaluation problems (512x512)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--c3-max-iters", type=int, default=5000,
                    help="iteration cap of the FA 1024^2 time-to-tolerance solves (a small cap shortens profiled runs)")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the planner's heuristic tile shapes instead of the autotuner (which runs at plan time, "
                         "outside the timed region; ADMM_TUNE_CACHE names an optional JSON cache)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes (HBM counter calibration)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))
        return

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (--gpus {args.gpus} requested); "
              "problems shard across GPUs by whole images, which is not measured here.", file=sys.stderr)
        sys.exit(2)

    data = host_data(args)

    import torch
    from paper_1210_2687_amd import admm as A
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    A.lib()   # fail loudly if the HIP library is missing
    tune = not args.no_tune
    graph = not args.no_graph

    configs = {}
    if args.quick and args.workload != "tv8x512":
        # one other workload alone, for profiling
        if args.workload == "fa1024":
            configs["c3"] = run_c3(data["c3"], max_iters=args.c3_max_iters)
        elif args.workload == "fs1024":
            configs["c3_fs"] = run_throughput("c3_fs", [data["c3_fs"]], 400, args.steps, args.warmup, tune,
                                              "FS-MD on the FA 1024x1024 J = 3 data, 400 iterations")
        elif args.workload == "tv4096":
            configs["tv4096"] = run_throughput("tv4096", data["c_big"], 100, args.steps, args.warmup, tune,
                                               "TV-MD 4096x4096, 100 iterations")
        elif args.workload == "tv16384":
            configs["tv16384"] = run_throughput("tv16384", data["c_16k"], 10, args.steps, args.warmup, tune,
                                                "TV-MD 16384x16384 (a 4096^2 image tiled 4 x 4), 10 iterations")
        elif args.workload == "tv8192":
            configs["tv8192"] = run_throughput("tv8192", data["c_huge"], 20, args.steps, args.warmup, tune,
                                               "TV-MD 8192x8192, 20 iterations")
        elif args.workload == "md_vs_cg":
            configs["md_vs_cg"] = run_md_vs_cg()
        elif args.workload == "tv8x512_cg":
            configs["headline_cg"] = run_throughput("headline_cg", data["c2"], args.iters, args.steps, args.warmup,
                                                    tune, f"TV-CG on the headline batch, {args.iters} iterations",
                                                    method=A.ADMM_METHOD_CG)
        elif args.workload == "ragged256":
            configs["c4"] = run_throughput("c4", data["c4"], 200, args.steps, args.warmup, tune,
                                           "TV-MD ragged batch of 256 problems, sides 128..1024 (7-smooth), "
                                           "kernels 5..31, 200 iterations")
        else:
            configs["beyond_cache"] = run_throughput("beyond_cache", data["c64"], 500, args.steps, args.warmup, tune,
                                                     "TV-MD batch of 64 x 512x512, 500 iterations")
        print(json.dumps({"metric": METRIC, "configs": configs}), flush=True)
        return

    # ---- headline
    probs = data["c2"]
    log(f"headline: TV-MD batch of {args.batch} x {args.size}^2, {args.iters} iterations, "
        f"{args.warmup} warm-up + {args.steps} timed steps")
    plan, ys, xs, r = timed_batch(probs, args.iters, args.steps, args.warmup, tune, graph)
    kt = kernel_breakdown(plan, ys, xs, min(args.iters, 100))
    roofline = dominant_roofline(plan, probs, kt)
    traffic = read_traffic(kernel_source_hash()) if roofline["kernel"] == "row_tv" else None
    roofline["traffic"] = traffic
    roofline["kernel_us_event_per_launch"] = kt
    roofline_it = iteration_roofline(probs, r["us_per_iter"])
    plan.close()
    log(f"headline: {r['value']:.1f} Mpx*iter/s; {roofline['kernel']} at {roofline['frac']:.3f}, "
        f"iteration at {roofline_it['frac']:.3f} of HBM peak")

    if not args.quick:
        configs["c1"] = run_c1(data["c1"])
        configs["c3"] = run_c3(data["c3"])
        configs["beyond_cache"] = run_throughput("beyond_cache", data["c64"], 500, 3, 1, tune,
                                                 "TV-MD batch of 64 x 512x512 (the 8 headline images repeated), "
                                                 "500 iterations")
        configs["c3_fs"] = run_throughput("c3_fs", [data["c3_fs"]], 400, 3, 1, tune,
                                          "FS-MD (frame synthesis, eq. (35)) on the FA 1024x1024 J = 3 data, "
                                          "400 iterations")
        configs["headline_cg"] = run_throughput("headline_cg", probs, args.iters, 3, 1, tune,
                                                f"TV-CG (Reeves-Sorel, one CG step) on the headline batch of "
                                                f"{args.batch} x {args.size}^2, {args.iters} iterations",
                                                method=A.ADMM_METHOD_CG)
        configs["md_vs_cg"] = run_md_vs_cg()
        configs["tv4096"] = run_throughput("tv4096", data["c_big"], 100, 3, 1, tune,
                                           "TV-MD 4096x4096 (the headline image family: 19x19 Gaussian sigma 3, 40% "
                                           "missing), 100 iterations: block-level column pass and three-pass TV rows")
        configs["c4"] = run_throughput("c4", data["c4"], 200, 2, 1, tune,
                                       "TV-MD ragged batch of 256 problems, sides 128..1024 (7-smooth), kernels "
                                       "Gaussian/uniform/motion 5..31, lambda log-uniform 1e-5..1e-3, 200 iterations")
        if args.ws_train:
            configs["c5"] = run_c5(data.pop("c5_train"), data.pop("c5_eval"), args.ws_steps)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_iters, [probs[0], probs[4 % len(probs)]], None if args.quick else data["c1"],
                           data.get("c3"), data.get("c4"))

    config = {"workload": f"TV-MD batch of {args.batch} x {args.size}x{args.size}, {args.iters} iterations",
              "batch": args.batch, "H": args.size, "W": args.size, "iters": args.iters,
              "kernels": "19x19 Gaussian sigma 3 (4) + 15-px motion (4)",
              "mask": "valid region minus 40% i.i.d. missing", "graph": graph, "tiles": r["tiles"]}
    out = {
        "metric": METRIC, "value": round(r["value"], 1), "unit": "Mpx*iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": config,
        "roofline": roofline, "roofline_iteration": roofline_it, "cpu_baseline": cpu, "configs": configs,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
