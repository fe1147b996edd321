"""Helpers shared by the GPU tests (no test functions here)."""

import numpy as np


def dev(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda").contiguous()


def host(t):
    return t.detach().to("cpu").double().numpy()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def check_iterate(z, ref, tol=1e-4, what=""):
    """The per-iterate bar: relative L2 error <= tol and every element within
    tol * max|ref| (one bad pixel fails the second even when the norm hides it).
    Returns (relative L2 error, largest element error over max|ref|)."""
    z = np.asarray(z, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    e2 = rel(z, ref)
    scale = np.max(np.abs(ref))
    einf = np.max(np.abs(z - ref)) / (scale if scale > 0 else 1.0)
    announce(f"  {what} rel L2 {e2:.3e}, max elem {einf:.3e}")
    assert np.all(np.isfinite(z)), what
    assert e2 <= tol and einf <= tol, (what, e2, einf)
    return e2, einf


def full_problem(seed, H, W, k, family="gaussian", missing=0.3, lam=2e-4, mu=0.01, reg="tv", levels=0):
    """A problem on a non-periodic synthetic image with a full spectrum (shapes,
    a smooth random field and noise), a k x k blur and i.i.d. missing pixels."""
    from paper_1210_2687_amd import workloads as WL
    g = WL.rng(seed)
    x = WL.synth_image(g, H, W, grf_scale=32.0)
    if family == "gaussian":
        h = WL.kernel_gaussian(k, k / 6.0)
    elif family == "uniform":
        h = WL.kernel_uniform(k)
    else:
        h = WL.kernel_motion(k, float(k), g.uniform(0, np.pi))
    m = WL.valid_mask(H, W, k // 2)
    m &= (g.uniform(size=(H, W)) >= missing).astype(np.uint8)
    y = WL.observe(g, x, h, m, 2e-3)
    return WL.Problem(y=y, mask=m, kernel=h, lam=lam, mu1=mu, mu2=mu, x_true=x, reg=reg, levels=levels)


def gpu_solve(plan, prob, iters, state=None, tol=0.0, check_every=10, graph=False, obj_tol=0.0):
    import torch
    y = dev(prob.y)
    x = torch.zeros_like(y)
    info = plan.solve(y, x, state, max_iters=iters, tol=tol, check_every=check_every, graph=graph, obj_tol=obj_tol)
    return host(x), info


def announce(msg):
    print(msg, flush=True)


def fast_tv_problem(seed, H=64, W=64, k=7, lam=2e-4, mu=0.01, missing=0.2):
    """A TV problem whose ADMM reaches residuals of 1e-4 in a few hundred iterations
    (penalties balanced for speed; the minimiser does not depend on them)."""
    from paper_1210_2687_amd import workloads as WL
    g = WL.rng(seed)
    x = WL.synth_image(g, H, W, grf_scale=16.0)
    h = WL.kernel_gaussian(k, k / 4.5)
    m = WL.valid_mask(H, W, k // 2)
    m &= (g.uniform(size=(H, W)) >= missing).astype(np.uint8)
    y = WL.observe(g, x, h, m, 2e-3)
    return WL.Problem(y=y, mask=m, kernel=h, lam=lam, mu1=mu, mu2=mu, x_true=x)
