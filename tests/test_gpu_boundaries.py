"""Unknown boundaries (MD) against periodic boundaries (BC, and BC on edge-tapered data, ET).

The paper's claim (Sec. V): posing the deconvolution on the unknown domain
with a mask over the observed (valid) region avoids the boundary artifacts
of a periodic model of the observed region alone; edge tapering the data
first reduces but does not remove them. The BC and ET problems are the same
library with M = I on the observed domain (Sec. IV-A: with M = I the method
reduces to the periodic-boundary ADMM). All three are checked against the
oracle at a small size, then compared by ISNR on the observed region at
480^2 (unknown domain 504^2, 25 x 25 kernels), for TV and for the frame
(J = 3); the paper's images are not available, so the synthetic family of
the other workloads stands in.
"""

import numpy as np
import pytest

import oracle as O
from paper_1210_2687_amd import admm as A
from paper_1210_2687_amd import workloads as WL
from gpu_util import rel, gpu_solve, announce

pytestmark = pytest.mark.gpu

ITER_TOL = 1e-4


def isnr(x_obs, y_obs, x_hat):
    return 10.0 * np.log10(np.sum((y_obs - x_obs) ** 2) / np.sum((x_hat - x_obs) ** 2))


def _oracle(p, K):
    if p.reg == "frame":
        return O.fa_md_run(p.y, p.mask, p.kernel, p.lam, p.mu1, p.mu2, p.levels, iters=K)["z"]
    return O.tv_md_run(p.y, p.mask, p.kernel, p.lam, p.mu1, p.mu2, iters=K)["z"]


@pytest.mark.parametrize("family,reg", [("uniform", "tv"), ("motion", "tv"), ("uniform", "frame")])
def test_md_bc_et_models_match_oracle(family, reg):
    md, bc, et, _, _ = WL.boundary_pair(2, observed=96, family=family, reg=reg, levels=2)
    K = 40
    for name, p in (("MD", md), ("BC", bc), ("ET", et)):
        with A.Plan([p]) as plan:
            z, info = gpu_solve(plan, p, K)
        e = rel(z, _oracle(p, K))
        announce(f"{family} {reg} {name} {p.shape}: k={K} rel err {e:.3e}")
        assert info["iters"] == K
        assert e <= ITER_TOL


@pytest.mark.parametrize("family,reg", [("uniform", "tv"), ("gaussian", "tv"), ("motion", "tv"),
                                        ("uniform", "frame")])
def test_unknown_boundaries_beat_periodic_boundaries(family, reg):
    md, bc, et, x_obs, y_obs = WL.boundary_pair(0, family=family, reg=reg)
    l = md.kernel.shape[0] // 2
    out = {}
    for name, p in (("MD", md), ("BC", bc), ("ET", et)):
        with A.Plan([p]) as plan:
            z, info = gpu_solve(plan, p, 6000, tol=1e-4, check_every=10, graph=True)
        if name == "MD":
            z = z[l:-l, l:-l]
        out[name] = isnr(x_obs, y_obs, z)
        announce(f"{family} {reg} {name} {p.shape}: ISNR {out[name]:.2f} dB, {info['iters']} iterations, "
                 f"converged {info['converged']}")
    assert out["MD"] > 0.0
    assert out["MD"] >= out["ET"] + 1.0
    assert out["ET"] >= out["BC"] + 3.0
