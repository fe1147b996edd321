"""Reader of the golden trajectory fixtures under tests/golden (no test functions here)."""

import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NAMES = ("tv_md_5x6", "fa_md_4x6_J2", "tv_md_8x10", "fa_md_8x8_J3")
CG_NAMES = ("tv_cg_5x6", "fa_cg_4x6_J2")
FS_NAMES = ("fs_md_4x6_J2",)


def load(name):
    """Parse ``tests/golden/<name>.txt``: inputs as float64 arrays (exact: dyadic
    fractions), the stored iterates z_k, the (r_pri, r_dual) residuals of the
    recorded iterations k >= 2 and the objective at the last iterate."""
    out = {"zs": {}, "residuals": {}}
    with open(os.path.join(GOLDEN, name + ".txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            if key == "z":
                out["zs"][int(vals[0])] = np.array([float(v) for v in vals[1:]])
            elif key == "residual":
                out["residuals"][int(vals[0])] = (float(vals[1]), float(vals[2]))
            elif key == "objective":
                out["objective"] = (int(vals[0]), float(vals[1]))
            elif key in ("reg", "method"):
                out[key] = vals[0]
            elif key in ("levels", "iters"):
                out[key] = int(vals[0])
            elif key == "shape":
                out["shape"] = (int(vals[0]), int(vals[1]))
            elif key in ("lambda", "mu1", "mu2"):
                out[key] = float(Fraction(vals[0]))
            else:
                out[key] = np.array([float(Fraction(v)) for v in vals])
    H, W = out["shape"]
    k = int(round(np.sqrt(out["kernel"].size)))
    out["kernel"] = out["kernel"].reshape(k, k)
    out["mask"] = out["mask"].reshape(H, W).astype(np.uint8)
    out["y"] = out["y"].reshape(H, W)
    out["zs"] = {kk: v.reshape(H, W) for kk, v in out["zs"].items()}
    return out
