"""Plain FP64 CPU oracle for mask-decoupled ADMM deconvolution.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or link
this package: only the test suite, the smoke check in ``__graft_entry__`` and
the ``cpu_baseline`` leg of ``bench.py`` use it. It shares no code with the HIP
library (no kernels, tables, constants or pre/post-processing).

What it computes follows Almeida & Figueiredo, "Deconvolving Images with
Unknown Boundaries Using the Alternating Direction Method of Multipliers":

* observation model y = M A x + n              (Sec. IV-A, eq. (34))
* TV-MD: Alg. 3 (ADMM-TV) with the data-term update of eq. (49)  (Sec. IV-D)
* FA-MD: Alg. 2 (ADMM-2) with H1 = A, H2 = P, the z-step of eqs. (24)-(25)
  and the proximity operators of eqs. (40) and (16)                (Sec. IV-C)
* TV-CG / FA-CG: the Reeves-Sorel variants with H1 = M A, the z-step by the
  Sherman-Morrison-Woodbury split and one warm-started conjugate-gradient
  iteration on the boundary system                         (Sec. IV-B..IV-D)
* FS-MD: frame synthesis, Alg. 2 with H1 = A W, H2 = I, the z-step of
  eq. (17) by eqs. (18) and (20)                                  (Sec. IV-C)

Design rules: the convolution A and its adjoint are direct spatial sums over
kernel taps, the z-step uses a naive dense-matrix DFT (never ``np.fft``), all
arithmetic is float64, and the steps run in the paper's order and notation.

Parity status per function is listed in each module header; every public
function is pinned by ``tests/test_oracle_*.py`` (none is "parity unpinned").
"""

from .operators import (
    conv_A, conv_At, diff_h, diff_v, diff_ht, diff_vt,
    dft_matrix, dft2, idft2, kernel_spectrum, diff_spectra,
    haar_analysis, haar_synthesis, haar_num_bands,
)
from .prox import mask_prox, vsoft, soft
from .admm import (
    TVState, FAState, tv_md_step, tv_md_run, fa_md_step, fa_md_run,
    tv_objective, fa_objective, tv_residuals, fa_residuals,
    warm_start_state, zsolve_tv, zsolve_fa, default_mu,
)
from .cg import (
    TVCGState, FACGState, tv_cg_step, tv_cg_run, fa_cg_step, fa_cg_run, boundary_cg, cg_zsolve,
)
from .fs import FSState, fs_zsolve, fs_md_step, fs_md_run, fs_objective, fs_residuals
from .cnn import conv3x3_fwd, conv3x3_dgrad, conv3x3_wgrad, relu, adam_step

__all__ = [
    "conv_A", "conv_At", "diff_h", "diff_v", "diff_ht", "diff_vt",
    "dft_matrix", "dft2", "idft2", "kernel_spectrum", "diff_spectra",
    "haar_analysis", "haar_synthesis", "haar_num_bands",
    "mask_prox", "vsoft", "soft",
    "TVState", "FAState", "tv_md_step", "tv_md_run", "fa_md_step", "fa_md_run",
    "tv_objective", "fa_objective", "tv_residuals", "fa_residuals",
    "warm_start_state", "zsolve_tv", "zsolve_fa", "default_mu",
    "TVCGState", "FACGState", "tv_cg_step", "tv_cg_run", "fa_cg_step", "fa_cg_run", "boundary_cg", "cg_zsolve",
    "FSState", "fs_zsolve", "fs_md_step", "fs_md_run", "fs_objective", "fs_residuals",
    "conv3x3_fwd", "conv3x3_dgrad", "conv3x3_wgrad", "relu", "adam_step",
]
