"""MI355X-native mask-decoupled ADMM deconvolution (images with unknown boundaries).

The compute path is the HIP library ``libadmmdeconv.so`` built from ``csrc/``
for gfx950; ``paper_1210_2687_amd.admm`` is its thin ctypes binding. Importing
this package loads nothing: the binding loads the library on first use and
raises if it is missing (there is no CPU fallback).
"""

__all__ = ["admm", "workloads"]
