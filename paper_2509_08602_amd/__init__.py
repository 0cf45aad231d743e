"""Batched ADMM for Gamma Knife plan optimisation on MI355X (gfx950).

The solver lives in the HIP library libladmm.so (C ABI in include/ladmm.h);
`paper_2509_08602_amd.ladmm` is its ctypes binding.
"""
from . import ladmm  # noqa: F401
from .ladmm import Batch, Case, Context, LadmmError, Options, solve_batch  # noqa: F401
