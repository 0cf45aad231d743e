"""Dose of a plan at arbitrary voxels and the low-dose band of Sec. 2.C.1.

Oracle code (test infrastructure).  The dose of plan j at a voxel is the sum of
the dose-rate kernels weighted by the plan's shot times, d_j(v) = phi(v) t_j.
The second-pass low-dose volume of plan j is the set of candidate voxels whose
first-pass dose lies in [D_LD, D_LD + Delta).
"""
from __future__ import annotations

import numpy as np


def dose(phi_vox: np.ndarray, t: np.ndarray) -> np.ndarray:
    """d = phi t in FP64: (M x n_t) times (n_t x k) -> M x k."""
    return np.asarray(phi_vox, np.float64) @ np.asarray(t, np.float64).reshape(phi_vox.shape[1], -1)


def ld_band(d: np.ndarray, d_ld: float, delta: float) -> np.ndarray:
    """k x M bool: True where D_LD <= d_j(v) < D_LD + Delta."""
    d = np.asarray(d, np.float64)
    return ((d >= d_ld) & (d < d_ld + delta)).T
