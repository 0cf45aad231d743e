"""Clinical plan metrics of Sec. 2.A, from the dose on a voxel grid.

Oracle code (test infrastructure).  Sec. 2.A defines, for one target with
prescription D_T and the plan's dose d on the patient volume:

    coverage       = fraction of the target volume receiving at least D_T,
    selectivity    = fraction of the volume receiving at least D_T that lies
                     in the target,
    gradient index = volume receiving at least D_T / 2 over the volume
                     receiving at least D_T,
    beam-on time   = total irradiation time of the plan.

Volumes are voxel counts on a grid of equal voxels.  With several targets a
voxel of target i is covered when it receives its own prescription D_i, and the
prescription volume uses a reference dose d_ref (the common prescription; the
paper leaves the gradient index out when prescriptions differ, Sec. 3.B).  The
beam-on time of an isocentre is the longest of its sectors' summed shot times
(the sectors irradiate in parallel, the collimator sizes of a sector one after
another); the plan's is the sum over isocentres.
"""
from __future__ import annotations

import numpy as np


def grid_dose(phi_vox, t):
    """d = phi_vox t: n_vox x k doses for shot times t (n_t x k)."""
    return np.asarray(phi_vox, np.float64) @ np.asarray(t, np.float64)


def beam_on_time(t, n_iso, sectors, collimators):
    """Sum over isocentres of the longest summed sector time (t: n_t x k)."""
    t = np.asarray(t, np.float64)
    k = t.shape[1]
    return t.reshape(n_iso, sectors, collimators, k).sum(axis=2).max(axis=1).sum(axis=0)


def clinical_metrics(phi_vox, t, vox_target, presc, d_ref, n_iso, sectors, collimators):
    """k x 4 array: coverage, selectivity, gradient index, beam-on time (NaN where a
    denominator is zero).  vox_target: target index per voxel, -1 outside."""
    t = np.asarray(t, np.float64).reshape(n_iso * sectors * collimators, -1)
    d = grid_dose(phi_vox, t)
    tgt = np.asarray(vox_target)
    inside = tgt >= 0
    D = np.where(inside, np.asarray(presc, np.float64)[np.maximum(tgt, 0)], np.inf)
    covered = ((d >= D[:, None]) & inside[:, None]).sum(axis=0).astype(np.float64)
    piv = (d >= d_ref).sum(axis=0).astype(np.float64)
    piv_half = (d >= 0.5 * d_ref).sum(axis=0).astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        coverage = covered / inside.sum() if inside.any() else np.full(t.shape[1], np.nan)
        selectivity = np.where(piv > 0, covered / piv, np.nan)
        gradient = np.where(piv > 0, piv_half / piv, np.nan)
    bot = beam_on_time(t, n_iso, sectors, collimators)
    return np.stack([coverage, selectivity, gradient, bot], axis=1)
