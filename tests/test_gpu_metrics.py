"""GPU: clinical metrics of the plans on a dose grid (Sec. 2.A) against the
oracle's definitions, from the same shot times."""
import sys

import numpy as np
import pytest

from synth import cases
from oracle import metrics as om

pytestmark = pytest.mark.gpu

ladmm = pytest.importorskip("paper_2509_08602_amd.ladmm")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_metrics_match_oracle_c0():
    say("clinical metrics c0 f64")
    case = cases.make_case(0)
    w = cases.config_weights(0)
    k = w.shape[0]
    ctx = ladmm.Context(0)
    dc = ladmm.Case.from_case(ctx, case, "f64")
    b = ladmm.Batch(dc, w, opts=ladmm.Options(max_iter=4000, check_every=50, tol_gap=1e-3,
                                              tol_pri=1e-3, tol_dual=1e-3, rho0=1e4,
                                              w0_bot=cases.W0_BOT))
    b.run()
    # dose grid: the box around the target with a 10 mm margin, 1 mm voxels
    types = case.point_types()
    tcoords = case.coords[(types == cases.TS) | (types == cases.TI)]
    lo, hi = tcoords.min(axis=0) - 10, tcoords.max(axis=0) + 10
    axes = [np.arange(a, z + 1) for a, z in zip(lo, hi)]
    grid = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.int32)
    inside = {tuple(v) for v in tcoords.tolist()}
    tgt = np.array([0 if tuple(v) in inside else -1 for v in grid.tolist()], np.int32)
    phi = case.kernel.dose_rate(grid)
    D = case.prescription_mean
    got = b.metrics(phi, tgt, [D], D)
    t = b.results()["t"].T
    b.close()
    dc.close()
    ref = om.clinical_metrics(phi, t, tgt, [D], D, case.n_iso, case.n_sectors, case.n_collimators)
    say("grid voxels", len(grid), "target voxels", int((tgt >= 0).sum()))
    say("coverage", got[:, 0], "selectivity", got[:, 1], "gradient index", got[:, 2],
        "beam-on", got[:, 3])
    # a voxel whose dose lies within rounding of a threshold may count on either side
    d = om.grid_dose(phi, t)
    near = lambda thr: (np.abs(d - thr) <= 1e-9 * thr).sum(axis=0)
    n_t, piv = (tgt >= 0).sum(), (d >= D).sum(axis=0)
    assert np.all(np.abs(got[:, 0] - ref[:, 0]) <= near(D) / n_t + 1e-12)
    assert np.all(np.abs(got[:, 1] - ref[:, 1]) <= 2 * near(D) / np.maximum(piv - near(D), 1) + 1e-12)
    assert np.all(np.abs(got[:, 2] - ref[:, 2]) <= 2 * (near(D) + near(D / 2)) / np.maximum(piv - near(D), 1) + 1e-12)
    assert np.allclose(got[:, 3], ref[:, 3], rtol=1e-12)
    assert np.all((got[:, 0] > 0) & (got[:, 0] <= 1) & (got[:, 1] <= 1) & (got[:, 2] >= 1))
