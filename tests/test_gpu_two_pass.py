"""GPU parity of the two-pass optimisation (Sec. 2.C) against the oracle.

Pass 1 is checked through its own results; the second-pass point set must be
exactly what the oracle's band + Algorithm 1 give from the same pass-1 shot
times (bit-exact index sets), and each converged pass-2 plan's objective must
match the exact optimum of the second-pass LP built by the oracle from that
point set and those per-plan subsets.
"""
import sys

import numpy as np
import pytest

from synth import cases
from oracle import lp as olp
from oracle import alg1 as oalg1
from oracle import dose as odose
from oracle.simplex import solve_plan

pytestmark = pytest.mark.gpu

ladmm = pytest.importorskip("paper_2509_08602_amd.ladmm")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_two_pass_c0_matches_oracle():
    say("two-pass c0 f64")
    case = cases.make_case(0)
    w = cases.config_weights(0)
    k = w.shape[0]
    ld_group = [g.type for g in case.groups].index(cases.LD)
    cand = case.ld_candidates
    phi = case.kernel.dose_rate(cand)
    d_ld, delta = 0.5 * case.prescription_mean, 0.1 * case.prescription_mean
    n_ld = np.full(k, 500)
    opts = ladmm.Options(max_iter=8000, check_every=50, tol_gap=1e-4, tol_pri=1e-4,
                         tol_dual=1e-4, rho0=1000.0, w0_bot=cases.W0_BOT, adapt_rho=False)
    ctx = ladmm.Context(0)
    r1, r2, P, n2, times = ladmm.two_pass(ctx, case, w, phi, d_ld, delta, n_ld, 12345, ld_group,
                                          "f64", opts)
    say("times ms", times, "|P|", len(P), "N2", n2)
    # band + Algorithm 1 from the pass-1 shot times, in the oracle
    vols = odose.ld_band(odose.dose(phi, r1["t"].T), d_ld, delta)
    assert vols.any(axis=1).all()
    Pref, pref = oalg1.select_ld_points(vols, n_ld, 12345)
    assert P.tolist() == Pref
    masks_P = oalg1.masks_over(Pref, pref)
    # the second-pass LP: non-LD points of pass 1 and the new LD points
    keep = np.nonzero(case.group != ld_group)[0]
    case2 = case.with_points(keep, extra_ld=cand[np.array(Pref)], ld_group=ld_group)
    assert case2.n_points == n2
    mask2 = np.zeros((k, n2), bool)
    mask2[:, len(keep):] = masks_P
    lp2 = olp.assemble(case2, w, mask2)
    Fstar = np.array([-solve_plan(lp2, j).objective for j in range(k)])
    F2 = olp.planning_objective(case2, w, r2["t"].T, mask2)[0]
    assert np.max(np.abs(F2 - r2["objective"]) / Fstar) < 1e-9
    rel = np.abs(r2["objective"] - Fstar) / Fstar
    say("pass-2 rel err", rel, "status", r2["plan_status"], "iters", r2["iters"])
    assert np.all(rel < 1e-3), rel
