"""GPU, large case (200,000 dose points x 4,800 shot columns, 441 plans).

The exact LP optimum is out of reach of the oracle's simplex at this size, so
every plan's result is checked against what the FP64 oracle can certify from
the GPU's own iterates: U = F(t) of the returned shot times (made
OAR-feasible) is an upper bound on F*, and L = -c'x_hat from the returned dual
iterate z1 (clipped and scaled to feasibility, App. A duality) is a lower
bound, so (U - L) / U bounds the relative error of the objective against the
exact optimum.  Both bounds are computed in FP64 on the host by the oracle.

The solve stops each plan on the device's own certified gap (the same dual
point, evaluated in the iteration precision) at 9e-4, together with the plain
gap and the residuals; the oracle's FP64 certificate must then show every plan
within 1e-3 of F*, and its FP64 residuals, recomputed from the final iterates
with the plans' final step sizes, must be within 1e-4.
"""
import json
import os
import sys
import time

import numpy as np
import pytest

from synth import cases
from oracle import lp as olp
from oracle import admm as oadmm

pytestmark = pytest.mark.gpu

ladmm = pytest.importorskip("paper_2509_08602_amd.ladmm")
# per-plan bounds are also written as JSON into this directory when it is set
OUT = os.environ.get("LADMM_RESULT_DIR")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["bf16"])
def test_large_case_every_plan_within_1e3_of_optimum(precision):
    t0 = time.time()
    case = cases.make_case(2)
    w = cases.config_weights(2)
    k = w.shape[0]
    N = case.n_points
    say(f"large case built {time.time() - t0:.1f} s: N={N} n_t={case.n_t} k={k}")
    ctx = ladmm.Context(0)
    dc = ladmm.Case.from_case(ctx, case, precision)
    opts = ladmm.Options(max_iter=20000, check_every=50, tol_gap=1e-4, tol_pri=5e-5,
                         tol_dual=5e-5, tol_cert=9e-4, rho0=1e4, w0_bot=cases.W0_BOT,
                         adapt_rho=True)
    b = ladmm.Batch(dc, w, opts=opts)
    t1 = time.time()
    b.run()
    solve_s = time.time() - t1
    res = b.results()
    z1, y1, z2, y2 = b.export()
    rho = b.step_sizes()
    b.close()
    dc.close()
    conv = res["plan_status"] == ladmm.PLAN_CONVERGED
    say(f"{precision} solve {solve_s:.1f} s, iterations max {res['iters'].max()} "
        f"median {np.median(res['iters'])}, converged {int(conv.sum())}/{k}, device cert gap "
        f"max {np.nanmax(res['cert_gap']):.2e}")
    t2 = time.time()
    lp = olp.assemble(case, w)
    cert = olp.certify(case, w, res["t"].T, z1[:N], lp=lp)
    say(f"oracle bounds {time.time() - t2:.1f} s")
    U, L, gap = cert["U"], cert["L"], cert["cert_gap"]
    # FP64 residuals of the final iterate: one oracle step from it
    t3 = time.time()
    slp = olp.precondition(lp, olp.bot_scale(case))
    del lp
    fac, _ = oadmm.schur_factor(slp)
    nxt = oadmm.admm_iterate(slp, rho, 1, oadmm.ADMMState(z1, y1, z2, y2), fac)
    r_pri, r_dual = oadmm.residuals(slp, rho, nxt)
    say(f"oracle residuals {time.time() - t3:.1f} s: r_pri max {r_pri.max():.2e}, "
        f"r_dual max {r_dual.max():.2e}")
    rel_F = np.abs(res["objective"] - U) / U
    rel_L = np.abs(res["lower_bound"] - L) / np.abs(U)
    summary = dict(precision=precision, plans=k, solve_seconds=round(solve_s, 2),
                   iters_max=int(res["iters"].max()), iters_median=float(np.median(res["iters"])),
                   cert_gap_max=float(gap.max()), cert_gap_median=float(np.median(gap)),
                   device_cert_gap_max=float(np.nanmax(res["cert_gap"])),
                   plain_gap_max=float(res["rel_gap"].max()),
                   reported_vs_oracle_F_max=float(rel_F.max()),
                   device_vs_oracle_L_max=float(rel_L.max()),
                   oracle_r_pri_max=float(r_pri.max()), oracle_r_dual_max=float(r_dual.max()),
                   plans_certified_1e3=int(np.sum(gap <= 1e-3)))
    say(json.dumps(summary))
    if OUT:
        os.makedirs(OUT, exist_ok=True)
        with open(os.path.join(OUT, f"large_{precision}_certified.json"), "w") as f:
            json.dump(dict(summary, per_plan=dict(U=U.tolist(), L=L.tolist(), cert_gap=gap.tolist(),
                                                  iters=res["iters"].tolist())), f)
    assert np.all(conv), int(np.sum(~conv))
    assert np.all(L <= U * (1 + 1e-12))
    assert rel_F.max() < 1e-4           # the device's F(t) agrees with the oracle's FP64 F(t)
    assert rel_L.max() < 1e-4           # and its lower bound with the oracle's
    assert np.all(res["rel_gap"] <= 1e-4)
    # every plan's objective within 1e-3 of the exact optimum, certified in FP64
    assert np.all(gap <= 1e-3), np.sort(gap)[-5:]
    assert np.all(r_pri <= 1e-4) and np.all(r_dual <= 1e-4), (r_pri.max(), r_dual.max())
