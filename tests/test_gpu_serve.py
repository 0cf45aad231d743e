"""GPU serving: continuous batching through ladmm_submit / poll / wait / cancel.

A plan's arithmetic does not depend on the other plans in its lane, on its slot
or on when it was admitted, so every plan served in a mix must equal, bitwise,
the same request solved alone by ladmm_solve_batch (same options, max_iter a
multiple of check_every).  The alone results are themselves pinned to the
oracle by the parity tests; here the served objectives are also checked against
the exact LP optimum F* of the stored golden values.
"""
import os
import sys
import time

import numpy as np
import pytest

from synth import cases
from oracle import lp as olp

pytestmark = pytest.mark.gpu

ladmm = pytest.importorskip("paper_2509_08602_amd.ladmm")


def read_fstar(config):
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    import make_golden
    return make_golden.read(config)


def golden_fstar(config):
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    import make_golden
    return make_golden.read(config)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    return ladmm.Context(0)


@pytest.fixture(scope="module")
def c0():
    return cases.make_case(0)


@pytest.fixture(scope="module")
def mini():
    spec = cases.mini_spec(n_iso=3, sectors=8, collimators=3, radius=4.0, n_ring=400, n_ld=300)
    return cases.build_case(spec, 11)


def opts(max_iter, tol=1e-4, K=50, adapt=True):
    return ladmm.Options(max_iter=max_iter, check_every=K, tol_gap=tol, tol_pri=tol, tol_dual=tol,
                         rho0=1000.0, w0_bot=cases.W0_BOT, autotune=False, adapt_rho=adapt)


def same(a, b):
    for key in ("t", "bot", "objective", "dual_obj", "rel_gap", "r_pri", "r_dual", "iters",
                "plan_status"):
        assert np.array_equal(a[key], b[key]), key


def test_served_plans_equal_plans_solved_alone(ctx, c0, mini):
    """Requests on two cases, sizes 1 to 9, submitted while others run, on 32
    slots per lane; the probe request R arrives mid-stream."""
    say("serve mix c0 + mini, f64")
    d0 = ladmm.Case.from_case(ctx, c0, "f64")
    dm = ladmm.Case.from_case(ctx, mini, "f64")
    w0 = cases.config_weights(0)
    wr = cases.random_weights(40, 3)
    o, oR = opts(1000), opts(8000, adapt=False)   # R: the paper's fixed step rule
    alone_R = ladmm.solve_batch(d0, w0, opts=oR)
    alone_m = [ladmm.solve_batch(dm, wr[i:i + 8], opts=o) for i in range(0, 40, 8)]
    alone_1 = ladmm.solve_batch(d0, wr[5:6], opts=o)
    srv = ladmm.Server(ctx, slots=32, check_every=50, autotune=False)
    tm = [srv.submit(dm, wr[i:i + 8], opts=o) for i in range(0, 24, 8)]
    t1 = srv.submit(d0, wr[5:6], opts=o)
    time.sleep(0.05)
    tR = srv.submit(d0, w0, opts=oR)
    tm += [srv.submit(dm, wr[i:i + 8], opts=o) for i in range(24, 40, 8)]
    same(tR.result(), alone_R)
    same(t1.result(), alone_1)
    for t, ref in zip(tm, alone_m):
        same(t.result(), ref)
    st = srv.stats()
    say("stats", st)
    assert st["completed"] == 7 and st["failed"] == 0 and st["plans_completed"] == 9 + 1 + 40
    assert st["p50_ms"] > 0 and st["p99_ms"] >= st["p50_ms"]
    srv.close()
    fstar = read_fstar(0)
    F = tR.out["objective"]
    for j, fs in fstar.items():
        assert abs(F[j] - fs) <= 1e-3 * abs(fs) + 1e-9, (j, F[j], fs)


@pytest.mark.parametrize("precision,eager", [("f32", False), ("bf16x3", False), ("bf16", False),
                                             ("f32", True)])
def test_slot_reuse_and_masks_match_alone(ctx, mini, precision, eager):
    """More plans than slots (plans start in freed slots), with LD masks.  The
    lanes replay captured graphs (or, eager, launch one by one); the requests
    solved alone replay graphs."""
    say("serve slot reuse mini", precision, "eager" if eager else "graphs")
    dm = ladmm.Case.from_case(ctx, mini, precision)
    k = 70
    w = cases.random_weights(k, 6)
    types = mini.point_types()
    rng = np.random.default_rng(2)
    mask = np.zeros((k, mini.n_points), bool)
    ld = np.nonzero(types == cases.LD)[0]
    for j in range(k):
        mask[j, ld[rng.random(ld.size) < 0.7]] = True
    reqs = [(0, 30, 200), (30, 31, 400), (31, 70, 100)]
    srv = ladmm.Server(ctx, slots=32, check_every=50, autotune=True, eager=eager)
    tickets = [srv.submit(dm, w[a:b], ld_mask=mask[a:b], opts=opts(m, tol=0.0)) for a, b, m in reqs]
    for (a, b, m), t in zip(reqs, tickets):
        ref = ladmm.solve_batch(dm, w[a:b], ld_mask=mask[a:b], opts=opts(m, tol=0.0))
        got = t.result()
        same(got, ref)
        assert np.all(got["iters"] == m)
        # the objective product runs in FP32 (f32) or as BF16 pairs (16
        # significant bits per operand, about 2^-16 relative per term)
        F = olp.planning_objective(mini, w[a:b], got["t"].T, mask[a:b])[0]
        tol = 1e-5 if precision == "f32" else 5e-5
        assert np.max(np.abs(got["objective"] - F) / np.maximum(np.abs(F), 1e-12)) < tol
    srv.close()


def test_cancel_poll_and_release(ctx, mini):
    say("serve cancel")
    dm = ladmm.Case.from_case(ctx, mini, "f64")
    w = cases.random_weights(4, 8)
    srv = ladmm.Server(ctx, slots=32, check_every=50, autotune=False)
    long = srv.submit(dm, w, opts=opts(200000, tol=0.0))
    short = srv.submit(dm, w[:2], opts=opts(100, tol=0.0))
    assert short.wait() == ladmm.OK
    status, _ = long.poll()
    assert status == ladmm.PENDING
    long.cancel()
    assert long.wait() == ladmm.E_CANCELLED
    # the ticket was released by the report; the library now rejects it
    rc = ladmm.library().ladmm_poll(srv._h, long.id, None)
    assert rc == ladmm.E_STATE
    ref = ladmm.solve_batch(dm, w[:2], opts=opts(100, tol=0.0))
    same(short.out, ref)
    st = srv.stats()
    assert st["cancelled"] == 1 and st["completed"] == 1
    with pytest.raises(ladmm.LadmmError):
        srv.submit(dm, w, opts=ladmm.Options(max_iter=100, check_every=7))   # wrong check_every
    srv.close()


def test_hbm_budget_evicts_idle_lanes(ctx, mini, c0):
    """A budget that holds both cases but one lane at a time: requests on the two
    cases still all complete (lanes are released and re-created), unchanged."""
    say("serve budget")
    probe = ladmm.Context(0)
    a = ladmm.Case.from_case(probe, mini, "f64")
    b = ladmm.Case.from_case(probe, c0, "f64")
    cases_bytes = probe.used_bytes
    srv = ladmm.Server(probe, slots=32, check_every=50, autotune=False)
    srv.submit(a, cases.random_weights(1, 1), opts=opts(50)).wait()
    lane_a = probe.used_bytes - cases_bytes
    srv.close()
    srv = ladmm.Server(probe, slots=32, check_every=50, autotune=False)
    srv.submit(b, cases.random_weights(1, 1), opts=opts(50)).wait()
    lane_b = probe.used_bytes - cases_bytes
    srv.close()
    a.close(), b.close()
    budget = cases_bytes + max(lane_a, lane_b) + min(lane_a, lane_b) // 2
    small = ladmm.Context(0, hbm_budget=budget)
    ca = ladmm.Case.from_case(small, mini, "f64")
    cb = ladmm.Case.from_case(small, c0, "f64")
    w = cases.random_weights(6, 12)
    o = opts(300)
    srv = ladmm.Server(small, slots=32, check_every=50, autotune=False)
    ts = [srv.submit(ca, w[:3], opts=o), srv.submit(cb, w[3:], opts=o), srv.submit(ca, w[3:], opts=o)]
    res = [t.result() for t in ts]
    assert small.used_bytes <= budget
    st = srv.stats()
    assert st["completed"] == 3 and st["lanes"] <= 1
    srv.close()
    same(res[0], ladmm.solve_batch(ca, w[:3], opts=o))
    same(res[1], ladmm.solve_batch(cb, w[3:], opts=o))
    same(res[2], ladmm.solve_batch(ca, w[3:], opts=o))


@pytest.mark.parametrize("precision", ["f64", "bf16x3", "bf16"])
def test_warm_start_from_nearest_solved_plan(ctx, c0, precision):
    """A server with a warm store starts each admitted plan from the stored
    solved plan of the nearest weighting.  Every plan stops on its certified
    gap (<= 9e-4: its objective provably within that of the exact optimum F*).
    The 9 slider plans solved a second time start from their own solutions and
    stop after far fewer iterations, and every result is within 1e-3 of the
    exact optimum (stored, from the oracle's simplex); perturbed weightings
    converge in fewer iterations than cold, each certified within 1e-3 of its
    optimum, and agree with the plans solved alone within 2e-3 (both within
    1e-3 of the same optimum)."""
    say("serve warm start c0", precision)
    dc = ladmm.Case.from_case(ctx, c0, precision)
    w0 = cases.config_weights(0)
    fs = golden_fstar(0)
    Fstar = np.array([fs[j] for j in range(w0.shape[0])])
    # the library's default step-size rule (balanced from rho0 = 1e4)
    o = ladmm.Options(max_iter=40000, check_every=50, tol_gap=1e-3, tol_pri=1e-4, tol_dual=1e-4,
                      tol_cert=9e-4, rho0=1e4, w0_bot=cases.W0_BOT, autotune=False, adapt_rho=True)
    srv = ladmm.Server(ctx, slots=32, check_every=50, autotune=False, warm_store=64)
    first = srv.submit(dc, w0, opts=o).result()
    say("  first pass status", first["plan_status"].tolist(), "iterations", first["iters"].tolist())
    assert np.all(first["plan_status"] == ladmm.PLAN_CONVERGED)   # all enter the store
    second = srv.submit(dc, w0, opts=o).result()
    assert srv.stats()["warm_starts"] == w0.shape[0]
    assert np.all(second["plan_status"] == ladmm.PLAN_CONVERGED)
    # the stopping criteria are not monotone along the ADMM iterates, so a plan
    # restarted from its own stopping point need not pass at its very next
    # check; it never needs more iterations than from cold, and far fewer in
    # total (the exact continuation is checked in the host emulation)
    say("  second pass iterations", second["iters"].tolist())
    assert np.all(second["iters"] <= first["iters"]), (second["iters"], first["iters"])
    assert second["iters"].sum() < 0.5 * first["iters"].sum()
    for res in (first, second):
        assert np.all(res["cert_gap"] <= 9e-4)
        rel = np.abs(res["objective"] - Fstar) / Fstar
        assert rel.max() <= 1e-3, rel
    # perturbed sliders: w_LD + 0.05 and the BOT slider + 0.05 (w_BOT x 10^0.15)
    w1 = w0.copy()
    w1[:, 2] = np.clip(w1[:, 2] + 0.05, 0.0, 1.0)
    w1[:, 3] *= 10 ** 0.15
    alone = ladmm.solve_batch(dc, w1, opts=o)
    warm = srv.submit(dc, w1, opts=o).result()
    st = srv.stats()
    srv.close()
    say("  cold iterations", first["iters"].tolist(), "perturbed alone", alone["iters"].tolist(),
        "perturbed warm", warm["iters"].tolist(), "warm starts", st["warm_starts"])
    assert st["warm_starts"] == 2 * w0.shape[0]
    assert np.all(warm["plan_status"] == ladmm.PLAN_CONVERGED)
    assert warm["iters"].sum() < alone["iters"].sum()
    # each certified within 9e-4 of its optimum, so within 2e-3 of each other
    assert np.all(warm["cert_gap"] <= 9e-4) and np.all(alone["cert_gap"] <= 9e-4)
    rel = np.abs(warm["objective"] - alone["objective"]) / np.abs(alone["objective"])
    assert rel.max() <= 2e-3, rel
