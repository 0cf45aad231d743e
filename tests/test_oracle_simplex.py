"""Pins of the oracle's dense simplex: brute force, HiGHS, KKT."""
import numpy as np
import pytest
from scipy.optimize import linprog

from synth import cases
from oracle import lp as olp
from oracle.simplex import simplex_solve, kkt_residuals, solve_plan
from oracle.vertex import enumerate_vertices


def random_app_a_lp(rng, m, n):
    """A small LP with the sign pattern of App. A: Ax <= b, b >= 0, 0 <= x <= u."""
    A = rng.standard_normal((m, n))
    b = np.abs(rng.standard_normal(m)) * (rng.random(m) < 0.6)   # many zero rows, as in App. A
    c = rng.standard_normal(n)
    u = np.where(rng.random(n) < 0.7, rng.uniform(0.0, 2.0, n), np.inf)
    u[rng.random(n) < 0.1] = 0.0                                  # fixed-at-zero columns
    # keep it bounded: every unbounded column gets a nonnegative cost
    c[~np.isfinite(u)] = np.abs(c[~np.isfinite(u)])
    return A, b, c, u


@pytest.mark.parametrize("seed", range(12))
def test_simplex_matches_vertex_enumeration(seed):
    rng = np.random.default_rng(seed)
    m, n = int(rng.integers(2, 5)), int(rng.integers(3, 8))
    A, b, c, u = random_app_a_lp(rng, m, n)
    res = simplex_solve(A, b, c, u)
    best, _ = enumerate_vertices(A, b, c, u)
    assert res.status == "optimal"
    assert abs(res.objective - best) <= 1e-9 * max(1.0, abs(best))
    kkt = kkt_residuals(A, b, c, u, res.x, res.lam)
    assert kkt["primal"] < 1e-9 and kkt["dual"] < 1e-9 and kkt["comp"] < 1e-9
    assert abs(kkt["gap"]) < 1e-9


def test_simplex_matches_vertex_enumeration_lightning_mini():
    """A Lightning LP with 1 isocentre, 2 sectors, 1 collimator and 6 points."""
    full = cases.build_case(cases.mini_spec(n_iso=1, sectors=2, collimators=1, radius=2.0,
                                            n_ring=4, n_ld=4), 4)
    keep = np.concatenate([np.nonzero(full.group == g)[0][:2 if g >= 2 else 1]
                           for g in range(len(full.groups))])
    case = full.with_points(keep)
    w = cases.random_weights(4, 1)
    lp = olp.assemble(case, w)
    assert lp.A.shape[1] <= 9
    for j in range(4):
        res = simplex_solve(lp.A, lp.b[:, j], lp.c, lp.u[:, j])
        best, _ = enumerate_vertices(lp.A, lp.b[:, j], lp.c, lp.u[:, j])
        assert abs(res.objective - best) <= 1e-10 * max(1.0, abs(best))


@pytest.mark.parametrize("config_plans", [(0, (0, 3, 5, 7))])
def test_simplex_matches_highs_config0(config_plans):
    config, plans = config_plans
    case = cases.make_case(config)
    w = cases.config_weights(config)
    lp = olp.assemble(case, w)
    for j in plans:
        res = solve_plan(lp, j)
        bounds = list(zip(np.zeros(lp.c.size), np.where(np.isfinite(lp.u[:, j]), lp.u[:, j], None)))
        h = linprog(lp.c, A_ub=lp.A, b_ub=lp.b[:, j], bounds=bounds, method="highs",
                    options=dict(primal_feasibility_tolerance=1e-10,
                                 dual_feasibility_tolerance=1e-10))
        assert abs(res.objective - h.fun) <= 1e-9 * abs(h.fun)
        kkt = kkt_residuals(lp.A, lp.b[:, j], lp.c, lp.u[:, j], res.x, res.lam)
        assert kkt["primal"] < 1e-12 and kkt["dual"] < 1e-10 and kkt["comp"] < 1e-12


def test_simplex_planted_error_is_caught():
    """A wrong sign in the LP (an error planted in the oracle's input) breaks
    agreement with brute force, so the comparison above has teeth."""
    rng = np.random.default_rng(3)
    A, b, c, u = random_app_a_lp(rng, 3, 6)
    good = simplex_solve(A, b, c, u).objective
    A2 = A.copy()
    A2[0] = -A2[0]
    bad = simplex_solve(A2, b, c, u).objective
    best, _ = enumerate_vertices(A, b, c, u)
    assert abs(good - best) < 1e-9
    assert abs(bad - best) > 1e-6 or np.allclose(A[0], 0)
