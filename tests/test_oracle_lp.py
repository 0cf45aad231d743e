"""Pins of the oracle's LP assembly, preconditioning and planning objective.

The strongest pin is strong duality: the planning LP of Sec. 2.A is written
out here independently (shot times, BOT per isocentre as the largest sector
time, hinge slacks) and solved with HiGHS; its optimum must equal minus the
optimum of the oracle's App. A dual LP, and the oracle's F(t) must reproduce it.
A dropped term, a wrong sign or a transposed block in either fails this.
"""
import os

import numpy as np
import pytest
from scipy.optimize import linprog

from synth import cases
from synth.cases import TS, TI, RING, LD, OAR
from oracle import lp as olp
from oracle.simplex import solve_plan

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def planning_lp_highs(case, w_row):
    """Sec. 2.A written directly: min sum_p u_p s_p + w_BOT sum_i tau_i."""
    n_t, n_iso, S, C = case.n_t, case.n_iso, case.n_sectors, case.n_collimators
    types = case.point_types()
    counts = case.group_counts()
    phi = np.asarray(case.dose, np.float64)
    pen = np.nonzero(types != OAR)[0]
    oar = np.nonzero(types == OAR)[0]
    nv = n_t + n_iso + len(pen)
    cost = np.zeros(nv)
    rows, rhs = [], []
    for q, p in enumerate(pen):
        g = case.groups[case.group[p]]
        w = {TS: w_row[0], TI: w_row[0], RING: w_row[1], LD: w_row[2]}[g.type] * g.share
        cost[n_t + n_iso + q] = w / counts[case.group[p]]
        r = np.zeros(nv)
        if g.type in (TS, TI):       # s_p >= 1 - d_p / D
            r[:n_t] = -phi[p] / g.threshold
            r[n_t + n_iso + q] = -1.0
            rhs.append(-1.0)
        else:                        # s_p >= d_p / D - 1
            r[:n_t] = phi[p] / g.threshold
            r[n_t + n_iso + q] = -1.0
            rhs.append(1.0)
        rows.append(r)
    for p in oar:                    # d_p <= D_O
        r = np.zeros(nv)
        r[:n_t] = phi[p]
        rows.append(r)
        rhs.append(case.groups[case.group[p]].threshold)
    for i in range(n_iso):           # tau_i >= (phi_cal / D_T) * (time of sector s)
        for s in range(S):
            r = np.zeros(nv)
            r[(i * S + s) * C:(i * S + s + 1) * C] = case.phi_cal / case.prescription_mean
            r[n_t + i] = -1.0
            rows.append(r)
            rhs.append(0.0)
    cost[n_t:n_t + n_iso] = w_row[3]
    res = linprog(cost, A_ub=np.array(rows), b_ub=np.array(rhs), bounds=(0, None),
                  method="highs", options=dict(primal_feasibility_tolerance=1e-10,
                                               dual_feasibility_tolerance=1e-10))
    assert res.status == 0
    return res.fun, res.x[:n_t]


@pytest.mark.parametrize("spec_kw,seed", [
    (dict(), 0),
    (dict(n_iso=2, sectors=3, collimators=2, n_ring=12, n_ld=8), 1),
    (dict(n_iso=2, sectors=8, collimators=3, n_ring=20, n_ld=10, oar=True), 2),
])
def test_strong_duality_mini(spec_kw, seed):
    case = cases.build_case(cases.mini_spec(**spec_kw), seed)
    w = cases.random_weights(4, seed)
    lp = olp.assemble(case, w)
    for j in range(w.shape[0]):
        res = solve_plan(lp, j)
        assert res.status == "optimal"
        F_direct, t_direct = planning_lp_highs(case, w[j])
        assert abs(res.objective + F_direct) <= 1e-9 * max(1.0, abs(F_direct))
        # F evaluated at the App. A multipliers and at the direct solution
        F_lam = olp.planning_objective(case, w[j:j + 1], res.lam[:lp.n_t, None])[0][0]
        F_dir = olp.planning_objective(case, w[j:j + 1], t_direct[:, None])[0][0]
        assert abs(F_lam - F_direct) <= 1e-8 * max(1.0, abs(F_direct))
        assert abs(F_dir - F_direct) <= 1e-8 * max(1.0, abs(F_direct))


def test_strong_duality_config0():
    case = cases.make_case(0)
    w = cases.config_weights(0)
    lp = olp.assemble(case, w)
    for j in (0, 4, 8):
        res = solve_plan(lp, j)
        F_direct, _ = planning_lp_highs(case, w[j])
        assert abs(res.objective + F_direct) <= 1e-9 * abs(F_direct)


def test_shapes_match_table1():
    """Rows of A = 25 N_iso and columns = points + 8 N_iso (Table 1, App. A)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_problem_sizes.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 20
    for _, n_iso, m, n in rows:
        n_iso, m, n = int(n_iso), int(m), int(n)
        assert m == 25 * n_iso
        assert n - 8 * n_iso > 0
    # our assembly produces the same row/column arithmetic
    for kw in (dict(n_iso=1), dict(n_iso=3, n_ring=30, n_ld=12)):
        case = cases.build_case(cases.mini_spec(**kw), 3)
        lp = olp.assemble(case, cases.random_weights(2, 0))
        spec_s, spec_c = case.n_sectors, case.n_collimators
        assert lp.A.shape == (case.n_iso * (spec_s * spec_c + 1), case.n_points + spec_s * case.n_iso)
    case = cases.build_case(cases.mini_spec(n_iso=3, sectors=8, collimators=3, n_ring=30, n_ld=12), 3)
    lp = olp.assemble(case, cases.random_weights(2, 0))
    assert lp.A.shape == (25 * 3, case.n_points + 8 * 3)


def test_beta_range_of_table1():
    """beta = points / 2000 spans 'about 1' to 'about 20' over Table 1 (Sec. 3.C)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_problem_sizes.txt"))
            if l.strip() and not l.startswith("#")]
    betas = [(int(n) - 8 * int(n_iso)) / 2000.0 for _, n_iso, _, n in rows]
    assert 1.5 < min(betas) < 2.5      # upper bound: OAR points are included here
    assert 19.0 < max(betas) < 21.0


def test_row_normalisation_makes_diag_two():
    """After row normalisation diag(S) = 2 and |S_ij| <= 1 (Sec. 3.C), beta = 1."""
    case = cases.make_case(0)
    lp = olp.assemble(case, cases.config_weights(0))
    slp = olp.precondition(lp, beta=1.0)
    S = slp.A @ slp.A.T + np.eye(lp.A.shape[0])
    assert np.allclose(np.diag(S), 2.0, atol=1e-13)
    off = S - np.diag(np.diag(S))
    assert np.max(np.abs(off)) <= 1.0 + 1e-13
    # S = A A' + I is SPD with smallest eigenvalue >= 1
    assert np.linalg.eigvalsh(S).min() >= 1.0 - 1e-10


def test_scaling_leaves_optimum_unchanged():
    """Row and BOT-column scaling do not change p* (LP scaling invariance)."""
    from oracle.simplex import simplex_solve
    case = cases.build_case(cases.mini_spec(n_iso=2, sectors=4, collimators=2, n_ring=16, n_ld=8), 5)
    w = cases.random_weights(3, 5)
    lp = olp.assemble(case, w)
    for beta in (0.5, 7.0):
        slp = olp.precondition(lp, beta=beta)
        for j in range(3):
            a = simplex_solve(lp.A, lp.b[:, j], lp.c, lp.u[:, j]).objective
            b = simplex_solve(slp.A, slp.b[:, j], slp.c, slp.u[:, j]).objective
            assert abs(a - b) <= 1e-10 * max(1.0, abs(a))


def test_rho_rule_and_beta_values():
    # rho = rho0 sqrt(w0 / w_BOT): equals rho0 at w_BOT = w0, scales as w_BOT^-1/2
    r = olp.rho_rule(np.array([1e-3, 4e-3, 1.0]), 2.5e-3, 1e-3)
    assert r[0] == pytest.approx(2.5e-3)
    assert r[1] == pytest.approx(1.25e-3)
    assert r[2] == pytest.approx(2.5e-3 / np.sqrt(1000.0))
    case = cases.make_case(0)
    assert olp.bot_scale(case) == pytest.approx(case.n_points / 2000.0)


def test_upper_bounds_and_masks():
    case = cases.make_case(0)
    w = cases.slider_weights([0.0, 1.0], [0.0, 1.0])
    u = olp.point_upper_bounds(case, w)
    counts = case.group_counts()
    types = case.point_types()
    # u sums to the group weight over each group (w_g / N_g summed N_g times)
    for g, grp in enumerate(case.groups):
        sel = case.group == g
        expect = {TS: w[:, 0], TI: w[:, 0], RING: w[:, 1], LD: w[:, 2]}[grp.type] * grp.share
        assert np.allclose(u[sel].sum(axis=0), expect)
        assert sel.sum() == counts[g]
    # a low-dose mask zeroes u outside p_j and renormalises by |p_j|
    ld = np.nonzero(types == LD)[0]
    mask = np.zeros((2, case.n_points), bool)
    mask[:, ld[:10]] = True
    um = olp.point_upper_bounds(case, w, mask)
    assert np.all(um[ld[10:]] == 0)
    assert np.allclose(um[ld[:10], 1], w[1, 2] / 10)


def test_certified_bounds_bracket_optimum():
    case = cases.build_case(cases.mini_spec(n_iso=2, sectors=8, collimators=3, n_ring=20,
                                            n_ld=10, oar=True), 2)
    w = cases.random_weights(3, 9)
    lp = olp.assemble(case, w)
    rng = np.random.default_rng(0)
    for j in range(3):
        res = solve_plan(lp, j)
        Fstar = -res.objective
        # at the optimum both bounds are tight
        cb = olp.certify(case, w[j:j + 1], res.lam[:lp.n_t, None], res.x[:lp.n_points, None])
        assert cb["L"][0] <= Fstar + 1e-10 and cb["U"][0] >= Fstar - 1e-10
        assert abs(cb["U"][0] - Fstar) <= 1e-8 * Fstar
        assert abs(cb["L"][0] - Fstar) <= 1e-8 * Fstar
        # perturbed points still give valid (looser) bounds
        for _ in range(5):
            t = np.abs(res.lam[:lp.n_t] * (1 + 0.3 * rng.standard_normal(lp.n_t)))
            x = res.x[:lp.n_points] * (1 + 0.3 * rng.standard_normal(lp.n_points))
            cb = olp.certify(case, w[j:j + 1], t[:, None], x[:, None])
            assert cb["L"][0] <= Fstar + 1e-10 <= cb["U"][0] + 2e-10
