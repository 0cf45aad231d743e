"""Pins of the oracle's reference ADMM (Sec. 2.B)."""
import numpy as np
import pytest

from synth import cases
from oracle import lp as olp
from oracle import admm
from oracle.simplex import solve_plan


def _random_scaled_lp(rng, m, n, k):
    A = rng.standard_normal((m, n))
    lp = olp.LP(A=A, b=np.abs(rng.standard_normal((m, k))), c=rng.standard_normal(n),
                u=np.abs(rng.standard_normal((n, k))), n_points=n, n_iso=1,
                n_sectors=1, n_collimators=1)
    return olp.ScaledLP(lp, A, lp.b, lp.c, lp.u, np.ones(m), 1.0)


def test_x_step_solves_the_equality_constrained_qp():
    """The closed-form x-step equals the direct solution of Eq. (x-step).

    minimise c'x1 + rho/2 |x1 - a1|^2 + rho/2 |x2 - a2|^2 subject to A x1 = x2,
    solved here through its full KKT system with a dense solver.  This also
    shows that the lower-right block of Eq. (eq_system) must be -I.
    """
    rng = np.random.default_rng(0)
    m, n, k = 5, 12, 3
    slp = _random_scaled_lp(rng, m, n, k)
    rho = np.array([0.7, 3.0, 20.0])
    st = admm.ADMMState(rng.standard_normal((n, k)), rng.standard_normal((n, k)),
                        rng.standard_normal((m, k)), rng.standard_normal((m, k)))
    out = admm.admm_iterate(slp, rho, 1, st)
    A, c = slp.A, slp.c
    for j in range(k):
        a1 = st.z1[:, j] - st.y1[:, j]
        a2 = st.z2[:, j] - st.y2[:, j]
        K = np.zeros((n + 2 * m, n + 2 * m))
        K[:n, :n] = rho[j] * np.eye(n)
        K[:n, n + m:] = A.T
        K[n:n + m, n:n + m] = rho[j] * np.eye(m)
        K[n:n + m, n + m:] = -np.eye(m)
        K[n + m:, :n] = A
        K[n + m:, n:n + m] = -np.eye(m)
        rhs = np.concatenate([rho[j] * a1 - c, rho[j] * a2, np.zeros(m)])
        sol = np.linalg.solve(K, rhs)
        assert np.allclose(out.x1[:, j], sol[:n], atol=1e-12, rtol=1e-12)
        assert np.allclose(out.x2[:, j], sol[n:n + m], atol=1e-12, rtol=1e-12)
        # the block system as printed (+I in the corner) gives another x1
        P = np.block([[np.eye(n), A.T], [A, np.eye(m)]])
        printed = np.linalg.solve(P, np.concatenate([a1 - c / rho[j], a2]))
        assert np.max(np.abs(printed[:n] - sol[:n])) > 1e-3


def test_z_and_y_steps_are_projections():
    rng = np.random.default_rng(1)
    slp = _random_scaled_lp(rng, 4, 9, 2)
    st = admm.admm_iterate(slp, np.array([1.0, 2.0]), 7)
    assert np.all(st.z1 >= 0) and np.all(st.z1 <= slp.u + 1e-15)
    assert np.all(st.z2 <= slp.b + 1e-15)
    # y1 = q - clip(q) and y2 = max(0, x2 + y2_prev - b) >= 0 after any step:
    assert np.allclose(st.z1, np.clip(st.z1 + st.y1, 0.0, slp.u), atol=1e-14)
    assert np.all(st.y2 >= -1e-15)
    assert np.allclose(st.z2, np.minimum(st.z2 + st.y2, slp.b), atol=1e-14)


def test_resume_is_bitwise_identical():
    case = cases.make_case(0)
    w = cases.config_weights(0)[[0, 4, 8]]
    slp = olp.precondition(olp.assemble(case, w), olp.bot_scale(case))
    rho = olp.rho_rule(w[:, 3], 1000.0, cases.W0_BOT)
    fac, _ = admm.schur_factor(slp)
    full = admm.admm_iterate(slp, rho, 60, factor=fac)
    half = admm.admm_iterate(slp, rho, 25, factor=fac)
    resumed = admm.admm_iterate(slp, rho, 35, half, factor=fac)
    for a, b in ((full.z1, resumed.z1), (full.y1, resumed.y1), (full.z2, resumed.z2),
                 (full.y2, resumed.y2)):
        assert np.array_equal(a, b)


def test_admm_converges_to_simplex_optimum():
    """Reference ADMM reaches the exact optimum of every plan (c0, 9 plans)."""
    case = cases.make_case(0)
    w = cases.config_weights(0)
    lp = olp.assemble(case, w)
    Fstar = np.array([-solve_plan(lp, j).objective for j in range(w.shape[0])])
    slp = olp.precondition(lp, olp.bot_scale(case))
    rho = olp.rho_rule(w[:, 3], 1000.0, cases.W0_BOT)
    fac, _ = admm.schur_factor(slp)
    st = None
    best = np.full(w.shape[0], np.inf)
    for _ in range(40):
        st = admm.admm_iterate(slp, rho, 100, st, fac)
        t, _ = admm.shot_times(slp, rho, st)
        assert np.all(t >= 0)
        F = olp.planning_objective(case, w, t)[0]
        best = np.minimum(best, np.abs(F - Fstar) / Fstar)
        # certified bounds bracket the optimum at every checked iterate
        cb = olp.certify(case, w, t, st.z1[:lp.n_points], lp)
        assert np.all(cb["L"] <= Fstar * (1 + 1e-12))
        assert np.all(cb["U"] >= Fstar * (1 - 1e-12))
    assert np.all(best < 1e-3)
    F = olp.planning_objective(case, w, admm.shot_times(slp, rho, st)[0])[0]
    assert np.all(np.abs(F - Fstar) / Fstar < 3e-3)
    gap = np.abs(F + admm.dual_objective(slp, st)) / F
    assert np.all(gap < 1e-2)
    r_pri, r_dual = admm.residuals(slp, rho, st)
    assert np.all(r_pri < 1e-3) and np.all(r_dual < 1e-3)


def test_adaptive_rho_switch_keeps_the_multipliers():
    """A step-size switch rescales the scaled duals so that rho * y (the
    multipliers, hence the shot times t = E rho y2) is unchanged, and with
    balancing disabled the adaptive run is the plain iteration, bitwise."""
    case = cases.make_case(0)
    w = cases.config_weights(0)
    slp = olp.precondition(olp.assemble(case, w), olp.bot_scale(case))
    rho = olp.rho_rule(w[:, 3], 1000.0, cases.W0_BOT)
    fac, _ = admm.schur_factor(slp)
    plain = admm.admm_iterate(slp, rho, 50, factor=fac)
    st, rho_new = admm.admm_adaptive(slp, rho, 50, 50, factor=fac)
    assert np.any(rho_new != rho)                    # some plan switched at the check
    assert np.all(np.isin(rho_new / rho, [0.5, 1.0, 2.0]))
    assert np.array_equal(st.z1, plain.z1) and np.array_equal(st.z2, plain.z2)
    assert np.array_equal(rho_new * st.y2, rho * plain.y2)
    assert np.array_equal(rho_new * st.y1, rho * plain.y1)
    off, rho_off = admm.admm_adaptive(slp, rho, 120, 50, mu=np.inf, factor=fac)
    ref = admm.admm_iterate(slp, rho, 120, factor=fac)
    assert np.array_equal(rho_off, rho)
    assert np.array_equal(off.y2, ref.y2) and np.array_equal(off.z1, ref.z1)


def test_adaptive_rho_recovers_from_a_poor_start():
    """Started 30x below the tuned step size, residual balancing brings every
    plan within 3e-3 of its exact optimum (c0, 9 plans) in 3,000 iterations,
    several times closer than the fixed step size gets."""
    case = cases.make_case(0)
    w = cases.config_weights(0)
    lp = olp.assemble(case, w)
    Fstar = np.array([-solve_plan(lp, j).objective for j in range(w.shape[0])])
    slp = olp.precondition(lp, olp.bot_scale(case))
    rho = olp.rho_rule(w[:, 3], 30.0, cases.W0_BOT)
    fac, _ = admm.schur_factor(slp)
    st, rho_end = admm.admm_adaptive(slp, rho, 3000, 50, factor=fac)
    F = olp.planning_objective(case, w, admm.shot_times(slp, rho_end, st)[0])[0]
    fixed = admm.admm_iterate(slp, rho, 3000, factor=fac)
    F_fixed = olp.planning_objective(case, w, admm.shot_times(slp, rho, fixed)[0])[0]
    err, err_fixed = np.abs(F - Fstar) / Fstar, np.abs(F_fixed - Fstar) / Fstar
    assert np.all(err < 3e-3), err
    assert err_fixed.max() > 5 * err.max()


def test_over_relaxed_admm_reaches_the_simplex_optimum():
    """Over-relaxed ADMM (alpha = 1.6) has the same fixed points: every plan of the
    small case reaches the exact LP optimum of the simplex within 1e-3."""
    case = cases.make_case(0)
    w = cases.config_weights(0)
    lp = olp.assemble(case, w)
    Fstar = np.array([-solve_plan(lp, j).objective for j in range(w.shape[0])])
    slp = olp.precondition(lp, olp.bot_scale(case))
    rho = olp.rho_rule(w[:, 3], 1000.0, cases.W0_BOT)
    fac, _ = admm.schur_factor(slp)
    st = None
    best = np.full(w.shape[0], np.inf)
    for _ in range(40):
        st = admm.admm_iterate(slp, rho, 100, st, fac, alpha=1.6)
        t, _ = admm.shot_times(slp, rho, st)
        F = olp.planning_objective(case, w, t)[0]
        best = np.minimum(best, np.abs(F - Fstar) / Fstar)
    assert np.all(best < 1e-3), best
    r_pri, r_dual = admm.residuals(slp, rho, st)
    assert np.all(r_pri < 1e-3) and np.all(r_dual < 1e-3)
