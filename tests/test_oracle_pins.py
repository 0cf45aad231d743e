"""Hand-worked pins of the oracle's residuals, dual objective and low-dose band.

Each value below was worked out on paper from the definitions the oracle
states (Boyd's scaled-form residuals over both blocks of the split of
Eq. (dual_problem_admm); the dual-LP objective c'z1; the half-open band
[D_LD, D_LD + Delta) of Sec. 2.C.1), so that a dropped block, a wrong norm or a
closed band edge fails here rather than only showing up in a convergence test.
"""
import numpy as np

from oracle import admm
from oracle import dose as odose
from oracle import lp as olp
from oracle.simplex import solve_plan
from synth import cases


def _tiny_slp(c):
    """A ScaledLP shell with the given cost vector (the residuals and the dual
    objective read only c and the iterates)."""
    n = len(c)
    lp = olp.LP(A=np.zeros((1, n)), b=np.zeros((1, 2)), c=np.asarray(c, float),
                u=np.ones((n, 2)), n_points=n, n_iso=1, n_sectors=1, n_collimators=1)
    return olp.ScaledLP(lp, lp.A, lp.b, lp.c, lp.u, np.ones(1), 1.0)


def _state():
    """Two plans; x1, z1, y1 have 2 rows (x block), x2, z2, y2 one row."""
    st = admm.ADMMState(
        z1=np.array([[0.0, 1.0], [0.0, 0.0]]),
        y1=np.array([[1.0, 0.0], [2.0, 0.0]]),
        z2=np.array([[4.0, 0.0]]),
        y2=np.array([[2.0, 4.0]]))
    st.x1 = np.array([[3.0, 1.0], [0.0, 2.0]])
    st.x2 = np.array([[4.0, 2.0]])
    st.z1_prev = np.array([[0.0, 1.0], [1.0, 0.0]])
    st.z2_prev = np.array([[2.0, 0.0]])
    return st


def test_residuals_hand_worked():
    """Plan 0: x = (3, 0, 4), z = (0, 0, 4): ||x - z|| = 3, ||x|| = 5, ||z|| = 4,
    so r_pri = 3 / 5.  z - z_prev = (0, -1, 2), y = (1, 2, 2), rho = 2:
    r_dual = 2 sqrt(5) / (2 * 3) = sqrt(5) / 3.
    Plan 1: x = (1, 2, 2), z = (1, 0, 0): r_pri = 2 sqrt(2) / 3; z = z_prev, so
    r_dual = 0.
    Without the x2/z2 block plan 0 would give r_pri = 1 and r_dual = 1/sqrt(5);
    normalising by ||x - z|| gives 1; by min(||x||, ||z||) gives 3/4."""
    slp = _tiny_slp([-1.0, 1.0])
    rho = np.array([2.0, 0.5])
    r_pri, r_dual = admm.residuals(slp, rho, _state())
    np.testing.assert_allclose(r_pri, [3.0 / 5.0, 2.0 * np.sqrt(2.0) / 3.0], rtol=1e-15)
    np.testing.assert_allclose(r_dual, [np.sqrt(5.0) / 3.0, 0.0], rtol=1e-15, atol=0)


def test_residuals_are_scale_free():
    """Both residuals are ratios: scaling every iterate of a plan by s leaves
    them unchanged, and r_dual does not depend on rho (one scalar per plan
    appears in the numerator and in ||rho y||)."""
    slp = _tiny_slp([-1.0, 1.0])
    st = _state()
    a = admm.residuals(slp, np.array([2.0, 0.5]), st)
    sc = st.copy()
    for name in ("z1", "y1", "z2", "y2", "x1", "x2", "z1_prev", "z2_prev"):
        setattr(sc, name, 7.0 * getattr(sc, name))
    b = admm.residuals(slp, np.array([9.0, 0.1]), sc)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-14)
    np.testing.assert_allclose(a[1], b[1], rtol=1e-14)


def test_dual_objective_hand_worked():
    """c = (-1, -1, 1, 0) (two target points, one ring point, one sector):
    c'z1 = -0.5 - 0.25 + 2 + 0 = 1.25 and -1 + 0 + 0 + 0 = -1; the duals y1
    (nonzero here) do not enter."""
    slp = _tiny_slp([-1.0, -1.0, 1.0, 0.0])
    st = admm.ADMMState(z1=np.array([[0.5, 1.0], [0.25, 0.0], [2.0, 0.0], [9.0, 3.0]]),
                        y1=np.array([[3.0, -1.0], [0.5, 2.0], [-4.0, 1.0], [1.0, 1.0]]),
                        z2=np.ones((1, 2)), y2=np.ones((1, 2)))
    np.testing.assert_array_equal(admm.dual_objective(slp, st), [1.25, -1.0])


def test_dual_objective_at_the_simplex_optimum_is_minus_fstar():
    """At the optimal point x* of the dual LP (the oracle's simplex, itself pinned
    by vertex enumeration and KKT), c'x* = p* = -F*, and the preconditioning
    of Sec. 3.C (E, beta) leaves c'x unchanged for the point block."""
    case = cases.make_case(0)
    w = cases.config_weights(0)[[0, 4, 8]]
    lp = olp.assemble(case, w)
    slp = olp.precondition(lp, olp.bot_scale(case))
    xs = []
    fstar = []
    for j in range(w.shape[0]):
        res = solve_plan(lp, j)
        x = res.x.copy()
        x[lp.n_points:] *= slp.beta          # scaled sector variables
        xs.append(x)
        fstar.append(-res.objective)
    st = admm.ADMMState(z1=np.stack(xs, axis=1), y1=np.zeros((lp.A.shape[1], 3)),
                        z2=np.zeros((lp.A.shape[0], 3)), y2=np.zeros((lp.A.shape[0], 3)))
    np.testing.assert_allclose(-admm.dual_objective(slp, st), fstar, rtol=1e-12)
    F = olp.planning_objective(case, w, np.stack(
        [solve_plan(lp, j).lam[:lp.n_t] for j in range(3)], axis=1))[0]
    np.testing.assert_allclose(F, fstar, rtol=1e-9)


def test_ld_band_edges():
    """[D_LD, D_LD + Delta) with D_LD = 10, Delta = 2: 10 is in, the largest
    double below 12 is in, 12 is out, the largest double below 10 is out."""
    below12 = np.nextafter(12.0, 0.0)
    below10 = np.nextafter(10.0, 0.0)
    d = np.array([[10.0, 0.0],
                  [below12, 12.0],
                  [12.0, below12],
                  [below10, 10.0],
                  [11.0, 25.0],
                  [0.0, 11.999]])          # voxels x plans
    bits = odose.ld_band(d, 10.0, 2.0)
    assert bits.shape == (2, 6)            # plans x voxels
    np.testing.assert_array_equal(bits[0], [True, True, False, False, True, False])
    np.testing.assert_array_equal(bits[1], [False, False, True, True, False, True])


def test_dose_is_the_rate_weighted_sum():
    """d_j(v) = sum_t phi(v, t) t_j: 2 voxels, 3 shots, 2 plans, by hand."""
    phi = np.array([[1.0, 2.0, 0.0], [0.5, 0.0, 4.0]])
    t = np.array([[1.0, 0.0], [2.0, 1.0], [0.5, 3.0]])
    np.testing.assert_array_equal(odose.dose(phi, t), [[5.0, 2.0], [2.5, 12.0]])
