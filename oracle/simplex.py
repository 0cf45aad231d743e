"""Dense bounded-variable simplex (FP64) for the LP of App. A.

Oracle code (test infrastructure).  Solves

    minimize c'x  subject to  A x <= b,  0 <= x <= u   (u_j may be +inf)

for b >= 0, where x = 0 with the slack basis is a feasible start.  The shot
rows of App. A have b = 0, so that start is highly degenerate; the solver
therefore works in the textbook way used by production simplex codes:

  1. primal simplex with bounded variables on a slightly perturbed right-hand
     side b + eps (eps > 0, tiny, fixed), Dantzig pricing, bound flips, and
     Bland's rule as a fallback while steps stay degenerate;
  2. the perturbation is removed; the final basis is still dual feasible
     (reduced costs do not depend on b), so any small primal infeasibility
     left is cleared by bounded dual simplex pivots;
  3. the answer is certified by `kkt_residuals` (primal and dual feasibility,
     complementary slackness, zero duality gap).

It stands in for the exact solver the paper compares against (Sec. 3.A).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class SimplexResult:
    x: np.ndarray        # optimal point (n)
    objective: float     # c'x = p*
    lam: np.ndarray      # multipliers of A x <= b (>= 0); the primal shot times
    reduced: np.ndarray  # reduced costs c + A' lam (n)
    iterations: int
    status: str          # "optimal" | "iteration_limit" | "unbounded" | "infeasible"


class _Tableau:
    """Basis bookkeeping for the bounded revised simplex on [A I] [x; s] = b."""

    def __init__(self, A, b, c, u):
        m, n = A.shape
        self.m, self.n = m, n
        self.M = np.hstack([A, np.eye(m)])
        self.cost = np.concatenate([c, np.zeros(m)])
        self.ub = np.concatenate([u, np.full(m, np.inf)])
        self.b = b.copy()
        self.basis = np.arange(n, n + m)
        self.in_basis = np.zeros(n + m, bool)
        self.in_basis[self.basis] = True
        self.at_upper = np.zeros(n + m, bool)
        self.Binv = np.eye(m)
        self.pivots = 0

    def refactor(self):
        self.Binv = np.linalg.inv(self.M[:, self.basis])

    def x_basic(self):
        up = self.at_upper & ~self.in_basis
        rhs = self.b - self.M[:, up] @ self.ub[up] if up.any() else self.b
        return self.Binv @ rhs

    def reduced_costs(self):
        y = self.cost[self.basis] @ self.Binv
        d = self.cost - y @ self.M
        d[self.basis] = 0.0
        return d, y

    def pivot(self, leave_row, enter, alpha, leave_to_upper):
        old = self.basis[leave_row]
        self.in_basis[old] = False
        self.at_upper[old] = leave_to_upper
        self.basis[leave_row] = enter
        self.in_basis[enter] = True
        self.at_upper[enter] = False
        row = self.Binv[leave_row] / alpha[leave_row]
        self.Binv -= np.outer(alpha, row)
        self.Binv[leave_row] = row
        self.pivots += 1
        if self.pivots % 40 == 0:
            self.refactor()

    def full_x(self):
        xb = self.x_basic()
        full = np.where(self.at_upper & ~self.in_basis, self.ub, 0.0)
        full[~np.isfinite(full)] = 0.0
        full[self.basis] = xb
        return full


def _primal(tb: _Tableau, max_iter, tol):
    degenerate_run = 0
    for _ in range(max_iter):
        xB = tb.x_basic()
        d, _ = tb.reduced_costs()
        movable = ~tb.in_basis & (tb.ub > 0)
        cand = movable & (((~tb.at_upper) & (d < -tol)) | (tb.at_upper & (d > tol)))
        if not cand.any():
            return "optimal"
        idx = np.nonzero(cand)[0]
        bland = degenerate_run > 30
        e = idx[0] if bland else idx[np.argmax(np.abs(d[idx]))]
        direction = -1.0 if tb.at_upper[e] else 1.0
        alpha = tb.Binv @ tb.M[:, e]
        delta = -direction * alpha                 # change of x_B per unit step
        theta, leave, to_upper = tb.ub[e], -1, False
        for i in np.nonzero(np.abs(delta) > 1e-11)[0]:
            if delta[i] < 0:
                lim, hit_upper = max(xB[i], 0.0) / -delta[i], False
            else:
                ubi = tb.ub[tb.basis[i]]
                if not np.isfinite(ubi):
                    continue
                lim, hit_upper = max(ubi - xB[i], 0.0) / delta[i], True
            if leave < 0 and lim < theta:
                better = True
            elif leave >= 0 and lim < theta - 1e-13:
                better = True
            elif leave >= 0 and lim <= theta + 1e-13:
                # tie: Bland takes the smallest variable index, otherwise the
                # largest pivot element for stability
                better = (tb.basis[i] < tb.basis[leave]) if bland else \
                    (abs(delta[i]) > abs(delta[leave]))
            else:
                better = False
            if better:
                theta, leave, to_upper = lim, i, hit_upper
        if not np.isfinite(theta):
            return "unbounded"
        degenerate_run = degenerate_run + 1 if theta <= 1e-13 else 0
        if leave < 0:
            tb.at_upper[e] = not tb.at_upper[e]    # bound flip, basis unchanged
            continue
        tb.pivot(leave, e, alpha, to_upper)
    return "iteration_limit"


def _dual(tb: _Tableau, max_iter, tol):
    """Bounded dual simplex from a dual-feasible basis until x_B is within bounds."""
    for _ in range(max_iter):
        xB = tb.x_basic()
        ubB = tb.ub[tb.basis]
        low_viol = -xB
        up_viol = np.where(np.isfinite(ubB), xB - ubB, -np.inf)
        viol = np.maximum(low_viol, up_viol)
        r = int(np.argmax(viol))
        if viol[r] <= tol:
            return "optimal"
        to_upper = up_viol[r] > low_viol[r]
        d, _ = tb.reduced_costs()
        alpha_r = tb.Binv[r] @ tb.M                # row r of B^-1 [A I]
        nb = ~tb.in_basis & (tb.ub > 0)
        lo, hi = nb & ~tb.at_upper, nb & tb.at_upper
        if not to_upper:       # x_r must increase
            elig = (lo & (alpha_r < -1e-11)) | (hi & (alpha_r > 1e-11))
        else:                  # x_r must decrease
            elig = (lo & (alpha_r > 1e-11)) | (hi & (alpha_r < -1e-11))
        if not elig.any():
            return "infeasible"
        idx = np.nonzero(elig)[0]
        ratios = np.abs(d[idx]) / np.abs(alpha_r[idx])
        best = ratios.min()
        ties = idx[ratios <= best + 1e-13]
        e = ties[np.argmax(np.abs(alpha_r[ties]))]
        alpha = tb.Binv @ tb.M[:, e]
        tb.pivot(r, e, alpha, to_upper)
    return "iteration_limit"


def simplex_solve(A, b, c, u, max_iter=200000, tol=1e-10, perturb=1e-9,
                  seed=12345) -> SimplexResult:
    A = np.asarray(A, np.float64)
    b = np.asarray(b, np.float64).ravel()
    c = np.asarray(c, np.float64).ravel()
    u = np.asarray(u, np.float64).ravel()
    if np.any(b < 0):
        raise ValueError("simplex_solve needs b >= 0 (slack basis feasible)")
    tb = _Tableau(A, b, c, u)
    if perturb > 0:
        rng = np.random.default_rng(seed)
        tb.b = b + perturb * (1.0 + rng.random(b.size)) * np.maximum(1.0, np.abs(b))
    status = _primal(tb, max_iter, tol)
    if status == "optimal" and perturb > 0:
        tb.b = b.copy()
        tb.refactor()
        status = _dual(tb, max_iter, 1e-13)
        if status == "optimal":
            tb.refactor()
            status = _primal(tb, max_iter, tol)     # clean up any dual slip
    tb.refactor()
    full = tb.full_x()
    _, y = tb.reduced_costs()
    lam = -y
    x = full[:tb.n]
    return SimplexResult(x=x, objective=float(c @ x), lam=lam, reduced=c + A.T @ lam,
                         iterations=tb.pivots, status=status)


def kkt_residuals(A, b, c, u, x, lam):
    """Largest violation of each KKT condition of min c'x, Ax <= b, 0 <= x <= u.

    primal: max(Ax - b, -x, x - u);  dual: lam >= 0 and the sign of each reduced
    cost r = c + A'lam matching the active bound (r >= 0 at 0, r <= 0 at u,
    r = 0 strictly inside, r >= 0 where u = inf);  comp: max |lam_i (b - Ax)_i|;
    gap: c'x minus the dual objective -b'lam - u'max(0, -r).
    """
    A = np.asarray(A, np.float64)
    x = np.asarray(x, np.float64)
    lam = np.asarray(lam, np.float64)
    b = np.asarray(b, np.float64).ravel()
    u = np.asarray(u, np.float64).ravel()
    r = c + A.T @ lam
    slack = b - A @ x
    fin = np.isfinite(u)
    primal = max(float(np.max(-slack, initial=0.0)), float(np.max(-x, initial=0.0)),
                 float(np.max((x - u)[fin], initial=0.0)))
    tol_b = 1e-9 * np.maximum(1.0, np.abs(x))
    at_lo = x <= tol_b
    at_hi = fin & (x >= np.where(fin, u, 0) - tol_b)
    inside = ~at_lo & ~at_hi
    dual = max(float(np.max(-lam, initial=0.0)),
               float(np.max(-r[at_lo & ~at_hi], initial=0.0)),
               float(np.max(r[at_hi & ~at_lo], initial=0.0)),
               float(np.max(np.abs(r[inside]), initial=0.0)),
               float(np.max(-r[~fin], initial=0.0)))
    comp = float(np.max(np.abs(lam * slack), initial=0.0))
    dual_obj = -(b @ lam) - np.sum(np.where(fin, u, 0.0) * np.maximum(0.0, -r))
    gap = float(c @ x - dual_obj)
    return dict(primal=primal, dual=dual, comp=comp, gap=gap)


def solve_plan(lp, j: int, **kw) -> SimplexResult:
    """Solve plan j of an assembled App. A LP on its row-normalised form.

    Row scaling does not change x or c'x; the multipliers of the original rows
    are E times those of the scaled rows.
    """
    E = 1.0 / np.sqrt(np.sum(lp.A * lp.A, axis=1))
    A = lp.A * E[:, None]
    res = simplex_solve(A, lp.b[:, j] * E, lp.c, lp.u[:, j], **kw)
    lam = res.lam * E
    return dataclasses.replace(res, lam=lam, reduced=lp.c + lp.A.T @ lam)
