"""Reference scaled-form ADMM of Sec. 2.B, batched over plans (FP64).

Oracle code (test infrastructure).  The split of Eq. (dual_problem_admm) keeps
copies z1 in [l, u] and z2 <= b of x1 and x2 = A x1.  One iteration, in the
order of Eq. (admm) with the x-step in the closed form that follows
Eq. (partial_elimination):

    W   = z1 - y1 - c / rho
    v   = S^{-1} (A W - z2 + y2),        S = A A' + I
    x1  = W - A' v
    x2  = v + z2 - y2
    z1' = clip(x1 + y1, l, u)
    z2' = min(x2 + y2, b)
    y1' = y1 + x1 - z1'
    y2' = y2 + x2 - z2'

Plans are columns (Sec. 2.B, last paragraph): W, v, x, y, z, u and b are
matrices with one column per weight vector, and rho is one value per plan
(Sec. 3.C).  S is the same for every plan and iteration, so it is factored once
(Cholesky) and each x-step is two triangular solves.  The solution of the
planning LP is rho * y2 (multipliers of the scaled rows), mapped back through
the row scales E.

The block system printed as Eq. (eq_system) has +I in its lower-right corner;
the x-step's optimality conditions give -I there, and Eq. (partial_elimination)
and the closed form agree with -I.  This module follows those two equations.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy import linalg

from .lp import ScaledLP


@dataclasses.dataclass
class ADMMState:
    z1: np.ndarray   # n_A x k
    y1: np.ndarray   # n_A x k
    z2: np.ndarray   # m_A x k
    y2: np.ndarray   # m_A x k
    x1: np.ndarray | None = None
    x2: np.ndarray | None = None
    z1_prev: np.ndarray | None = None
    z2_prev: np.ndarray | None = None
    iterations: int = 0

    def copy(self):
        return ADMMState(*(None if a is None else a.copy() for a in
                           (self.z1, self.y1, self.z2, self.y2, self.x1, self.x2,
                            self.z1_prev, self.z2_prev)), iterations=self.iterations)


def zero_state(slp: ScaledLP, k: int) -> ADMMState:
    m, n = slp.A.shape
    return ADMMState(np.zeros((n, k)), np.zeros((n, k)), np.zeros((m, k)), np.zeros((m, k)))


def schur_factor(slp: ScaledLP):
    """Cholesky factor of S = A A' + I (Eq. partial_elimination)."""
    S = slp.A @ slp.A.T + np.eye(slp.A.shape[0])
    return linalg.cho_factor(S, lower=True), S


def admm_iterate(slp: ScaledLP, rho, iters: int, state: ADMMState | None = None,
                 factor=None, alpha: float = 1.0) -> ADMMState:
    """Run `iters` iterations of Eq. (admm) from `state` (zeros if None).

    alpha != 1: over-relaxation (an extension; the paper uses alpha = 1): the
    z- and y-steps take x_hat = alpha x + (1 - alpha) z in place of x, with z the
    copies before the step.  The residuals keep the unrelaxed x."""
    rho = np.asarray(rho, np.float64).ravel()
    k = rho.size
    st = zero_state(slp, k) if state is None else state.copy()
    if factor is None:
        factor, _ = schur_factor(slp)
    A, c, b, u = slp.A, slp.c, slp.b, slp.u
    c_over_rho = c[:, None] / rho[None, :]
    for _ in range(iters):
        W = st.z1 - st.y1 - c_over_rho
        v = linalg.cho_solve(factor, A @ W - st.z2 + st.y2)
        x1 = W - A.T @ v
        x2 = v + st.z2 - st.y2
        x1h = x1 if alpha == 1.0 else alpha * x1 + (1.0 - alpha) * st.z1
        x2h = x2 if alpha == 1.0 else alpha * x2 + (1.0 - alpha) * st.z2
        z1 = np.clip(x1h + st.y1, 0.0, u)
        z2 = np.minimum(x2h + st.y2, b)
        st.z1_prev, st.z2_prev = st.z1, st.z2
        st.y1 = st.y1 + x1h - z1
        st.y2 = st.y2 + x2h - z2
        st.z1, st.z2, st.x1, st.x2 = z1, z2, x1, x2
        st.iterations += 1
    return st


def shot_times(slp: ScaledLP, rho, state: ADMMState):
    """Primal solution rho * y2 mapped back to the unscaled rows: (t, tau)."""
    rho = np.asarray(rho, np.float64).ravel()
    lam = slp.E[:, None] * rho[None, :] * state.y2
    n_t = slp.lp.n_t
    return lam[:n_t], lam[n_t:]


def dual_objective(slp: ScaledLP, state: ADMMState):
    """c' z1 for each plan (the dual LP objective at the box-feasible copy)."""
    return slp.c @ state.z1


def residuals(slp: ScaledLP, rho, state: ADMMState):
    """Relative primal and dual residuals per plan (scaled form, both blocks).

    r_pri  = ||x - z|| / max(||x||, ||z||)
    r_dual = rho ||z - z_prev|| / ||rho y||
    """
    rho = np.asarray(rho, np.float64).ravel()
    x = np.vstack([state.x1, state.x2])
    z = np.vstack([state.z1, state.z2])
    zp = np.vstack([state.z1_prev, state.z2_prev])
    y = np.vstack([state.y1, state.y2])
    nx, nz = np.linalg.norm(x, axis=0), np.linalg.norm(z, axis=0)
    r_pri = np.linalg.norm(x - z, axis=0) / np.maximum(np.maximum(nx, nz), 1e-300)
    r_dual = (rho * np.linalg.norm(z - zp, axis=0)
              / np.maximum(rho * np.linalg.norm(y, axis=0), 1e-300))
    return r_pri, r_dual


def admm_adaptive(slp: ScaledLP, rho, iters: int, check_every: int, mu: float = 10.0,
                  tau: float = 2.0, rho_range: float = 1e3, state: ADMMState | None = None,
                  factor=None, alpha: float = 1.0):
    """Eq. (admm) with per-plan step sizes balanced at every check.

    The step sizes start from the rule of Sec. 3.C (rho) and, after every
    `check_every` iterations, each plan's rho is multiplied by tau when its
    relative primal residual exceeds mu times its relative dual residual, and
    divided by tau in the opposite case (residual balancing), within
    [rho / rho_range, rho * rho_range] of its starting value.  The scaled duals
    are multiplied by rho_old / rho_new so that the multipliers rho * y, and
    hence the iterate, are unchanged by the switch.  S does not depend on rho,
    so no refactorisation is needed.  Returns (state, final rho).
    """
    rho_start = np.asarray(rho, np.float64).ravel()
    rho = rho_start.copy()
    st = zero_state(slp, rho.size) if state is None else state.copy()
    if factor is None:
        factor, _ = schur_factor(slp)
    done = 0
    while done < iters:
        n = min(check_every, iters - done)
        st = admm_iterate(slp, rho, n, st, factor, alpha)
        done += n
        if n < check_every:
            break
        r_pri, r_dual = residuals(slp, rho, st)
        new = rho.copy()
        up = r_pri > mu * r_dual
        down = r_dual > mu * r_pri
        new[up] *= tau
        new[down] /= tau
        new = np.clip(new, rho_start / rho_range, rho_start * rho_range)
        scale = rho / new
        st.y1 = st.y1 * scale[None, :]
        st.y2 = st.y2 * scale[None, :]
        rho = new
    return st, rho
