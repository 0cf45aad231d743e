"""The planning LP of App. A, its preconditioning (Sec. 3.C) and its objectives.

Oracle code (test infrastructure; see the package docstring).  Everything here
is FP64 and dense, written to be checked against the paper by eye.

The LP the solver works on is the dual LP of Eq. (dual_problem):

    minimize c'x  subject to  A x <= b,  l <= x <= u,

with the blocks of App. A.  Columns of A are the dose points (in the order
TS_k, TI_k, R_k, LD, O_m of the case) followed by the 8 * N_iso sector
variables; rows are the 24 * N_iso shot rows followed by the N_iso BOT rows.

    A = [ phi_TS'  phi_TI'  -phi_R'  -phi_LD'  -phi_O'  -C_S' ]
        [   0        0        0        0         0       T'   ]
    c = (-1, -1, 1, 1, 1, 0),  b = (0, w_BOT),  l = 0,
    u = (w_TS/N_TS, w_TI/N_TI, w_R/N_R, w_LD/N_LD, inf, inf),
    phi_alpha = Phi_alpha / D_alpha,  C_S = C / (D_T / phi_cal),
    C = I_Niso (x) I_8 (x) 1_{1x3},   T = I_Niso (x) 1_{8x1}.

Multi-target extension (end of App. A): one TS/TI/R block per target with
w_k,TS = q_k,A w_TS, w_k,TI = q_k,V w_TI, w_k,R = w_R / n, and D_T replaced by
the mean prescription in C_S.

The planning (primal) LP whose optimum F* equals -p* is the weighted sum of
Sec. 2.A: hinge penalties on target underdose, ring and low-dose overdose, and
the beam-on time, with hard OAR max-dose constraints.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from synth.cases import TS, TI, RING, LD, OAR


# ---------------------------------------------------------------------------
# App. A: the blocks of the LP
# ---------------------------------------------------------------------------

def point_sign(case) -> np.ndarray:
    """+1 for target points (TS, TI), -1 for ring, low-dose and OAR points.

    This is the sign with which phi_alpha' enters A (App. A), and c_p = -sign.
    """
    types = case.point_types()
    return np.where((types == TS) | (types == TI), 1.0, -1.0)


def point_threshold(case) -> np.ndarray:
    """D_alpha of each dose point (D_O for OAR points)."""
    thr = np.array([g.threshold for g in case.groups], np.float64)
    return thr[case.group]


def group_weights(case, weights) -> np.ndarray:
    """Objective weight w_{g,j} of every point group g and plan j (G x k).

    weights: (k, 4) rows (w_T, w_R, w_LD, w_BOT); w_TS = w_TI = w_T (App. A).
    OAR groups carry no weight (they are constraints): +inf is returned.
    """
    w = np.atleast_2d(np.asarray(weights, np.float64))
    out = np.empty((len(case.groups), w.shape[0]))
    for g, grp in enumerate(case.groups):
        if grp.type in (TS, TI):
            out[g] = grp.share * w[:, 0]
        elif grp.type == RING:
            out[g] = grp.share * w[:, 1]
        elif grp.type == LD:
            out[g] = grp.share * w[:, 2]
        else:
            out[g] = np.inf
    return out


def point_upper_bounds(case, weights, ld_mask=None) -> np.ndarray:
    """u of the dose-point block, N x k: w_{g,j} / N_{g,j}; +inf for OAR points.

    ld_mask (k x N bool, optional): the per-plan low-dose subsets p_j of the
    second pass.  A low-dose point outside p_j gets u = 0 and N_LD,j = |p_j|
    (Sec. 2.C.2: one shared point set, zero upper bound outside a plan's own
    points).
    """
    w = np.atleast_2d(np.asarray(weights, np.float64))
    k = w.shape[0]
    gw = group_weights(case, w)                       # G x k
    types = case.point_types()
    n = case.n_points
    member = np.ones((k, n), bool) if ld_mask is None else np.asarray(ld_mask, bool).copy()
    member[:, types != LD] = True
    u = np.empty((n, k))
    for g, grp in enumerate(case.groups):
        rows = np.nonzero(case.group == g)[0]
        if grp.type == OAR:
            u[rows] = np.inf
            continue
        for j in range(k):
            inside = member[j, rows]
            cnt = int(inside.sum())
            u[rows, j] = np.where(inside, gw[g, j] / cnt if cnt else 0.0, 0.0)
    return u


@dataclasses.dataclass
class LP:
    """min c'x s.t. A x <= b, 0 <= x <= u; b and u have one column per plan."""
    A: np.ndarray   # m_A x n_A
    b: np.ndarray   # m_A x k
    c: np.ndarray   # n_A
    u: np.ndarray   # n_A x k
    n_points: int
    n_iso: int
    n_sectors: int
    n_collimators: int

    @property
    def n_t(self):
        return self.n_iso * self.n_sectors * self.n_collimators

    @property
    def n_sec(self):
        return self.n_iso * self.n_sectors


def assemble(case, weights, ld_mask=None) -> LP:
    """The dense LP of App. A for every plan (weights: k x 4)."""
    w = np.atleast_2d(np.asarray(weights, np.float64))
    k = w.shape[0]
    n_iso, S, C = case.n_iso, case.n_sectors, case.n_collimators
    n_t, n_sec = n_iso * S * C, n_iso * S
    N = case.n_points
    m_A, n_A = n_t + n_iso, N + n_sec
    A = np.zeros((m_A, n_A))
    sigma = point_sign(case)
    A[:n_t, :N] = (np.asarray(case.dose, np.float64) * (sigma / point_threshold(case))[:, None]).T
    # C = I_Niso (x) I_8 (x) 1_{1x3}: sector (i,s) sums collimator columns (i,s,c)
    Cmat = np.kron(np.eye(n_sec), np.ones((1, C)))     # n_sec x n_t
    C_S = Cmat * (case.phi_cal / case.prescription_mean)
    A[:n_t, N:] = -C_S.T
    # T = I_Niso (x) 1_{8x1}
    T = np.kron(np.eye(n_iso), np.ones((S, 1)))        # n_sec x n_iso
    A[n_t:, N:] = T.T
    c = np.concatenate([-sigma, np.zeros(n_sec)])
    b = np.zeros((m_A, k))
    b[n_t:, :] = w[:, 3][None, :]
    u = np.vstack([point_upper_bounds(case, w, ld_mask), np.full((n_sec, k), np.inf)])
    return LP(A, b, c, u, N, n_iso, S, C)


# ---------------------------------------------------------------------------
# Sec. 3.C: preconditioning and step size
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class ScaledLP:
    """The LP after row normalisation E and BOT-column scaling beta.

    A_s = E A B with B = diag(1 (points), beta (sectors)); b_s = E b.  Because
    c and u of the sector block are 0 and +inf, the column scaling leaves c and
    u unchanged, and x_sec = beta * x_s,sec.  The multipliers of the original
    rows are E times those of the scaled rows.
    """
    lp: LP
    A: np.ndarray
    b: np.ndarray
    c: np.ndarray
    u: np.ndarray
    E: np.ndarray     # m_A row scales (1 / row 2-norm of the unscaled A)
    beta: float


def bot_scale(case, denominator=2000.0) -> float:
    """beta = (number of non-OAR dose points) / 2000 (Sec. 3.C)."""
    types = case.point_types()
    return float(np.count_nonzero(types != OAR)) / denominator


def precondition(lp: LP, beta: float, row_normalize=True) -> ScaledLP:
    """Normalise the rows of A to unit 2-norm, then scale the sector columns by beta."""
    if row_normalize:
        E = 1.0 / np.sqrt(np.sum(lp.A * lp.A, axis=1))
    else:
        E = np.ones(lp.A.shape[0])
    A = lp.A * E[:, None]
    A[:, lp.n_points:] *= beta
    return ScaledLP(lp, A, lp.b * E[:, None], lp.c.copy(), lp.u.copy(), E, float(beta))


def rho_rule(w_bot, rho0, w0_bot) -> np.ndarray:
    """rho_j = rho0 * sqrt(w0_BOT / w_BOT,j) (Eq. rho_rule), one value per plan."""
    w_bot = np.asarray(w_bot, np.float64)
    return rho0 * np.sqrt(w0_bot / w_bot)


# ---------------------------------------------------------------------------
# Sec. 2.A: the planning objective and bounds on its optimum
# ---------------------------------------------------------------------------

def sector_bot(case, t) -> np.ndarray:
    """Beam-on time variable of each isocentre: (phi_cal/D_T) max_s sum_c t_isc."""
    t = np.atleast_2d(np.asarray(t, np.float64).T).T       # n_t x k
    n_iso, S, C = case.n_iso, case.n_sectors, case.n_collimators
    per_sector = t.reshape(n_iso, S, C, -1).sum(axis=2)   # n_iso x S x k
    return (case.phi_cal / case.prescription_mean) * per_sector.max(axis=1)


def planning_objective(case, weights, t, ld_mask=None):
    """F_j(t) for every plan: hinge terms + w_BOT * sum_i tau_i.

    t: n_t x k shot times (t >= 0 expected).  Returns (F, terms, oar_ratio)
    where terms = (target underdose, ring overdose, low-dose overdose, BOT) and
    oar_ratio = max over OAR points of d_p / D_O (<= 1 when feasible).
    """
    w = np.atleast_2d(np.asarray(weights, np.float64))
    t = np.asarray(t, np.float64).reshape(case.n_t, -1)
    d = np.asarray(case.dose, np.float64) @ t                 # N x k
    ratio = d / point_threshold(case)[:, None]
    sigma = point_sign(case)
    hinge = np.maximum(0.0, sigma[:, None] * (1.0 - ratio))
    u = point_upper_bounds(case, w, ld_mask)
    types = case.point_types()
    terms = np.zeros((4, w.shape[0]))
    for idx, sel in enumerate([(types == TS) | (types == TI), types == RING, types == LD]):
        if sel.any():
            terms[idx] = np.sum(u[sel] * hinge[sel], axis=0)
    tau = sector_bot(case, t)
    terms[3] = w[:, 3] * tau.sum(axis=0)
    oar = types == OAR
    oar_ratio = ratio[oar].max(axis=0) if oar.any() else np.zeros(w.shape[0])
    return terms.sum(axis=0), terms, oar_ratio


def oar_feasible(case, t) -> np.ndarray:
    """Scale each plan's t by min(1, min_O D_O / d_O) so every OAR limit holds."""
    t = np.asarray(t, np.float64).reshape(case.n_t, -1)
    types = case.point_types()
    oar = types == OAR
    if not oar.any():
        return t.copy()
    d = np.asarray(case.dose, np.float64)[oar] @ t
    lim = point_threshold(case)[oar][:, None]
    with np.errstate(divide="ignore"):
        s = np.min(np.where(d > 0, lim / d, np.inf), axis=0)
    return t * np.minimum(1.0, s)[None, :]


def dual_feasible_point(lp: LP, x_points: np.ndarray, D_T: float, phi_cal: float):
    """A point feasible for the dual LP built from the dose-point block of x.

    Clip the points to [0, u]; give each sector the smallest value that
    satisfies its three shot rows; then scale all of x by one factor in (0, 1]
    so that every BOT row sum stays within w_BOT.  Returns x (n_A x k).
    """
    N, n_t, n_sec = lp.n_points, lp.n_t, lp.n_sec
    C = lp.n_collimators
    xp = np.clip(x_points, 0.0, lp.u[:N])
    shot = lp.A[:n_t, :N] @ xp                           # n_t x k
    need = np.maximum(0.0, shot.reshape(n_sec, C, -1).max(axis=1)) * (D_T / phi_cal)
    bot_sum = need.reshape(lp.n_iso, lp.n_sectors, -1).sum(axis=1)   # n_iso x k
    w_bot = lp.b[n_t:]                                   # n_iso x k
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(bot_sum > 0, w_bot / bot_sum, np.inf)
    theta = np.minimum(1.0, ratio.min(axis=0))
    return np.vstack([xp, need]) * theta[None, :]


def certify(case, weights, t, x_points, lp: LP | None = None, ld_mask=None):
    """Certified bounds on F*_j: U = F(t feasible) >= F* >= L = -c'x_hat.

    Returns dict(U, L, cert_gap = (U - L) / U).
    """
    if lp is None:
        lp = assemble(case, weights, ld_mask)
    tf = oar_feasible(case, np.maximum(0.0, np.asarray(t, np.float64).reshape(case.n_t, -1)))
    U = planning_objective(case, weights, tf, ld_mask)[0]
    xh = dual_feasible_point(lp, x_points, case.prescription_mean, case.phi_cal)
    L = -(lp.c @ xh)
    return dict(U=U, L=L, cert_gap=(U - L) / np.maximum(np.abs(U), 1e-300))
