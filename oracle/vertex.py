"""Brute-force vertex enumeration for tiny LPs (pins the dense simplex).

Oracle code (test infrastructure).  An LP  min c'x, A x <= b, 0 <= x <= u  with
a bounded feasible set attains its minimum at a vertex: a point where n
linearly independent constraints are active.  For n <= 8 variables every
n-subset of the constraints can be tried, and the best feasible one is the
exact optimum.
"""
from __future__ import annotations

import itertools

import numpy as np


def enumerate_vertices(A, b, c, u, tol=1e-9, chunk=20000):
    """Return (p*, x*) by trying every basis of the constraint system."""
    A = np.asarray(A, np.float64)
    b = np.asarray(b, np.float64).ravel()
    c = np.asarray(c, np.float64).ravel()
    u = np.asarray(u, np.float64).ravel()
    m, n = A.shape
    if n > 10:
        raise ValueError("vertex enumeration is only for tiny LPs")
    fin = np.isfinite(u)
    G = np.vstack([A, -np.eye(n), np.eye(n)[fin]])
    h = np.concatenate([b, np.zeros(n), u[fin]])
    best, best_x = np.inf, None
    subsets = itertools.combinations(range(G.shape[0]), n)
    while True:
        block = list(itertools.islice(subsets, chunk))
        if not block:
            break
        idx = np.array(block)
        Gs = G[idx]                                     # B x n x n
        det = np.linalg.det(Gs)
        ok = np.abs(det) > 1e-10
        if not ok.any():
            continue
        xs = np.linalg.solve(Gs[ok], h[idx[ok]][..., None])[..., 0]   # B' x n
        feas = np.all(xs @ G.T <= h[None, :] + tol * (1.0 + np.abs(h[None, :])), axis=1)
        if not feas.any():
            continue
        vals = xs[feas] @ c
        i = int(np.argmin(vals))
        if vals[i] < best:
            best, best_x = float(vals[i]), xs[feas][i]
    return best, best_x
