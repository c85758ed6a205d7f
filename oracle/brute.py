"""Vertex enumeration for tiny bounded LPs.  Test infrastructure only.

An independent ground truth for the LP of eq. (lp) (Sec. 2.1): every finite
bound becomes a half-space g^T x >= h; every choice of n linearly independent
half-spaces taken with equality is a candidate vertex; the optimum of a
bounded feasible LP with at least one vertex is attained at a feasible one.
Only meant for n <= 8 and a few dozen half-spaces.
"""
from __future__ import annotations

import itertools

import numpy as np


def halfspaces(A, lc, uc, lv, uv):
    """Stack the finite bounds as rows of G x >= h."""
    A = np.asarray(A.todense()) if hasattr(A, "todense") else np.asarray(A)
    m, n = A.shape
    G, h = [], []
    for i in range(m):
        if np.isfinite(lc[i]):
            G.append(A[i]); h.append(lc[i])
        if np.isfinite(uc[i]):
            G.append(-A[i]); h.append(-uc[i])
    eye = np.eye(n)
    for j in range(n):
        if np.isfinite(lv[j]):
            G.append(eye[j]); h.append(lv[j])
        if np.isfinite(uv[j]):
            G.append(-eye[j]); h.append(-uv[j])
    return np.array(G), np.array(h)


def brute_force(A, c, lc, uc, lv, uv, feas_tol=1e-9):
    """Return (optimal value, an optimal vertex) by enumerating all vertices."""
    G, h = halfspaces(A, lc, uc, lv, uv)
    n = G.shape[1]
    best = np.inf
    best_x = None
    for S in itertools.combinations(range(G.shape[0]), n):
        M = G[list(S)]
        if abs(np.linalg.det(M)) < 1e-12:
            continue
        x = np.linalg.solve(M, h[list(S)])
        if np.all(G @ x >= h - feas_tol * (1.0 + np.abs(h))):
            val = float(c @ x)
            if val < best:
                best, best_x = val, x
    return best, best_x
