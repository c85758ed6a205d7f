"""Relative KKT error on the original (unscaled) LP.  Test infrastructure only.

Follows Sec. 4 ("Optimality termination criteria") and the dual of eq. (lp)
in Sec. 2.1:

  * dual objective  -p(-y; lc, uc) - p(-r; lv, uv),  p(y; l, u) = u^T y+ - l^T y-
    (Sec. 1.2, notations), with 0 * inf taken as 0;
  * r is the projection of c - A^T y onto the sign set R (Sec. 2.1), so the
    fourth criterion of Sec. 4 vanishes identically and the third one is the
    distance of c - A^T y to R;
  * ||(L, U)||_2 is the 2-norm of the finite entries of (lc, uc) concatenated;
  * the single relative KKT number is the largest of the three ratios.
"""
from __future__ import annotations

import numpy as np


def proj_R(g, lv, uv):
    """Projection onto R (Sec. 2.1): R_j is the reals when both bounds are
    finite, [0, inf) with only lv finite, (-inf, 0] with only uv finite and
    {0} with neither."""
    fl = np.isfinite(lv)
    fu = np.isfinite(uv)
    r = np.where(fl & fu, g, 0.0)
    r = np.where(fl & ~fu, np.maximum(g, 0.0), r)
    r = np.where(~fl & fu, np.minimum(g, 0.0), r)
    return r


def _neg_p_of_neg(v, lo, hi):
    """-p(-v; lo, hi) = lo^T v+ - hi^T v-, summing only finite-bound terms."""
    vp = np.maximum(v, 0.0)
    vm = np.maximum(-v, 0.0)
    fl = np.isfinite(lo)
    fu = np.isfinite(hi)
    return float(np.sum(lo[fl] * vp[fl]) - np.sum(hi[fu] * vm[fu]))


def dual_objective(y, r, lc, uc, lv, uv):
    return _neg_p_of_neg(y, lc, uc) + _neg_p_of_neg(r, lv, uv)


def kkt(A, c, lc, uc, lv, uv, x, y):
    """Relative KKT parts at (x, y) for the original LP.

    Returns a dict with pobj, dobj, the absolute residuals and the relative
    gap / primal / dual errors, their maximum ``rel_kkt`` and r."""
    Ax = A @ x
    g = c - A.T @ y
    r = proj_R(g, lv, uv)
    pobj = float(c @ x)
    dobj = dual_objective(y, r, lc, uc, lv, uv)
    rho_p = float(np.linalg.norm(Ax - np.minimum(np.maximum(Ax, lc), uc)))
    rho_d = float(np.linalg.norm(g - r))
    bnd = np.concatenate([lc[np.isfinite(lc)], uc[np.isfinite(uc)]])
    nb = float(np.linalg.norm(bnd))
    nc = float(np.linalg.norm(c))
    rel_gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
    rel_p = rho_p / (1.0 + nb)
    rel_d = rho_d / (1.0 + nc)
    return dict(pobj=pobj, dobj=dobj, rho_p=rho_p, rho_d=rho_d, rel_gap=rel_gap,
                rel_primal=rel_p, rel_dual=rel_d, rel_kkt=max(rel_gap, rel_p, rel_d), r=r)
