"""HiGHS (through scipy.optimize.linprog) as an independent reference solver.

Maps the LP  min c^T x, lc <= Ax <= uc, lv <= x <= uv  to linprog's
A_ub/A_eq form and maps its marginals back to the sign convention of the
paper's dual (y_i >= 0 on an active lower row bound, <= 0 on an active upper).
"""
import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog


def highs(A, c, lc, uc, lv, uv):
    A = sp.csr_matrix(A)
    m = A.shape[0]
    eq = (lc == uc) & np.isfinite(lc)
    lo = np.isfinite(lc) & ~eq
    hi = np.isfinite(uc) & ~eq
    blocks, rhs, kinds = [], [], []
    if lo.any():
        blocks.append(-A[lo]); rhs.append(-lc[lo]); kinds.append(("lo", np.nonzero(lo)[0]))
    if hi.any():
        blocks.append(A[hi]); rhs.append(uc[hi]); kinds.append(("hi", np.nonzero(hi)[0]))
    A_ub = sp.vstack(blocks).tocsr() if blocks else None
    b_ub = np.concatenate(rhs) if rhs else None
    A_eq = A[eq] if eq.any() else None
    b_eq = lc[eq] if eq.any() else None
    bounds = [(None if not np.isfinite(a) else a, None if not np.isfinite(b) else b) for a, b in zip(lv, uv)]
    res = linprog(c, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=b_eq, bounds=bounds, method="highs")
    assert res.status == 0, res.message
    y = np.zeros(m)
    if eq.any():
        y[eq] = res.eqlin.marginals
    off = 0
    for kind, idx in kinds:
        mg = res.ineqlin.marginals[off:off + idx.size]
        off += idx.size
        if kind == "lo":
            y[idx] += -mg
        else:
            y[idx] += mg
    return res.fun, res.x, y
