"""Restarted reflected Halpern PDHG, step by step, in FP64.  Test infrastructure only.

The method (arXiv 2507.14051):

  * the LP of eq. (lp), Sec. 2.1, solved through the saddle problem (lp-pd);
  * one PDHG step, eq. (pdhg) in Sec. 2.2, with tau = eta/omega and
    sigma = eta*omega;
  * the reflected Halpern update of Sec. 3:
        z^{k+1} = (k+1)/(k+2) ((1+gamma) PDHG(z^k) - gamma z^k) + 1/(k+2) z^0 ;
  * the fixed-point residual r(z) = ||z - PDHG(z)||_P in the norm of Sec. 2.2,
    P = [[omega/eta I, A^T], [A, 1/(eta omega) I]], and the three restart tests
    of Sec. 3 (sufficient decay, necessary decay with no local progress,
    artificial restart), the anchor reset to the current solution;
  * the constant stepsize eta = 0.998 / ||A||_2 with ||A||_2 from power
    iteration (Sec. 3, stepsize);
  * the PID update of log omega at each restart (Sec. 3, primal weight
    update), starting from omega = 1;
  * all-zero start (Sec. 4, initialization) and the relative KKT test on the
    original LP (Sec. 4).

Readings taken where the paper is silent or garbled (each is a parameter):

  * the bilinear term: the update rule and the dual constraint c - A^T y = r
    fix the sign; the "+y^T A x" printed in (lp-pd) is read as a typo;
  * the dual step is written  y+ = sigma (clamp(w, lc, uc) - w),
    w = A(2x+ - x) - y/sigma, which equals the printed form exactly;
  * gamma = 1; restart betas (0.2, 0.8, 0.36); PID gains (0.99, 0.01, 0);
  * the restart and termination tests run every ``eval_freq`` iterations and
    at ``max_iter``; "r(z^{n,k-1})" is the previous check of the same epoch
    (+inf at the start of an epoch); r(z^{n,0}) is measured exactly at the
    first iteration of each epoch; k and T count PDHG applications, k within
    the epoch and T in total, both after the increment;
  * the new anchor at a restart is the PDHG output zhat = PDHG(z^{n,k}); the
    KKT test is taken at zhat, which lies in X x Y;
  * PID error e = log(omega ||xhat - x^0|| / ||yhat - y^0||) in the scaled
    space; the sum includes the current e; the derivative term starts at 0;
    the update is skipped if either distance is below ``pid_min_norm``;
  * preconditioning: Ruiz infinity-norm equilibration then one Pock-Chambolle
    pass with alpha = 1 (the paper names preconditioning but not its kind);
  * power iteration from the all-1/sqrt(n) vector, stopping when sqrt of the
    Rayleigh-type estimate changes by at most power_tol relative;
    eta = 1 when ||A|| = 0;  r^2 is clamped at 0 before the square root.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .kkt import kkt as _kkt

OPTIMAL, ITER_LIMIT, TIME_LIMIT, NUMERICAL = 0, 1, 2, 3


@dataclass
class Params:
    tol: float = 1e-8
    max_iter: int = 10_000_000
    time_limit_s: float = 3600.0
    eval_freq: int = 64
    gamma: float = 1.0
    beta_sufficient: float = 0.2
    beta_necessary: float = 0.8
    beta_artificial: float = 0.36
    kp: float = 0.99
    ki: float = 0.01
    kd: float = 0.0
    omega0: float = 1.0
    eta_override: float = 0.0       # <= 0: power iteration
    ruiz_iters: int = 10
    pock_chambolle: int = 1
    power_max_iter: int = 5000
    power_tol: float = 1e-8
    restart_to_current: int = 0     # 0: new anchor = PDHG(z); 1: the Halpern iterate z
    pid_min_norm: float = 1e-10
    trace_iters: int = 0
    trace_at: tuple = ()            # further iterations t whose (xhat, yhat, x, y) are kept in trace["at"][t]


@dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    r: np.ndarray
    status: int
    iters: int
    restarts: int
    info: dict
    omega: float
    eta: float
    dr: np.ndarray
    dc: np.ndarray
    trace: dict = field(default_factory=dict)
    log: list = field(default_factory=list)


# ----------------------------------------------------------------------------- O1
def validate(A, c, lc, uc, lv, uv):
    """Input contract: CSR with in-range, strictly increasing columns per row,
    no NaN anywhere, lower <= upper, no lower bound of +inf and no upper bound
    of -inf.  Raises ValueError."""
    if not sp.isspmatrix_csr(A):
        raise ValueError("A must be CSR")
    m, n = A.shape
    ip = np.asarray(A.indptr)
    ix = np.asarray(A.indices)
    if ip.size != m + 1 or ip[0] != 0 or np.any(np.diff(ip) < 0):
        raise ValueError("row pointers must start at 0 and be nondecreasing")
    if ix.size != ip[-1]:
        raise ValueError("row pointers do not match the number of nonzeros")
    if ix.size and (ix.min() < 0 or ix.max() >= n):
        raise ValueError("column index out of range")
    for i in range(m):
        seg = ix[ip[i]:ip[i + 1]]
        if seg.size > 1 and np.any(np.diff(seg) <= 0):
            raise ValueError(f"row {i}: columns not strictly increasing")
    if np.any(np.isnan(A.data)) or np.any(np.isinf(A.data)):
        raise ValueError("matrix values must be finite")
    for name, v, size in (("c", c, n), ("lc", lc, m), ("uc", uc, m), ("lv", lv, n), ("uv", uv, n)):
        if np.asarray(v).shape != (size,):
            raise ValueError(f"{name} has the wrong length")
        if np.any(np.isnan(v)):
            raise ValueError(f"{name} contains NaN")
    if np.any(np.isinf(c)):
        raise ValueError("c must be finite")
    for lo, hi, nm in ((lc, uc, "row"), (lv, uv, "column")):
        if np.any(lo > hi):
            raise ValueError(f"{nm} lower bound above upper bound")
        if np.any(lo == np.inf) or np.any(hi == -np.inf):
            raise ValueError(f"{nm} bound of the wrong infinity")


# ----------------------------------------------------------------------------- O2
def rescale(A, ruiz_iters=10, pock_chambolle=1):
    """Diagonal preconditioning  A~ = D_r A D_c.

    Ruiz: each pass divides row i by sqrt(max_j |A~_ij|) and column j by
    sqrt(max_i |A~_ij|) (1 for an empty row or column), both measured on the
    same A~.  Pock-Chambolle (alpha = 1): the same with sums of |A~_ij|.
    Returns (A~, d_r, d_c)."""
    m, n = A.shape
    At = A.copy().astype(np.float64)
    dr = np.ones(m)
    dc = np.ones(n)

    def apply(rho, kap):
        nonlocal At, dr, dc
        At = sp.diags(1.0 / rho) @ At @ sp.diags(1.0 / kap)
        At = sp.csr_matrix(At)
        dr = dr / rho
        dc = dc / kap

    for _ in range(ruiz_iters):
        absA = abs(At)
        rmax = np.asarray(absA.max(axis=1).todense()).ravel() if m else np.zeros(0)
        cmax = np.asarray(absA.max(axis=0).todense()).ravel() if n else np.zeros(0)
        rho = np.where(rmax > 0, np.sqrt(rmax), 1.0)
        kap = np.where(cmax > 0, np.sqrt(cmax), 1.0)
        apply(rho, kap)
    if pock_chambolle:
        absA = abs(At)
        rsum = np.asarray(absA.sum(axis=1)).ravel()
        csum = np.asarray(absA.sum(axis=0)).ravel()
        rho = np.where(rsum > 0, np.sqrt(rsum), 1.0)
        kap = np.where(csum > 0, np.sqrt(csum), 1.0)
        apply(rho, kap)
    At.sort_indices()
    return At, dr, dc


# ----------------------------------------------------------------------------- O3
def power_norm(At, max_iter=5000, tol=1e-8):
    """Estimate ||A~||_2 by power iteration on A~^T A~ (Sec. 3, stepsize).

    v starts at 1/sqrt(n) everywhere; each pass u = A~^T (A~ v), s = ||u||,
    v = u/s; stop when |sqrt(s) - sqrt(s_prev)| <= tol sqrt(s).
    Returns (estimate, passes)."""
    m, n = At.shape
    if n == 0 or m == 0:
        return 0.0, 0
    AtT = At.T.tocsr()
    v = np.full(n, 1.0 / math.sqrt(n))
    prev = None
    s = 0.0
    it = 0
    for it in range(1, max_iter + 1):
        u = AtT @ (At @ v)
        s = float(np.linalg.norm(u))
        if s == 0.0:
            return 0.0, it
        v = u / s
        root = math.sqrt(s)
        if prev is not None and abs(root - prev) <= tol * root:
            break
        prev = root
    return math.sqrt(s), it


def pdhg_operator(At, AtT, ct, lvt, uvt, lct, uct, tau, sigma, x, y):
    """One PDHG step, eq. (pdhg), in the scaled space.  Returns (xhat, yhat, h)
    with h = A~ (2 xhat - x)."""
    g = AtT @ y
    xh = np.minimum(np.maximum(x - tau * (ct - g), lvt), uvt)
    xb = 2.0 * xh - x
    h = At @ xb
    w = h - y / sigma
    yh = sigma * (np.minimum(np.maximum(w, lct), uct) - w)
    return xh, yh, h


def fixed_point_residual(At, dx, dy, eta, omega):
    """r(z) = ||dz||_P with dz = z - PDHG(z) (Sec. 2.2 norm, Sec. 3 metric).

    r^2 = (omega/eta)||dx||^2 + 2 dy^T A~ dx + 1/(eta omega)||dy||^2, clamped
    at zero before the root."""
    q = (omega / eta) * float(dx @ dx) + 2.0 * float(dy @ (At @ dx)) + float(dy @ dy) / (eta * omega)
    return math.sqrt(max(q, 0.0))


def scale_problem(lp_A, c, lc, uc, lv, uv, ruiz_iters, pock_chambolle):
    At, dr, dc = rescale(lp_A, ruiz_iters, pock_chambolle)
    ct = dc * c
    lvt = lv / dc
    uvt = uv / dc
    lct = dr * lc
    uct = dr * uc
    return At, dr, dc, ct, lct, uct, lvt, uvt



# ----------------------------------------------------------------------------- controller
def restart_decision(r, r0, r_prev, k, t, p: Params):
    """The three restart tests of Sec. 3 (adaptive restart): sufficient decay,
    necessary decay with no local progress, artificial restart.  k and t are
    the inner and total iteration counts after the increment."""
    return (r <= p.beta_sufficient * r0) or \
           (r <= p.beta_necessary * r0 and r > r_prev) or \
           (k >= p.beta_artificial * t)


def pid_update(omega, dxn, dyn, state, p: Params):
    """PID control of log omega (Sec. 3, primal weight update).

    e = log(omega ||dx|| / ||dy||);  log omega <- log omega - (Kp e + Ki sum e + Kd (e - e_prev)).
    ``state`` is a dict holding the running sum and the previous error; it is
    updated in place.  Skipped when either distance is below pid_min_norm."""
    if not (dxn > p.pid_min_norm and dyn > p.pid_min_norm):
        return omega
    e = math.log(omega * dxn / dyn)
    state["sum"] = state.get("sum", 0.0) + e
    de = 0.0 if state.get("prev") is None else e - state["prev"]
    state["prev"] = e
    return math.exp(math.log(omega) - (p.kp * e + p.ki * state["sum"] + p.kd * de))

# ----------------------------------------------------------------------------- O4-O7
def solve(A, c, lc, uc, lv, uv, params: Params | None = None, x0=None, y0=None):
    """Restarted reflected Halpern PDHG to the relative KKT tolerance.

    Returns a Result whose x, y, r are in the original (unscaled) space."""
    p = params or Params()
    validate(A, c, lc, uc, lv, uv)
    if p.max_iter < 1 or p.eval_freq < 1:
        raise ValueError("max_iter and eval_freq must be positive")
    t_start = time.perf_counter()
    m, n = A.shape
    At, dr, dc, ct, lct, uct, lvt, uvt = scale_problem(A, c, lc, uc, lv, uv, p.ruiz_iters,
                                                       p.pock_chambolle)
    AtT = At.T.tocsr()
    if p.eta_override > 0:
        eta = float(p.eta_override)
    else:
        nrm, _ = power_norm(At, p.power_max_iter, p.power_tol)
        eta = 0.998 / nrm if nrm > 0 else 1.0
    t_iter = time.perf_counter()

    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64) / dc
    y = np.zeros(m) if y0 is None else np.asarray(y0, dtype=np.float64) / dr
    xa = x.copy()
    ya = y.copy()
    omega = float(p.omega0)
    gam = float(p.gamma)
    k = 0
    t = 0
    restarts = 0
    pid = {}
    r0 = math.inf
    r_prev = math.inf
    trace = {}
    if p.trace_iters > 0:
        T = p.trace_iters
        trace = dict(xh=np.zeros((T, n)), yh=np.zeros((T, m)), x=np.zeros((T, n)), y=np.zeros((T, m)))
    if p.trace_at:
        trace["at"] = {}
    log = []

    while True:
        tau = eta / omega
        sigma = eta * omega
        xh, yh, _ = pdhg_operator(At, AtT, ct, lvt, uvt, lct, uct, tau, sigma, x, y)
        check = ((t + 1) % p.eval_freq == 0) or (t + 1 == p.max_iter)
        r = None
        if k == 0 or check:
            r = fixed_point_residual(At, x - xh, y - yh, eta, omega)
            if k == 0:
                r0 = r
        k += 1
        t += 1
        a = k / (k + 1)
        x = a * ((1.0 + gam) * xh - gam * x) + (1.0 - a) * xa
        y = a * ((1.0 + gam) * yh - gam * y) + (1.0 - a) * ya
        if t <= p.trace_iters:
            trace["xh"][t - 1] = xh
            trace["yh"][t - 1] = yh
            trace["x"][t - 1] = x
            trace["y"][t - 1] = y
        if t in p.trace_at:
            trace["at"][t] = (xh.copy(), yh.copy(), x.copy(), y.copy())
        if not check:
            continue

        xu = dc * xh
        yu = dr * yh
        kk = _kkt(A, c, lc, uc, lv, uv, xu, yu)
        entry = dict(t=t, k=k, r=r, r0=r0, rel_kkt=kk["rel_kkt"], rel_gap=kk["rel_gap"],
                     rel_primal=kk["rel_primal"], rel_dual=kk["rel_dual"], omega=omega, restart=False)
        log.append(entry)
        status = None
        if not all(math.isfinite(v) for v in (kk["pobj"], kk["dobj"], kk["rho_p"], kk["rho_d"], r)):
            status = NUMERICAL
        elif kk["rel_kkt"] <= p.tol:
            status = OPTIMAL
        elif t >= p.max_iter:
            status = ITER_LIMIT
        elif time.perf_counter() - t_start >= p.time_limit_s:
            status = TIME_LIMIT
        if status is not None:
            info = {key: kk[key] for key in ("pobj", "dobj", "rel_gap", "rel_primal", "rel_dual", "rel_kkt")}
            info["setup_s"] = t_iter - t_start
            info["iter_s"] = time.perf_counter() - t_iter
            return Result(xu, yu, kk["r"], status, t, restarts, info, omega, eta, dr, dc, trace, log)

        if restart_decision(r, r0, r_prev, k, t, p):
            entry["restart"] = True
            restarts += 1
            dxn = float(np.linalg.norm(xh - xa))
            dyn = float(np.linalg.norm(yh - ya))
            omega = pid_update(omega, dxn, dyn, pid, p)
            if p.restart_to_current:
                xa = x.copy()
                ya = y.copy()
            else:
                xa = xh.copy()
                ya = yh.copy()
                x = xh.copy()
                y = yh.copy()
            k = 0
            r_prev = math.inf
        else:
            r_prev = r
