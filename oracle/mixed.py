"""Mixed precision with iterative refinement (IR).  Test infrastructure only.

Not in the paper: an extension that runs the PDHG iteration of Sec. 2.2 /
Sec. 3 in FP32 and keeps FP64 accuracy with a refinement loop in the spirit of
Gleixner, Steffy and Wolter (2016).

Shifted coordinates.  Given an FP64 centre (xb, yb) in the scaled space and
powers of two P, D, write x = xb + x'/P, y = yb + y'/D.  Substituting into
eq. (pdhg) gives, exactly, the PDHG step of a correction problem on (x', y'):

    tau' = tau P / D,   sigma' = sigma D / P,
    c'   = D (c~ - A~^T yb),           lv' = P (lv~ - xb),  uv' = P (uv~ - xb),
    lc'  = P (lc~ - A~ xb),            uc' = P (uc~ - A~ xb),   b = D yb,
    xhat' = clamp(x' - tau'(c' - A~^T y'), lv', uv')
    h     = A~ (2 xhat' - x')
    yhat' = y' + sigma' (clamp(h - (b + y')/sigma', lc', uc') - h)

(the last line is sigma(clamp(w) - w) rewritten so that the large shift b
cancels exactly whenever a row bound is active).  The fixed-point residual
ratios and the PID error are invariant under the change of variables, so the
restart and primal-weight controller runs unchanged with omega' = omega D / P.

The loop.  Iterates, anchors and the data of the correction problem are FP32;
A~ is held in FP32 for the iteration and in FP64 for the checks.  Every
eval_freq iterations the FP64 point zhat = (xb + xhat'/P, yb + yhat'/D) is
formed and the relative KKT error of the original LP is evaluated in FP64;
the restart tests use r(z') accumulated in FP64.  At every restart the
refinement step re-centres: (xb, yb) <- zhat, then P, D are recomputed from
the FP64 primal violation dP and dual violation dD at the new centre
(infinity norms, scaled space): P = 2^floor(log2(1/dP)), D likewise, each at
most 2^12 times its previous value and at most 2^40; the correction data are
rebuilt from FP64 residuals and (x', y') and the anchor restart at 0.  This is
the FP64 method's own restart (anchor := zhat), so the outer loop costs no
extra iterations; each epoch solves the current correction problem to the
restart criterion.  The first epoch is the FP32 solve of the original LP
(centre at the start point, P = D = 1).
"""
from __future__ import annotations

import math
import time

import numpy as np

from .kkt import kkt as _kkt, proj_R
from .pdhg import (OPTIMAL, ITER_LIMIT, TIME_LIMIT, NUMERICAL, Params, pid_update, power_norm,
                   restart_decision, scale_problem, validate)

F32 = np.float32


def pow2_scale(delta, prev):
    """2^floor(log2(1/delta)), at least 1, at most min(2^12 prev, 2^40)."""
    cap = min(prev * 2.0 ** 12, 2.0 ** 40)
    if not (delta > 0) or not math.isfinite(delta):
        return cap
    s = 2.0 ** math.floor(math.log2(1.0 / delta))
    return float(min(max(s, 1.0), cap))


def shifted_step(A, AT, cd, tau, sigma, x, y):
    """One PDHG step in shifted coordinates (the formulas in the module
    docstring), in the dtype of the inputs.  Returns (xhat', yhat')."""
    two = x.dtype.type(2)
    xh = np.minimum(np.maximum(x - tau * (cd["c"] - AT @ y), cd["lv"]), cd["uv"])
    h = A @ (two * xh - x)
    w = h - (cd["b"] + y) / sigma
    yh = y + sigma * (np.minimum(np.maximum(w, cd["lc"]), cd["uc"]) - h)
    return xh, yh


def solve_mixed(A, c, lc, uc, lv, uv, params: Params | None = None, trace_iters=0):
    p = params or Params()
    validate(A, c, lc, uc, lv, uv)
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
    A32 = At.astype(F32)
    A32T = AtT.astype(F32)
    A32_64 = A32.astype(np.float64)       # FP32 values, FP64 accumulation
    gam = F32(p.gamma)

    def centre(xb, yb, P, D):
        """Correction data at the centre (xb, yb) with scales P, D (FP64 -> FP32)."""
        Ax = At @ xb
        gbar = ct - AtT @ yb
        return dict(c=(D * gbar).astype(F32), lv=(P * (lvt - xb)).astype(F32),
                    uv=(P * (uvt - xb)).astype(F32), lc=(P * (lct - Ax)).astype(F32),
                    uc=(P * (uct - Ax)).astype(F32), b=(D * yb).astype(F32))

    def violations(xb, yb):
        Ax = At @ xb
        gbar = ct - AtT @ yb
        dP = max(float(np.max(np.abs(Ax - np.minimum(np.maximum(Ax, lct), uct)), initial=0.0)),
                 float(np.max(np.abs(xb - np.minimum(np.maximum(xb, lvt), uvt)), initial=0.0)))
        dD = float(np.max(np.abs(gbar - proj_R(gbar, lvt, uvt)), initial=0.0))
        return dP, dD

    xb = np.zeros(n); yb = np.zeros(m)
    P = D = 1.0
    cd = centre(xb, yb, P, D)
    omega = float(p.omega0)            # in original units; omega' = omega D / P
    x = np.zeros(n, F32); y = np.zeros(m, F32)
    xa = x.copy(); ya = y.copy()
    k = 0; t = 0; restarts = 0
    pid = {}
    r0 = math.inf; r_prev = math.inf
    trace = dict(xh=[], yh=[]) if trace_iters else {}
    log = []
    while True:
        om = omega * D / P
        tau = F32(eta / om); sigma = F32(eta * om)
        xh, yh = shifted_step(A32, A32T, cd, tau, sigma, x, y)
        check = ((t + 1) % p.eval_freq == 0) or (t + 1 == p.max_iter)
        r = None
        if k == 0 or check:
            dx = (x - xh).astype(np.float64); dy = (y - yh).astype(np.float64)
            q = (om / eta) * float(dx @ dx) + 2.0 * float(dy @ (A32_64 @ dx)) + float(dy @ dy) / (eta * om)
            r = math.sqrt(max(q, 0.0))
            if k == 0:
                r0 = r
        k += 1; t += 1
        a = F32(k / (k + 1))
        x = a * ((F32(1) + gam) * xh - gam * x) + (F32(1) - a) * xa
        y = a * ((F32(1) + gam) * yh - gam * y) + (F32(1) - a) * ya
        if trace_iters and t <= trace_iters:
            trace["xh"].append(xb + xh.astype(np.float64) / P)
            trace["yh"].append(yb + yh.astype(np.float64) / D)
        if t in p.trace_at:  # further iterations kept by number (Params.trace_at)
            trace.setdefault("at", {})[t] = (xb + xh.astype(np.float64) / P, yb + yh.astype(np.float64) / D)
        if not check:
            continue
        xc = xb + xh.astype(np.float64) / P
        yc = yb + yh.astype(np.float64) / D
        kk = _kkt(A, c, lc, uc, lv, uv, dc * xc, dr * yc)
        log.append(dict(t=t, k=k, r=r, rel_kkt=kk["rel_kkt"], P=P, D=D, omega=omega))
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
            info.update(restarts=restarts)
            return dict(x=dc * xc, y=dr * yc, r=kk["r"], status=status, iters=t,
                        info=info, eta=eta, omega=omega, log=log, trace=trace)
        if not restart_decision(r, r0, r_prev, k, t, p):
            r_prev = r
            continue
        restarts += 1
        dxn = float(np.linalg.norm((xh - xa).astype(np.float64)))
        dyn = float(np.linalg.norm((yh - ya).astype(np.float64)))
        om = pid_update(om, dxn, dyn, pid, p)
        omega = om * P / D
        # refinement: re-centre at zhat, rescale, rebuild the correction data
        xb, yb = xc, yc
        dP, dD = violations(xb, yb)
        P = pow2_scale(dP, P)
        D = pow2_scale(dD, D)
        cd = centre(xb, yb, P, D)
        x = np.zeros(n, F32); y = np.zeros(m, F32)
        xa = x.copy(); ya = y.copy()
        k = 0
        r_prev = math.inf
