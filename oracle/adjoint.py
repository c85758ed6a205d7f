"""Reverse mode of K unrolled iterations, controller frozen.  Test infrastructure only.

Not in the paper: an extension that differentiates the iteration map of
Sec. 2.2 (eq. pdhg) and Sec. 3 (reflected Halpern update, restarts).  The
controller -- eta, the primal weight omega of every iteration, the inner
Halpern index k and the restart iterations -- is recorded by a live forward
run and then held fixed ("frozen"), so the map from (c, lc, uc, lv, uv) to
the output is piecewise linear and its derivative is the chain rule through:

    v    = x - tau (c~ - A~^T y)          xhat = clamp(v, lv~, uv~)
    xbar = 2 xhat - x                      w    = A~ xbar - y / sigma
    yhat = sigma (clamp(w, lc~, uc~) - w)
    z'   = a ((1+gamma) zhat - gamma z) + (1-a) z0,  a = (k+1)/(k+2)
    at a restart after the iteration: z' = z0' = zhat.

The output is (xhat, yhat) of the last iteration, unscaled: x = D_c xhat,
y = D_r yhat.  A clamp whose argument ties a bound counts as active at that
bound, the lower bound first.  Infinite bounds get zero gradient.  D_r, D_c
and eta depend on A only and are constants here.
"""
from __future__ import annotations

import math

import numpy as np

from .pdhg import Params, fixed_point_residual, pid_update, power_norm, restart_decision, scale_problem, validate


def _setup(A, c, lc, uc, lv, uv, p: Params, eta=None):
    validate(A, c, lc, uc, lv, uv)
    At, dr, dc, ct, lct, uct, lvt, uvt = scale_problem(A, c, lc, uc, lv, uv, p.ruiz_iters,
                                                       p.pock_chambolle)
    if eta is None:
        if p.eta_override > 0:
            eta = float(p.eta_override)
        else:
            nrm, _ = power_norm(At, p.power_max_iter, p.power_tol)
            eta = 0.998 / nrm if nrm > 0 else 1.0
    return At, At.T.tocsr(), dr, dc, ct, lct, uct, lvt, uvt, eta


def unrolled_forward(A, c, lc, uc, lv, uv, params: Params | None, K: int, schedule=None, eta=None,
                     x0=None, y0=None):
    """Run exactly K iterations.  With ``schedule`` None the restart/PID
    controller runs live (restart tests every eval_freq iterations, as in the
    solver, but no termination test) and the decisions are recorded;
    otherwise the given schedule is replayed.  (x0, y0) is an optional warm
    start in the original space, held constant (no gradient flows to it).

    Returns dict(x, y, schedule, eta, dr, dc); x, y are unscaled."""
    p = params or Params()
    At, AtT, dr, dc, ct, lct, uct, lvt, uvt, eta = _setup(A, c, lc, uc, lv, uv, p, eta)
    m, n = A.shape
    gam = float(p.gamma)
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64) / dc
    y = np.zeros(m) if y0 is None else np.asarray(y0, dtype=np.float64) / dr
    xa = x.copy(); ya = y.copy()
    live = schedule is None
    if live:
        schedule = dict(omega=np.zeros(K), k=np.zeros(K, dtype=np.int64), restart=np.zeros(K, dtype=bool))
    omega = float(p.omega0)
    k = 0
    pid = {}
    r0 = math.inf
    r_prev = math.inf
    xh = np.zeros(n); yh = np.zeros(m)
    for t in range(K):
        if live:
            schedule["omega"][t] = omega
            schedule["k"][t] = k
        else:
            omega = float(schedule["omega"][t])
            k = int(schedule["k"][t])
        tau = eta / omega
        sigma = eta * omega
        g = AtT @ y
        xh = np.minimum(np.maximum(x - tau * (ct - g), lvt), uvt)
        xb = 2.0 * xh - x
        w = At @ xb - y / sigma
        yh = sigma * (np.minimum(np.maximum(w, lct), uct) - w)
        check = (t + 1) % p.eval_freq == 0
        if live and (k == 0 or check):
            r = fixed_point_residual(At, x - xh, y - yh, eta, omega)
            if k == 0:
                r0 = r
        a = (k + 1) / (k + 2)
        xn = a * ((1.0 + gam) * xh - gam * x) + (1.0 - a) * xa
        yn = a * ((1.0 + gam) * yh - gam * y) + (1.0 - a) * ya
        k += 1
        restart = False
        if live and check:
            restart = restart_decision(r, r0, r_prev, k, t + 1, p)
            if restart:
                dxn = float(np.linalg.norm(xh - xa))
                dyn = float(np.linalg.norm(yh - ya))
                omega = pid_update(omega, dxn, dyn, pid, p)
                r_prev = math.inf
            else:
                r_prev = r
            schedule["restart"][t] = restart
        elif not live:
            restart = bool(schedule["restart"][t])
        if restart:
            xa = xh.copy(); ya = yh.copy()
            x = xh.copy(); y = yh.copy()
            k = 0
        else:
            x, y = xn, yn
    return dict(x=dc * xh, y=dr * yh, schedule=schedule, eta=eta, dr=dr, dc=dc)


def unrolled_vjp(A, c, lc, uc, lv, uv, params: Params | None, K: int, schedule, eta, gx, gy,
                 x0=None, y0=None):
    """Gradient of <gx, x_out> + <gy, y_out> with respect to (c, lc, uc, lv, uv)
    for the frozen K-step map.  Stores every iterate (this is the slow,
    obviously correct version; no checkpointing)."""
    p = params or Params()
    At, AtT, dr, dc, ct, lct, uct, lvt, uvt, eta = _setup(A, c, lc, uc, lv, uv, p, eta)
    m, n = A.shape
    gam = float(p.gamma)
    # forward replay, keeping what the reverse pass needs
    xs, ys, vs, ws = [], [], [], []
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64) / dc
    y = np.zeros(m) if y0 is None else np.asarray(y0, dtype=np.float64) / dr
    xa = x.copy(); ya = y.copy()
    for t in range(K):
        omega = float(schedule["omega"][t]); k = int(schedule["k"][t])
        tau = eta / omega; sigma = eta * omega
        v = x - tau * (ct - AtT @ y)
        xh = np.minimum(np.maximum(v, lvt), uvt)
        w = At @ (2.0 * xh - x) - y / sigma
        yh = sigma * (np.minimum(np.maximum(w, lct), uct) - w)
        xs.append(x); ys.append(y); vs.append(v); ws.append(w)
        if schedule["restart"][t]:
            xa = xh.copy(); ya = yh.copy(); x = xh.copy(); y = yh.copy()
        else:
            a = (k + 1) / (k + 2)
            x = a * ((1.0 + gam) * xh - gam * x) + (1.0 - a) * xa
            y = a * ((1.0 + gam) * yh - gam * y) + (1.0 - a) * ya

    g_ct = np.zeros(n); g_lvt = np.zeros(n); g_uvt = np.zeros(n)
    g_lct = np.zeros(m); g_uct = np.zeros(m)
    gx_next = np.zeros(n); gy_next = np.zeros(m)   # adjoint of the state entering t+1
    gxa = np.zeros(n); gya = np.zeros(m)           # adjoint of the current epoch's anchor
    for t in range(K - 1, -1, -1):
        omega = float(schedule["omega"][t]); k = int(schedule["k"][t])
        tau = eta / omega; sigma = eta * omega
        a = (k + 1) / (k + 2)
        gx_in = np.zeros(n); gy_in = np.zeros(m)
        if t == K - 1:
            gxh = dc * gx
            gyh = dr * gy
        elif schedule["restart"][t]:
            # z_{t+1} = z0 = zhat: both the state and the next epoch's anchor
            gxh = gx_next + gxa
            gyh = gy_next + gya
            gxa = np.zeros(n); gya = np.zeros(m)
        else:
            gxh = a * (1.0 + gam) * gx_next
            gyh = a * (1.0 + gam) * gy_next
            gx_in -= a * gam * gx_next
            gy_in -= a * gam * gy_next
            gxa = gxa + (1.0 - a) * gx_next
            gya = gya + (1.0 - a) * gy_next
        # yhat = sigma (clamp(w) - w)
        w = ws[t]
        lo = w <= lct
        hi = (~lo) & (w >= uct)
        inside = ~(lo | hi)
        g_lct += np.where(lo, sigma * gyh, 0.0)
        g_uct += np.where(hi, sigma * gyh, 0.0)
        gw = np.where(inside, 0.0, -sigma * gyh)
        # w = A~ xbar - y / sigma
        gxb = AtT @ gw
        gy_in -= gw / sigma
        # xbar = 2 xhat - x
        gxh = gxh + 2.0 * gxb
        gx_in -= gxb
        # xhat = clamp(v), v = x - tau (c~ - A~^T y)
        v = vs[t]
        lo = v <= lvt
        hi = (~lo) & (v >= uvt)
        inside = ~(lo | hi)
        g_lvt += np.where(lo, gxh, 0.0)
        g_uvt += np.where(hi, gxh, 0.0)
        gv = np.where(inside, gxh, 0.0)
        gx_in += gv
        g_ct -= tau * gv
        gy_in += tau * (At @ gv)
        gx_next, gy_next = gx_in, gy_in
    # back to the original parametrisation
    return dict(c=dc * g_ct, lc=dr * g_lct, uc=dr * g_uct, lv=g_lvt / dc, uv=g_uvt / dc)
