"""Pins of the oracle's reverse mode (frozen controller) and of its mixed
precision / iterative refinement, against independent computations."""
import math

import numpy as np
import pytest
import torch

import lpgen
import oracle
from oracle.adjoint import unrolled_forward, unrolled_vjp
from oracle.mixed import shifted_step, solve_mixed
from oracle.pdhg import Params, pdhg_operator, scale_problem
from tests._highs import highs


def _lp_small(seed=1):
    return lpgen.config("c2", seed=seed, scale=0.001)     # m=100, n=200, 8 nnz/row


def _loss_grads(lp, out, xt):
    gx = 2.0 * (out["x"] - xt) + lp.c
    gy = np.zeros(lp.m)
    return gx, gy


def _flat(d, lp):
    return np.concatenate([d["c"], d["lc"][np.isfinite(lp.lc)], d["uc"][np.isfinite(lp.uc)],
                           d["lv"][np.isfinite(lp.lv)], d["uv"][np.isfinite(lp.uv)]])


@pytest.mark.parametrize("seed", [1, 2])
def test_vjp_matches_central_differences(seed):
    lp = _lp_small(seed)
    p = Params(eval_freq=16)
    K = 300
    fw = unrolled_forward(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p, K)
    sched, eta = fw["schedule"], fw["eta"]
    assert sched["restart"].sum() >= 2           # the frozen map crosses restarts
    rng = np.random.default_rng(seed)
    gx = rng.standard_normal(lp.n); gy = rng.standard_normal(lp.m)
    g = unrolled_vjp(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p, K, sched, eta, gx, gy)
    d = lpgen.directions(lp, seed)
    h = 1e-6

    def F(s):
        o = unrolled_forward(lp.A, lp.c + s * d["c"], lp.lc + s * d["lc"], lp.uc + s * d["uc"],
                             lp.lv + s * d["lv"], lp.uv + s * d["uv"], p, K, schedule=sched, eta=eta)
        return gx @ o["x"] + gy @ o["y"]

    fd = kink_free_central_difference(F, h)
    an = sum(float(g[key] @ np.where(np.isfinite(d[key]), d[key], 0.0)) for key in d)
    assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3)


def kink_free_central_difference(F, h, tries=12):
    """Central difference of a piecewise-linear F at 0.  A clamp that changes
    side inside [-h, h] shows up as one-sided slopes that disagree; h is then
    halved until they agree, so the difference is taken on one linear piece."""
    f0 = F(0.0)
    for _ in range(tries):
        fp, fm = F(h), F(-h)
        fwd, bwd = (fp - f0) / h, (f0 - fm) / h
        cen = (fp - fm) / (2 * h)
        if abs(fwd - bwd) <= 1e-7 * max(abs(cen), 1e-3) + 1e-12 * abs(f0) / h:
            return cen
        h *= 0.5
    raise AssertionError("no kink-free step found")


def _torch_frozen_map(A, ct, lct, uct, lvt, uvt, dr, dc, eta, sched, K, gamma):
    """The frozen K-step map written directly in torch (CPU, FP64), dense A."""
    m, n = A.shape
    x = torch.zeros(n, dtype=torch.float64); y = torch.zeros(m, dtype=torch.float64)
    xa, ya = x, y
    for t in range(K):
        om = float(sched["omega"][t]); k = int(sched["k"][t])
        tau, sig = eta / om, eta * om
        xh = torch.minimum(torch.maximum(x - tau * (ct - A.T @ y), lvt), uvt)
        w = A @ (2 * xh - x) - y / sig
        yh = sig * (torch.minimum(torch.maximum(w, lct), uct) - w)
        if sched["restart"][t]:
            xa, ya, x, y = xh, yh, xh, yh
        else:
            a = (k + 1) / (k + 2)
            x = a * ((1 + gamma) * xh - gamma * x) + (1 - a) * xa
            y = a * ((1 + gamma) * yh - gamma * y) + (1 - a) * ya
    return dc * xh, dr * yh


def test_vjp_matches_torch_autograd():
    lp = _lp_small(3)
    p = Params(eval_freq=16)
    K = 200
    fw = unrolled_forward(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p, K)
    sched, eta = fw["schedule"], fw["eta"]
    rng = np.random.default_rng(0)
    gx = rng.standard_normal(lp.n); gy = rng.standard_normal(lp.m)
    g = unrolled_vjp(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p, K, sched, eta, gx, gy)
    At, dr, dc, *_ = scale_problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p.ruiz_iters, p.pock_chambolle)
    T = lambda v: torch.tensor(v, dtype=torch.float64, requires_grad=True)
    c, lc, uc, lv, uv = T(lp.c), T(lp.lc), T(lp.uc), T(lp.lv), T(lp.uv)
    dr_t, dc_t = torch.tensor(dr), torch.tensor(dc)
    A = torch.tensor(At.toarray())
    x, y = _torch_frozen_map(A, dc_t * c, dr_t * lc, dr_t * uc, lv / dc_t, uv / dc_t, dr_t, dc_t,
                             eta, sched, K, 1.0)
    loss = (torch.tensor(gx) * x).sum() + (torch.tensor(gy) * y).sum()
    tg = [torch.nan_to_num(t, nan=0.0).numpy() for t in torch.autograd.grad(loss, [c, lc, uc, lv, uv])]
    # torch splits a tie of min/max evenly, so on an equality row (lc = uc) only
    # the sum -- the derivative with respect to the right-hand side b -- is unique
    eq = lp.lc == lp.uc
    for gg in (g, None):
        if gg is None:
            gg = dict(zip(("c", "lc", "uc", "lv", "uv"), tg))
        gg["lc"] = gg["lc"].copy(); gg["uc"] = gg["uc"].copy()
        gg["lc"][eq] += gg["uc"][eq]; gg["uc"][eq] = 0.0
        if gg is not g:
            tg = [gg[key] for key in ("c", "lc", "uc", "lv", "uv")]
    for key, t in zip(("c", "lc", "uc", "lv", "uv"), tg):
        fin = np.isfinite(getattr(lp, key))
        np.testing.assert_allclose(g[key][fin], t[fin], rtol=1e-9, atol=1e-11 * (1 + np.abs(t).max()))
        assert np.all(g[key][~fin] == 0.0)
    np.testing.assert_allclose(x.detach().numpy(), fw["x"], rtol=1e-12, atol=1e-13)


def test_envelope_theorem_at_convergence():
    """Warm-started at the 1e-8 solution, d(c^T x)/dc -> x* and the gradient
    with respect to an equality row's right-hand side -> y* (unique optimum)."""
    lp = lpgen.config("c1", seed=2, scale=0.1)
    p = Params(tol=1e-10)
    sol = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p)
    assert sol.status == oracle.pdhg.OPTIMAL
    K = 400
    fw = unrolled_forward(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p, K, x0=sol.x, y0=sol.y)
    g = unrolled_vjp(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p, K, fw["schedule"], fw["eta"],
                     lp.c, np.zeros(lp.m), x0=sol.x, y0=sol.y)
    gc = g["c"] + fw["x"]                       # direct term of c^T x
    assert np.abs(gc - sol.x).max() <= 1e-3 * (1 + np.abs(sol.x).max())
    eq = lp.lc == lp.uc
    gb = g["lc"][eq] + g["uc"][eq]
    assert np.abs(gb - sol.y[eq]).max() <= 1e-3 * (1 + np.abs(sol.y).max())


# ------------------------------------------------------------------ mixed precision / IR
def test_shifted_step_is_exact_reformulation():
    """In FP64 the shifted-coordinate step maps back to the plain eq. (pdhg) step."""
    lp = lpgen.gen_mixed(40, 60, rowlen=4, seed=2)
    At, dr, dc, ct, lct, uct, lvt, uvt = scale_problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, 10, 1)
    AtT = At.T.tocsr()
    rng = np.random.default_rng(0)
    eta, omega = 0.5, 1.7
    tau, sigma = eta / omega, eta * omega
    for P, D in ((1.0, 1.0), (2.0 ** 10, 2.0 ** 3), (2.0 ** 4, 2.0 ** 20)):
        xb = rng.standard_normal(lp.n); yb = rng.standard_normal(lp.m)
        x = rng.standard_normal(lp.n); y = rng.standard_normal(lp.m)
        xh, yh, _ = pdhg_operator(At, AtT, ct, lvt, uvt, lct, uct, tau, sigma, x, y)
        Ax = At @ xb
        cd = dict(c=D * (ct - AtT @ yb), lv=P * (lvt - xb), uv=P * (uvt - xb), lc=P * (lct - Ax),
                  uc=P * (uct - Ax), b=D * yb)
        xh2, yh2 = shifted_step(At, AtT, cd, tau * P / D, sigma * D / P, P * (x - xb), D * (y - yb))
        np.testing.assert_allclose(xb + xh2 / P, xh, rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(yb + yh2 / D, yh, rtol=1e-11, atol=1e-11)


def test_mixed_reaches_fp64_tolerance_and_matches_highs():
    lp = lpgen.config("c1", seed=1)
    fun, xs, ys = highs(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv)
    res = solve_mixed(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, Params(tol=1e-8))
    assert res["status"] == oracle.pdhg.OPTIMAL
    k = oracle.kkt(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, res["x"], res["y"])
    assert k["rel_kkt"] <= 1e-8
    assert abs(k["pobj"] - fun) <= 1e-7 * (1 + abs(fun))
