"""Pins of the oracle's controller, residual and scaling, written as functions
of the oracle package so that the same checks can run on deliberately broken
copies of it (tests/test_oracle_mutants.py) as well as on the oracle itself
(tests/test_oracle_pins.py).

Every expected value here comes from the paper's definitions or from hand
arithmetic, never from the oracle:

  * r(z) = ||z - PDHG(z)||_P with P = [[omega/eta I, A^T], [A, 1/(eta omega) I]]
    built densely as the paper defines it (Sec. 2.2);
  * the reflected Halpern update in closed form for the first iterations
    (Sec. 3, "Halpern scheme" and "Reflection");
  * the restart bookkeeping (Sec. 3, "Adaptive restart"): hand-computed
    artificial-restart schedules, r(z^{n,0}) taken at an epoch's first
    iteration only, r(z^{n,k-1}) the previous check of the same epoch;
  * hand-computed scaling factors on a 3x3 matrix (tests/golden/scaling_3x3.json)
    and KKT parts on a 2x2 LP (tests/golden/kkt_2x2.json).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import scipy.sparse as sp

import lpgen

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def dense_P(A, eta, omega):
    """The matrix of the P-norm exactly as Sec. 2.2 defines it."""
    A = np.asarray(A.toarray() if hasattr(A, "toarray") else A, dtype=np.float64)
    m, n = A.shape
    P = np.zeros((n + m, n + m))
    P[:n, :n] = (omega / eta) * np.eye(n)
    P[:n, n:] = A.T
    P[n:, :n] = A
    P[n:, n:] = np.eye(m) / (eta * omega)
    return P


def p_norm(A, eta, omega, dz):
    return math.sqrt(max(float(dz @ dense_P(A, eta, omega) @ dz), 0.0))


def _tiny(seed=4):
    return lpgen.gen_mixed(12, 16, rowlen=3, seed=seed)


def _no_restarts(**kw):
    return dict(beta_sufficient=-1.0, beta_necessary=-1.0, beta_artificial=1e18, **kw)


def _unscaled(orc, lp, **kw):
    """A solve with the preconditioner off, so the scaled space is the
    original one, and eta fixed below 1/||A||_2."""
    eta = 0.95 / np.linalg.norm(lp.A.toarray(), 2)
    p = orc.Params(ruiz_iters=0, pock_chambolle=0, eta_override=eta, **kw)
    return eta, p


# ------------------------------------------------------------------ r(z)
def pin_residual_is_p_norm(orc):
    """fixed_point_residual(A, dx, dy, eta, omega) = sqrt(dz^T P dz) on random
    dz for several (eta, omega)."""
    lp = _tiny()
    A = lp.A
    rng = np.random.default_rng(21)
    for eta, omega in ((0.3, 1.0), (0.05, 7.0), (1.3, 0.02), (0.7, 0.5)):
        for _ in range(5):
            dx = rng.standard_normal(lp.n)
            dy = rng.standard_normal(lp.m)
            got = orc.pdhg.fixed_point_residual(A, dx, dy, eta, omega)
            want = p_norm(A, eta, omega, np.concatenate([dx, dy]))
            assert abs(got - want) <= 1e-12 * max(want, 1e-300), (eta, omega, got, want)


def pin_logged_residual_is_definition(orc):
    """Each check's r in a solve is ||z - PDHG(z)||_P of that iteration's z and
    PDHG(z) (taken from the trace), with the primal weight then in force; after
    a restart z is the PDHG output of the restart iteration (the new anchor)."""
    lp = _tiny()
    T = 60
    eta, p = _unscaled(orc, lp, tol=1e-300, max_iter=T, eval_freq=1, trace_iters=T)
    res = orc.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p)
    assert res.restarts >= 2, "the case must cross restarts"
    n = lp.n
    tr = res.trace
    log = res.log
    assert [e["t"] for e in log] == list(range(1, T + 1))
    for i, e in enumerate(log):
        t = e["t"]
        if t == 1:
            z = np.zeros(n + lp.m)
        elif log[i - 1]["restart"]:
            z = np.concatenate([tr["xh"][t - 2], tr["yh"][t - 2]])
        else:
            z = np.concatenate([tr["x"][t - 2], tr["y"][t - 2]])
        zh = np.concatenate([tr["xh"][t - 1], tr["yh"][t - 1]])
        want = p_norm(lp.A, eta, e["omega"], z - zh)
        assert abs(e["r"] - want) <= 1e-10 * max(want, 1e-300), (t, e["r"], want)


# ------------------------------------------------------------------ Halpern + reflection
def pin_reflected_halpern_closed_form(orc):
    """With restarts off and anchor z^0 (the start point):
    z^1 = 1/2((1+g)T z^0 - g z^0) + 1/2 z^0,  z^2 = 2/3((1+g)T z^1 - g z^1) + 1/3 z^0,
    z^3 = 3/4((1+g)T z^2 - g z^2) + 1/4 z^0, with T the PDHG step at the initial
    primal weight."""
    lp = _tiny(seed=6)
    rng = np.random.default_rng(8)
    x0 = rng.uniform(-1, 1, lp.n)
    y0 = rng.uniform(-1, 1, lp.m)
    A = lp.A.tocsr()
    AT = lp.A.T.tocsr()
    for gam in (0.0, 0.5, 1.0):
        omega = 1.7
        eta, p = _unscaled(orc, lp, tol=1e-300, max_iter=3, eval_freq=1000, trace_iters=3,
                           omega0=omega, **_no_restarts(gamma=gam))
        res = orc.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p, x0=x0, y0=y0)
        z0 = np.concatenate([x0, y0])
        z = z0
        for k in range(3):
            xh, yh, _ = orc.pdhg.pdhg_operator(A, AT, lp.c, lp.lv, lp.uv, lp.lc, lp.uc, eta / omega, eta * omega,
                                               z[:lp.n], z[lp.n:])
            Tz = np.concatenate([xh, yh])
            want = (k + 1) / (k + 2) * ((1 + gam) * Tz - gam * z) + z0 / (k + 2)
            got = np.concatenate([res.trace["x"][k], res.trace["y"][k]])
            np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-14, err_msg=f"gamma={gam} k={k}")
            z = want


# ------------------------------------------------------------------ restart bookkeeping
# Artificial restarts only, checks every 64 iterations: a restart at check T
# (the total count) when k = T - T_last >= 0.36 T.  By hand: T=64 (k=64),
# 128 (64 >= 46.08), 192 no (64 < 69.12), 256 (128 >= 92.16), 320/384 no,
# 448 (192 >= 161.28), 512..640 no, 704 (256 >= 253.44), 768..1088 no
# (1088: 384 < 391.68), 1152 (448 >= 414.72); max_iter 1200 ends the run.
ARTIFICIAL_SCHEDULE = [64, 128, 256, 448, 704, 1152]


def pin_artificial_restart_schedule(orc):
    lp = _tiny(seed=2)
    _, p = _unscaled(orc, lp, tol=0.0, max_iter=1200, eval_freq=64, beta_sufficient=-1.0,
                     beta_necessary=-1.0, beta_artificial=0.36)
    res = orc.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p)
    got = [e["t"] for e in res.log if e["restart"]]
    assert got == ARTIFICIAL_SCHEDULE, got
    assert res.iters == 1200 and res.restarts == len(ARTIFICIAL_SCHEDULE)


def pin_counts_after_increment(orc):
    """beta_artificial = 1 and a check every iteration: k >= T holds only in
    the first epoch, where k = T, and only when both count the PDHG application
    just made -- so exactly one restart, at T = 1."""
    lp = _tiny(seed=2)
    _, p = _unscaled(orc, lp, tol=0.0, max_iter=40, eval_freq=1, beta_sufficient=-1.0,
                     beta_necessary=-1.0, beta_artificial=1.0)
    res = orc.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p)
    assert [e["t"] for e in res.log if e["restart"]] == [1]


def pin_epoch_bookkeeping(orc):
    """Checks every iteration, default tests: within an epoch k counts from 1,
    r(z^{n,0}) is the residual measured at the epoch's first iteration (the
    same value for every check of the epoch) and the restart decision at each
    check uses the previous check of the same epoch as r(z^{n,k-1})."""
    lp = _tiny(seed=3)
    _, p = _unscaled(orc, lp, tol=1e-300, max_iter=400, eval_freq=1)
    res = orc.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p)
    log = res.log
    assert res.restarts >= 3
    first = None
    prev_r = math.inf
    t_last = 0
    for i, e in enumerate(log):
        if i == 0 or log[i - 1]["restart"]:
            first = e
            prev_r = math.inf
            t_last = e["t"] - 1
        assert e["k"] == e["t"] - t_last
        assert e["r0"] == first["r"], (e["t"], e["r0"], first["r"])
        if e["t"] < p.max_iter:
            expect = orc.pdhg.restart_decision(e["r"], first["r"], prev_r, e["k"], e["t"], p)
            assert e["restart"] == expect, e["t"]
        prev_r = e["r"]


# ------------------------------------------------------------------ scaling and KKT goldens
def _closed(expr):
    return float(eval(expr, {"__builtins__": {}}, {"sqrt": math.sqrt}))


def pin_scaling_golden(orc):
    g = json.load(open(os.path.join(GOLDEN, "scaling_3x3.json")))
    A = sp.csr_matrix(np.array(g["A"]))
    for case in g["cases"]:
        At, dr, dc = orc.pdhg.rescale(A, case["ruiz_iters"], case["pock_chambolle"])
        want_r = np.array([_closed(s) for s in case["d_r"]])
        want_c = np.array([_closed(s) for s in case["d_c"]])
        np.testing.assert_allclose(dr, want_r, rtol=1e-14, err_msg=case["name"])
        np.testing.assert_allclose(dc, want_c, rtol=1e-14, err_msg=case["name"])
        np.testing.assert_allclose(At.toarray(), np.diag(want_r) @ A.toarray() @ np.diag(want_c),
                                   rtol=1e-14, atol=1e-300, err_msg=case["name"])


def pin_kkt_golden(orc):
    g = json.load(open(os.path.join(GOLDEN, "kkt_2x2.json")))
    f = lambda v: np.array([float(t) for t in v])
    A = sp.csr_matrix(np.array(g["A"]))
    for case in g["cases"]:
        x = f(case.get("x", g["x"]))
        y = f(case.get("y", g["y"]))
        k = orc.kkt(A, f(g["c"]), f(g["lc"]), f(g["uc"]), f(case["lv"]), f(case["uv"]), x, y)
        for key in ("pobj", "dobj", "rho_p", "rho_d", "rel_gap", "rel_primal", "rel_dual", "rel_kkt"):
            want = case[key]
            assert abs(k[key] - want) <= 1e-14 * abs(want) + 1e-15, (case["name"], key, k[key], want)
        np.testing.assert_array_equal(k["r"], case["r"])


# ------------------------------------------------------------------ anchor, PID, power iteration
def pin_new_anchor_is_pdhg_output(orc):
    """A restart makes zhat = PDHG(z) the new anchor and the new iterate
    (Sec. 3, the anchor of the next epoch): with a restart forced at T = 1
    (beta_artificial = 1, a check every iteration, the primal weight left
    alone), the second iterate is z^2 = 1/2((1+g) T zhat^1 - g zhat^1) + 1/2 zhat^1."""
    lp = _tiny(seed=5)
    A = lp.A.tocsr()
    AT = lp.A.T.tocsr()
    omega = 1.3
    eta, p = _unscaled(orc, lp, tol=1e-300, max_iter=2, eval_freq=1, trace_iters=2, omega0=omega,
                       beta_sufficient=-1.0, beta_necessary=-1.0, beta_artificial=1.0, kp=0.0, ki=0.0, kd=0.0)
    res = orc.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p)
    assert [e["t"] for e in res.log if e["restart"]] == [1]
    zh1 = np.concatenate([res.trace["xh"][0], res.trace["yh"][0]])
    xh, yh, _ = orc.pdhg.pdhg_operator(A, AT, lp.c, lp.lv, lp.uv, lp.lc, lp.uc, eta / omega, eta * omega,
                                       zh1[:lp.n], zh1[lp.n:])
    g = p.gamma
    want = 0.5 * ((1 + g) * np.concatenate([xh, yh]) - g * zh1) + 0.5 * zh1
    got = np.concatenate([res.trace["x"][1], res.trace["y"][1]])
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-14)


def pin_pid_ratio_rule(orc):
    """Gains (1, 0, 0) give omega = ||dy|| / ||dx|| exactly: with
    e = log(omega ||dx|| / ||dy||) the update moves log omega by -e."""
    p = orc.Params(kp=1.0, ki=0.0, kd=0.0)
    rng = np.random.default_rng(11)
    for _ in range(10):
        om, dx, dy = math.exp(rng.uniform(-3, 3)), rng.uniform(0.1, 10), rng.uniform(0.1, 10)
        got = orc.pdhg.pid_update(om, dx, dy, {}, p)
        assert abs(got - dy / dx) <= 1e-12 * (dy / dx), (om, dx, dy, got)


def pin_pid_sequence(orc):
    """Two hand-computed PID steps with all three gains (0.5, 0.25, 0.125)
    from omega = 2: the integral sums the errors including the current one,
    the derivative term starts at 0."""
    p = orc.Params(kp=0.5, ki=0.25, kd=0.125)
    e1 = math.log(2.0 * 1.0 / 3.0)                       # omega 2, dx 1, dy 3
    om1 = math.exp(math.log(2.0) - (0.5 * e1 + 0.25 * e1))
    e2 = math.log(om1 * 2.0 / 1.0)                       # dx 2, dy 1
    om2 = math.exp(math.log(om1) - (0.5 * e2 + 0.25 * (e1 + e2) + 0.125 * (e2 - e1)))
    st = {}
    om = 2.0
    for (dx, dy), want in (((1.0, 3.0), om1), ((2.0, 1.0), om2)):
        om = orc.pdhg.pid_update(om, dx, dy, st, p)
        assert abs(om - want) <= 1e-13 * want, (om, want)


def pin_power_norm_dense(orc):
    """The power iteration's estimate of ||A||_2 against the largest singular
    value of a dense SVD (Sec. 3, stepsize)."""
    rng = np.random.default_rng(13)
    M = rng.standard_normal((30, 45)) * (rng.random((30, 45)) < 0.3)
    est, _ = orc.pdhg.power_norm(sp.csr_matrix(M), 5000, 1e-12)
    true = float(np.linalg.svd(M, compute_uv=False)[0])
    assert abs(est - true) <= 1e-6 * true, (est, true)


ALL_PINS = [pin_residual_is_p_norm, pin_logged_residual_is_definition, pin_reflected_halpern_closed_form,
            pin_artificial_restart_schedule, pin_counts_after_increment, pin_epoch_bookkeeping,
            pin_scaling_golden, pin_kkt_golden, pin_new_anchor_is_pdhg_output, pin_pid_ratio_rule,
            pin_pid_sequence, pin_power_norm_dense]

