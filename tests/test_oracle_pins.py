"""Pins of the FP64 CPU oracle against things other than itself.

Each test names what fixes the expected value: vertex enumeration, HiGHS,
closed forms, a hand-computed fixture, or an invariant of the method
(fixed point of eq. (pdhg), firm nonexpansiveness in the P-norm of Sec. 2.2,
the Halpern rate, the PID special case that reduces to cuPDLP's rule).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
import oracle
from oracle.brute import brute_force
from oracle.kkt import kkt
from oracle.pdhg import Params, pdhg_operator, pid_update, power_norm, rescale, restart_decision
from tests import _pins
from tests._highs import highs

HERE = os.path.dirname(os.path.abspath(__file__))


def _solve(lp, **kw):
    return oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, Params(**kw))


def _invariants(lp, x, y, tol):
    """Optimality invariants at a returned point (original space)."""
    k = kkt(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, x, y)
    Ax = lp.A @ x
    scale = 1.0 + np.abs(np.concatenate([lp.lc[np.isfinite(lp.lc)], lp.uc[np.isfinite(lp.uc)]])).max()
    assert np.all(x >= lp.lv - 1e-12) and np.all(x <= lp.uv + 1e-12)          # X
    assert np.all(Ax >= lp.lc - tol * scale) and np.all(Ax <= lp.uc + tol * scale)  # S
    # y in the sign set Y
    assert np.all(y[~np.isfinite(lp.lc)] <= 1e-12) and np.all(y[~np.isfinite(lp.uc)] >= -1e-12)
    # complementary slackness: a nonzero multiplier sits on an active bound
    act_lo = np.abs(Ax - lp.lc) <= 1e-5 * scale
    act_hi = np.abs(Ax - lp.uc) <= 1e-5 * scale
    big = np.abs(y) > 1e-5 * (1 + np.abs(y).max())
    assert np.all(~big | act_lo | act_hi)
    return k


# ------------------------------------------------------------------ whole solve
@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_solve_matches_vertex_enumeration(seed):
    lp = lpgen.gen_mixed(5, 5, rowlen=2, seed=seed, box_only=True)
    best, _ = brute_force(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv)
    res = _solve(lp, tol=1e-10, eval_freq=16)
    assert res.status == oracle.pdhg.OPTIMAL
    assert abs(res.info["pobj"] - best) <= 1e-7 * (1 + abs(best))
    _invariants(lp, res.x, res.y, 1e-8)


def test_solve_matches_highs_c1():
    lp = lpgen.config("c1", seed=1)
    fun, xs, ys = highs(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv)
    res = _solve(lp, tol=1e-8)
    assert res.status == oracle.pdhg.OPTIMAL and res.info["rel_kkt"] <= 1e-8
    assert abs(res.info["pobj"] - fun) <= 1e-7 * (1 + abs(fun))
    _invariants(lp, res.x, res.y, 1e-7)


@pytest.mark.parametrize("seed", [1, 2])
def test_solve_matches_highs_all_bound_types(seed):
    lp = lpgen.gen_mixed(60, 80, rowlen=4, seed=seed)
    fun, xs, ys = highs(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv)
    res = _solve(lp, tol=1e-9)
    assert res.status == oracle.pdhg.OPTIMAL
    assert abs(res.info["pobj"] - fun) <= 1e-7 * (1 + abs(fun))
    _invariants(lp, res.x, res.y, 1e-7)


def test_kkt_at_highs_optimum():
    lp = lpgen.gen_mixed(40, 50, rowlen=3, seed=7)
    fun, xs, ys = highs(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv)
    k = kkt(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, xs, ys)
    assert k["rel_kkt"] <= 1e-9


# ------------------------------------------------------------------ closed forms
def test_box_lp_closed_form():
    """A = 0: the LP separates; x_j = lv_j when c_j > 0, uv_j when c_j < 0."""
    rng = np.random.default_rng(3)
    m, n = 4, 30
    A = sp.csr_matrix((m, n))
    c = rng.standard_normal(n)
    lv = -rng.random(n); uv = rng.random(n)
    lc = -np.ones(m); uc = np.ones(m)
    res = oracle.solve(A, c, lc, uc, lv, uv, Params(tol=1e-12, eval_freq=4))
    assert res.status == oracle.pdhg.OPTIMAL
    assert res.eta == 1.0                       # ||A|| = 0 gives eta = 1
    np.testing.assert_allclose(res.x, np.where(c > 0, lv, uv), atol=1e-10)


def test_knapsack_greedy():
    """One row w^T x <= W, 0 <= x <= 1, maximise v^T x: fractional greedy."""
    rng = np.random.default_rng(5)
    n = 25
    w = rng.uniform(0.5, 2.0, n); v = rng.uniform(0.5, 2.0, n); W = 7.3
    order = np.argsort(-v / w)
    x = np.zeros(n); cap = W
    for j in order:
        take = min(1.0, cap / w[j]); x[j] = take; cap -= take * w[j]
        if cap <= 0:
            break
    A = sp.csr_matrix(w[None, :])
    res = oracle.solve(A, -v, np.array([-np.inf]), np.array([W]), np.zeros(n), np.ones(n),
                       Params(tol=1e-11, eval_freq=16))
    assert res.status == oracle.pdhg.OPTIMAL
    assert abs(res.info["pobj"] - (-v @ x)) <= 1e-8 * (1 + abs(v @ x))
    np.testing.assert_allclose(res.x, x, atol=1e-6)


def test_diagonal_lp_separable():
    """A = diag(a): each x_j lives in an interval; it sits at the end c_j prefers."""
    rng = np.random.default_rng(11)
    n = 20
    a = rng.uniform(0.5, 2.0, n) * np.where(rng.random(n) < 0.5, -1, 1)
    A = sp.csr_matrix(sp.diags(a))
    lc = rng.uniform(-2, -0.5, n); uc = rng.uniform(0.5, 2, n)
    lv = rng.uniform(-3, -1, n); uv = rng.uniform(1, 3, n)
    c = rng.standard_normal(n)
    lo = np.maximum(lv, np.minimum(lc / a, uc / a))
    hi = np.minimum(uv, np.maximum(lc / a, uc / a))
    res = oracle.solve(A, c, lc, uc, lv, uv, Params(tol=1e-12, eval_freq=8))
    assert res.status == oracle.pdhg.OPTIMAL
    np.testing.assert_allclose(res.x, np.where(c > 0, lo, hi), atol=1e-9)


def test_kkt_hand_example():
    """tests/golden/kkt_2x2.json: hand-computed KKT parts, including a case with
    objectives of the same sign (fixes the gap's denominator)."""
    _pins.pin_kkt_golden(oracle)


# ------------------------------------------------------------------ invariants of the operator
def _identity_scaled(lp):
    return lp.A.tocsr(), lp.A.T.tocsr()


def test_highs_optimum_is_fixed_point():
    """An optimum z* is a fixed point of eq. (pdhg) for any admissible eta, omega
    (this fixes the sign of the bilinear term and of the projection)."""
    lp = lpgen.gen_mixed(40, 50, rowlen=3, seed=9)
    fun, xs, ys = highs(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv)
    A, AT = _identity_scaled(lp)
    nrm = np.linalg.norm(A.toarray(), 2)
    for omega in (0.3, 1.0, 4.0):
        eta = 0.9 / nrm
        xh, yh, _ = pdhg_operator(A, AT, lp.c, lp.lv, lp.uv, lp.lc, lp.uc, eta / omega, eta * omega, xs, ys)
        assert np.abs(xh - xs).max() <= 1e-9 * (1 + np.abs(xs).max())
        assert np.abs(yh - ys).max() <= 1e-9 * (1 + np.abs(ys).max())


def _pnorm_inner(A, eta, omega, a, b, n):
    ax, ay = a[:n], a[n:]
    bx, by = b[:n], b[n:]
    return (omega / eta) * ax @ bx + ay @ (A @ bx) + by @ (A @ ax) + (ay @ by) / (eta * omega)


def test_firm_nonexpansive_in_P_norm():
    lp = lpgen.gen_mixed(30, 40, rowlen=3, seed=4)
    A, AT = _identity_scaled(lp)
    n = lp.n
    eta = 0.998 / np.linalg.norm(A.toarray(), 2)
    rng = np.random.default_rng(0)
    for trial in range(100):
        omega = math.exp(rng.uniform(-2, 2))
        z1 = rng.standard_normal(n + lp.m) * 3
        z2 = rng.standard_normal(n + lp.m) * 3
        T = lambda z: np.concatenate(pdhg_operator(A, AT, lp.c, lp.lv, lp.uv, lp.lc, lp.uc,
                                                   eta / omega, eta * omega, z[:n], z[n:])[:2])
        d = T(z1) - T(z2)
        lhs = _pnorm_inner(A, eta, omega, d, d, n)
        rhs = _pnorm_inner(A, eta, omega, d, z1 - z2, n)
        assert lhs <= rhs + 1e-9 * abs(rhs)


def test_halpern_rate_without_restarts():
    """Reflected Halpern with restarts off: ||z^k - T z^k||_P <= 2||z^0 - z*||_P / ((1+g)(k+1))."""
    lp = lpgen.gen_mixed(30, 40, rowlen=3, seed=2, box_only=True)
    fun, xs, ys = highs(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv)
    A = lp.A
    eta = 0.998 / np.linalg.norm(A.toarray(), 2)
    for gamma in (0.0, 0.5, 1.0):
        p = Params(tol=1e-300, max_iter=400, eval_freq=1, ruiz_iters=0, pock_chambolle=0,
                   eta_override=eta, gamma=gamma, beta_sufficient=-1.0, beta_necessary=-1.0,
                   beta_artificial=1e18)
        res = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p)
        assert res.restarts == 0
        zs = np.concatenate([xs, ys])
        dist = math.sqrt(_pnorm_inner(A, eta, 1.0, zs, zs, lp.n))   # z^0 = 0
        for e in res.log:
            kk = e["t"] - 1                        # r is measured at z^{k} before the update
            assert e["r"] <= 2 * dist / ((1 + gamma) * (kk + 1)) * (1 + 1e-9)


# ------------------------------------------------------------------ controller pieces
def test_restart_decision_sequences():
    p = Params()
    # sufficient decay
    assert restart_decision(0.19, 1.0, math.inf, 5, 100, p)
    assert not restart_decision(0.21, 1.0, math.inf, 5, 100, p)
    # necessary decay + no local progress
    assert restart_decision(0.79, 1.0, 0.7, 5, 100, p)
    assert not restart_decision(0.79, 1.0, 0.8, 5, 100, p)
    assert not restart_decision(0.81, 1.0, 0.5, 5, 100, p)
    # artificial: k >= 0.36 T
    assert restart_decision(0.9, 1.0, 0.5, 36, 100, p)
    assert not restart_decision(0.9, 1.0, 0.5, 35, 100, p)


def test_pid_proportional_only_is_cupdlp_rule():
    """(Kp, Ki, Kd) = (1, 0, 0) gives omega = ||dy|| / ||dx|| exactly (cuPDLP's
    unsmoothed rule that the PID controller generalises)."""
    p = Params(kp=1.0, ki=0.0, kd=0.0)
    rng = np.random.default_rng(1)
    for _ in range(20):
        om, dx, dy = math.exp(rng.uniform(-3, 3)), rng.uniform(0.1, 10), rng.uniform(0.1, 10)
        assert pid_update(om, dx, dy, {}, p) == pytest.approx(dy / dx, rel=1e-13)


def test_pid_integral_and_derivative_terms():
    p = Params(kp=0.5, ki=0.25, kd=0.125)
    st = {}
    om = 2.0
    errs = []
    for dx, dy in ((1.0, 3.0), (2.0, 1.0), (1.5, 1.5)):
        e = math.log(om * dx / dy)
        errs.append(e)
        de = 0.0 if len(errs) == 1 else errs[-1] - errs[-2]
        expect = math.exp(math.log(om) - (0.5 * e + 0.25 * sum(errs) + 0.125 * de))
        om = pid_update(om, dx, dy, st, p)
        assert om == pytest.approx(expect, rel=1e-14)
    assert pid_update(om, 1e-12, 1.0, st, p) == om       # skipped below pid_min_norm


# ------------------------------------------------------------------ setup steps
def test_power_norm_matches_dense_svd():
    lp = lpgen.gen_mixed(40, 60, rowlen=4, seed=3)
    est, it = power_norm(lp.A, 5000, 1e-10)
    true = np.linalg.norm(lp.A.toarray(), 2)
    assert abs(est - true) <= 1e-4 * true
    assert est <= true * (1 + 1e-12)       # a Rayleigh-type estimate never overshoots


def test_power_norm_matches_svds_medium():
    from scipy.sparse.linalg import svds
    lp = lpgen.config("c2", seed=2, scale=0.02)
    est, _ = power_norm(lp.A, 5000, 1e-8)
    true = svds(lp.A, k=1, return_singular_vectors=False)[0]
    assert abs(est - true) <= 2e-3 * true


def test_ruiz_equilibrates():
    lp = lpgen.config("c1", seed=3)
    At, dr, dc = rescale(lp.A, ruiz_iters=20, pock_chambolle=0)
    absA = abs(At)
    rmax = absA.max(axis=1).toarray().ravel()
    cmax = absA.max(axis=0).toarray().ravel()
    assert np.all(np.abs(rmax[rmax > 0] - 1) < 1e-3)
    assert np.all(np.abs(cmax[cmax > 0] - 1) < 1e-3)
    # the scaling is D_r A D_c with the returned diagonals
    np.testing.assert_allclose((sp.diags(dr) @ lp.A @ sp.diags(dc)).toarray(), At.toarray(), rtol=1e-13)


def test_scaling_invariance_of_solution():
    lp = lpgen.gen_mixed(50, 70, rowlen=3, seed=5)
    a = _solve(lp, tol=1e-9)
    b = _solve(lp, tol=1e-9, ruiz_iters=0, pock_chambolle=0)
    assert a.status == b.status == oracle.pdhg.OPTIMAL
    assert abs(a.info["pobj"] - b.info["pobj"]) <= 1e-7 * (1 + abs(a.info["pobj"]))


# ------------------------------------------------------------------ status codes and validation
def test_iteration_and_time_limits():
    lp = lpgen.config("c1", seed=1)
    r = _solve(lp, max_iter=1)
    assert r.status == oracle.pdhg.ITER_LIMIT and r.iters == 1
    r = _solve(lp, time_limit_s=0.0)
    assert r.status == oracle.pdhg.TIME_LIMIT and r.iters == 64


@pytest.mark.parametrize("bad", ["nan_c", "l_gt_u", "col_range", "unsorted", "plus_inf_lower", "minus_inf_upper"])
def test_validation_rejects(bad):
    lp = lpgen.gen_mixed(6, 8, rowlen=3, seed=1)
    A, c, lc, uc, lv, uv = lp.A.copy(), lp.c.copy(), lp.lc.copy(), lp.uc.copy(), lp.lv.copy(), lp.uv.copy()
    if bad == "nan_c":
        c[2] = np.nan
    elif bad == "l_gt_u":
        lv[0], uv[0] = 1.0, 0.0
    elif bad == "col_range":
        A.indices[0] = 8
    elif bad == "unsorted":
        A.indices[0], A.indices[1] = A.indices[1], A.indices[0]
    elif bad == "plus_inf_lower":
        lc[1] = np.inf
    elif bad == "minus_inf_upper":
        uv[1] = -np.inf
    with pytest.raises(ValueError):
        oracle.solve(A, c, lc, uc, lv, uv)


# ------------------------------------------------------------------ definitions and hand arithmetic (tests/_pins.py)
@pytest.mark.parametrize("pin", [p for p in _pins.ALL_PINS if p is not _pins.pin_kkt_golden],
                         ids=lambda p: p.__name__)
def test_pin(pin):
    """r(z) against the dense P of Sec. 2.2; the reflected Halpern closed form;
    hand-computed restart schedules and epoch bookkeeping; hand-computed
    Ruiz / Pock-Chambolle factors."""
    pin(oracle)


def test_flipped_P_breaks_firm_nonexpansiveness():
    """The firm-nonexpansiveness pin can tell the sign of P's off-diagonal
    blocks: with -A in place of A it fails on some random pair."""
    lp = lpgen.gen_mixed(30, 40, rowlen=3, seed=4)
    A, AT = _identity_scaled(lp)
    n = lp.n
    eta = 0.998 / np.linalg.norm(A.toarray(), 2)
    rng = np.random.default_rng(0)
    violated = 0
    for trial in range(100):
        omega = math.exp(rng.uniform(-2, 2))
        z1 = rng.standard_normal(n + lp.m) * 3
        z2 = rng.standard_normal(n + lp.m) * 3
        T = lambda z: np.concatenate(pdhg_operator(A, AT, lp.c, lp.lv, lp.uv, lp.lc, lp.uc,
                                                   eta / omega, eta * omega, z[:n], z[n:])[:2])
        d = T(z1) - T(z2)
        lhs = _pnorm_inner(-A, eta, omega, d, d, n)
        rhs = _pnorm_inner(-A, eta, omega, d, z1 - z2, n)
        violated += lhs > rhs + 1e-9 * abs(rhs)
    assert violated > 0
