"""GPU reverse mode (hand-written adjoint behind torch.autograd.Function)
against the oracle's reverse mode, finite differences of the GPU's own frozen
map, and checkpoint invariance.  Bars: outputs of the unrolled forward within
1e-10 relative of the oracle; gradients within 1e-9 relative of the oracle's;
directional derivatives within 1e-6 relative of kink-free central differences
(the target the extension states)."""
import numpy as np
import pytest
import torch

import lpgen
from oracle.adjoint import unrolled_forward, unrolled_vjp
from oracle.pdhg import Params
from tests._gpu import announce, oracle_eta, problem, rel
from tests.test_oracle_adjoint import kink_free_central_difference

pytestmark = pytest.mark.gpu

KEYS = ("c", "lc", "uc", "lv", "uv")


def _grads(prob, lp, K, ckpt, gx, gy, **params):
    from paper_2507_14051_amd.autograd import PDHGUnrolled
    ts = [torch.tensor(getattr(lp, k), dtype=torch.float64, device="cuda:0", requires_grad=True) for k in KEYS]
    x, y = PDHGUnrolled.apply(*ts, prob, K, ckpt, params)
    loss = (x * torch.tensor(gx, device="cuda:0")).sum() + (y * torch.tensor(gy, device="cuda:0")).sum()
    loss.backward()
    return x.detach().cpu().numpy(), y.detach().cpu().numpy(), {k: t.grad.cpu().numpy() for k, t in zip(KEYS, ts)}


def _eq_sum(g, lp):
    """On an equality row only lc + uc is the derivative w.r.t. b; compare that."""
    g = dict(g)
    eq = lp.lc == lp.uc
    g["lc"] = g["lc"].copy(); g["uc"] = g["uc"].copy()
    g["lc"][eq] += g["uc"][eq]; g["uc"][eq] = 0.0
    return g


@pytest.mark.parametrize("seed", [1, 2])
def test_gradients_match_oracle(seed):
    lp = lpgen.config("c5", seed=seed, scale=0.01)      # m=500, n=1000, 8 nnz/row
    K, ckpt = 300, 40
    announce(f"adjoint vs oracle seed={seed} m={lp.m} n={lp.n} K={K} ckpt={ckpt}")
    eta = oracle_eta(lp)
    prob = problem(lp, eta=eta)
    rng = np.random.default_rng(seed)
    gx = rng.standard_normal(lp.n); gy = rng.standard_normal(lp.m)
    x, y, g = _grads(prob, lp, K, ckpt, gx, gy, eval_freq=16)
    p = Params(eval_freq=16)
    fw = unrolled_forward(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p, K, eta=eta)
    assert fw["schedule"]["restart"].sum() >= 2
    assert rel(x, fw["x"]) <= 1e-10 and rel(y, fw["y"]) <= 1e-10
    go = unrolled_vjp(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p, K, fw["schedule"], eta, gx, gy)
    for key in KEYS:
        assert rel(g[key], go[key]) <= 1e-9, (key, rel(g[key], go[key]))
    prob.close()


def test_gradients_long_rows_match_oracle():
    """Rows longer than 64 nonzeros (some beyond the LDS stage) take the
    block-wide reduction path in the reverse kernels too."""
    lp = lpgen.gen(1500, 12000, zipf_alpha=1.3, cap=6000, eq_frac=0.3, free_frac=0.2, values="normal", seed=9)
    assert (np.diff(lp.A.indptr) > 4096).sum() > 10
    K, ckpt = 120, 25
    announce(f"adjoint long rows nnz={lp.nnz} K={K}")
    eta = oracle_eta(lp)
    prob = problem(lp, eta=eta)
    rng = np.random.default_rng(5)
    gx = rng.standard_normal(lp.n); gy = rng.standard_normal(lp.m)
    x, y, g = _grads(prob, lp, K, ckpt, gx, gy, eval_freq=16)
    p = Params(eval_freq=16)
    fw = unrolled_forward(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p, K, eta=eta)
    assert rel(x, fw["x"]) <= 1e-10 and rel(y, fw["y"]) <= 1e-10
    go = unrolled_vjp(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, p, K, fw["schedule"], eta, gx, gy)
    for key in KEYS:
        assert rel(g[key], go[key]) <= 1e-9, (key, rel(g[key], go[key]))
    prob.close()


def test_checkpoint_interval_does_not_change_gradients():
    lp = lpgen.config("c5", seed=3, scale=0.01)
    K = 120
    announce("adjoint checkpoint invariance")
    prob = problem(lp)
    rng = np.random.default_rng(0)
    gx = rng.standard_normal(lp.n); gy = rng.standard_normal(lp.m)
    base = _grads(prob, lp, K, K, gx, gy, eval_freq=16)[2]
    for ck in (1, 7, 50):
        g = _grads(prob, lp, K, ck, gx, gy, eval_freq=16)[2]
        for key in KEYS:
            assert np.array_equal(g[key], base[key]), (ck, key)
    prob.close()


def _fd_check(lp, K, ckpt, seed, h0=1e-6):
    from paper_2507_14051_amd import hlp
    prob = problem(lp)
    rng = np.random.default_rng(seed)
    xt = lpgen.x_target(lp.n, seed)
    # loss = ||x - x_target||^2 + c^T x (the differentiation workload's loss)
    from paper_2507_14051_amd.autograd import PDHGUnrolled
    ts = [torch.tensor(getattr(lp, k), dtype=torch.float64, device="cuda:0", requires_grad=True) for k in KEYS]
    x, y = PDHGUnrolled.apply(*ts, prob, K, ckpt, None)
    loss = ((x - torch.tensor(xt, device="cuda:0")) ** 2).sum() + (ts[0] * x).sum()
    loss.backward()
    g = {k: t.grad.cpu().numpy() for k, t in zip(KEYS, ts)}
    d = lpgen.directions(lp, seed)
    # replay the frozen map on the GPU along the direction
    tape = torch.empty(hlp.hlp_tape_bytes(prob.handle, K, ckpt), dtype=torch.uint8, device="cuda:0")
    xo = torch.empty(lp.n, dtype=torch.float64, device="cuda:0")
    yo = torch.empty(lp.m, dtype=torch.float64, device="cuda:0")
    prob.update_vectors(lp.c, lp.lc, lp.uc, lp.lv, lp.uv)
    hlp.hlp_unrolled_forward(prob.handle, prob.params_for(), K, ckpt, 0, None, None, xo, yo, tape)

    def F(s):
        v = {k: getattr(lp, k) + s * np.where(np.isfinite(getattr(lp, k)), d[k], 0.0) for k in KEYS}
        prob.update_vectors(*(v[k] for k in KEYS))
        hlp.hlp_unrolled_forward(prob.handle, prob.params_for(), K, ckpt, 1, None, None, xo, yo, tape)
        xs = xo.cpu().numpy()
        return float(((xs - xt) ** 2).sum() + v["c"] @ xs)

    fd = kink_free_central_difference(F, h0)
    an = sum(float(g[k] @ np.where(np.isfinite(d[k]), d[k], 0.0)) for k in KEYS)
    prob.close()
    return fd, an


def test_directional_derivative_matches_finite_differences_small():
    lp = lpgen.config("c5", seed=4, scale=0.02)
    announce("adjoint FD small")
    fd, an = _fd_check(lp, 400, 50, 4)
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_differentiation_workload_full_size():
    """m=50,000, n=100,000, 8 nnz/row, K=2,000 unrolled iterations,
    checkpoint every 100; loss ||x - x_target||^2 + c^T x."""
    lp = lpgen.config("c5", seed=1)
    announce(f"adjoint FD full c5 m={lp.m} n={lp.n} nnz={lp.nnz} K=2000 ckpt=100")
    fd, an = _fd_check(lp, 2000, 100, 1)
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_envelope_theorem_at_convergence():
    """Warm-started at the oracle's 1e-10 solution, the GPU derivative of
    c^T x_K with respect to c tends to x*, and that with respect to an equality
    row's right-hand side to y* (the envelope theorem for the optimal value;
    unique optimum).  The bar is the oracle's own envelope test's."""
    from paper_2507_14051_amd.autograd import PDHGUnrolled
    import oracle
    lp = lpgen.config("c1", seed=2, scale=0.1)
    announce(f"adjoint envelope theorem m={lp.m} n={lp.n}")
    sol = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, Params(tol=1e-10))
    assert sol.status == oracle.pdhg.OPTIMAL
    prob = problem(lp, eta=oracle_eta(lp))
    dev = "cuda:0"
    ts = [torch.tensor(getattr(lp, k), dtype=torch.float64, device=dev, requires_grad=True) for k in KEYS]
    x0 = torch.tensor(sol.x, dtype=torch.float64, device=dev)
    y0 = torch.tensor(sol.y, dtype=torch.float64, device=dev)
    x, y = PDHGUnrolled.apply(*ts, prob, 400, 50, None, x0, y0)
    (ts[0] * x).sum().backward()            # c^T x_K: direct term plus the reverse pass
    g = _eq_sum({k: t.grad.cpu().numpy() for k, t in zip(KEYS, ts)}, lp)
    prob.close()
    assert np.abs(g["c"] - sol.x).max() <= 1e-3 * (1 + np.abs(sol.x).max())
    eq = lp.lc == lp.uc
    assert eq.sum() > 0
    assert np.abs(g["lc"][eq] - sol.y[eq]).max() <= 1e-3 * (1 + np.abs(sol.y).max())
    print(f"envelope: |dc - x*| {np.abs(g['c'] - sol.x).max():.1e}, |db - y*| {np.abs(g['lc'][eq] - sol.y[eq]).max():.1e}")
