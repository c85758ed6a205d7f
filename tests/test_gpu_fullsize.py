"""Parity at the full sizes of the medium and large workloads.

Reference values come from the FP64 CPU oracle: either run here (the first
100 iterations of the 29.6M-nonzero LP) or stored by tests/golden/make_goldens.py,
a script that calls only the oracle (the medium LP's solve to 1e-8, the
stepsize and scaling of the large LPs, the first iterations of the 692M-nonzero
LP, whose oracle set-up takes about an hour).  Each test runs the GPU in the
launch configuration the benchmark times (column panels and dense rows chosen
by the automatic rule, HIP graphs).

Bars: scaling diagonals 1e-12 relative (norm-wise, and entry-wise at the
stored sampled indices); the trajectory 1e-10 relative per compared
iteration (the per-iteration bar of the first 100 iterations); the same
restart iterations, primal weights and residuals at every check; a solve to
1e-8 reaches it by the oracle's own KKT routine in the same number of
iterations and restarts as the oracle.
"""
import json
import os

import numpy as np
import pytest

import lpgen
import oracle
from oracle.pdhg import Params
from tests._gpu import announce, np_out, problem, rel

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _sample_index(size, seed, k=4096):
    """The sampled indices of tests/golden/make_goldens.py (same seeded draw)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(size, size=min(k, size), replace=False))


def _match_summary(v, s, tol, what):
    """v (full vector) against a stored summary: 2-norm and sampled entries,
    both relative to the stored vector's scale."""
    v = np.asarray(v, dtype=np.float64)
    assert v.size == s["size"], what
    vals = np.asarray(s["values"])
    got = v[_sample_index(v.size, s["index_seed"])]
    scale = max(np.abs(vals).max(), 1e-300)
    e_ent = float(np.abs(got - vals).max() / scale)
    e_nrm = abs(float(np.linalg.norm(v)) - s["norm2"]) / max(s["norm2"], 1e-300)
    print(f"{what}: sampled entries {e_ent:.1e}, norm {e_nrm:.1e}")
    assert e_ent <= tol and e_nrm <= tol, (what, e_ent, e_nrm)


def _compare_logs(gpu_log, ref_log, r_tol, omega_tol):
    assert [e["iter"] for e in gpu_log] == [e["t"] for e in ref_log]
    assert [bool(e["restart"]) for e in gpu_log] == [bool(e["restart"]) for e in ref_log]
    for g, o in zip(gpu_log, ref_log):
        assert g["k"] == o["k"]
        assert abs(g["omega"] - o["omega"]) <= omega_tol * o["omega"], (g["iter"], g["omega"], o["omega"])
        assert abs(g["r"] - o["r"]) <= r_tol * o["r"], (g["iter"], g["r"], o["r"])
        assert abs(g["r0"] - o["r0"]) <= r_tol * o["r0"], (g["iter"], g["r0"], o["r0"])
        for key in ("rel_kkt", "rel_gap", "rel_primal", "rel_dual"):
            assert abs(g[key] - o[key]) <= 1e-8 * o[key] + 1e-15, (g["iter"], key, g[key], o[key])


@pytest.mark.timeout(300)
def test_c2_solve_to_1e8_matches_oracle():
    """The medium LP solved to 1e-8 in FP64 with the oracle's stepsize: the same
    iteration count, restart iterations and primal weights as the oracle's
    solve (stored), the objective within 1e-10, the point within the
    tolerance by the oracle's KKT routine."""
    g = _golden("c2_solve.json")
    lp = lpgen.config("c2", seed=1)
    assert g["workload"] == f"c2: m={lp.m} n={lp.n} nnz={lp.nnz}"
    announce(f"c2 solve to 1e-8 vs stored oracle solve ({g['iters']} iterations)")
    prob = problem(lp, eta=g["eta"])
    out = prob.solve(tol=1e-8, want_r=False)
    prob.close()
    info, log = out["info"], out["log"]
    assert info["status"] == g["status"] == oracle.pdhg.OPTIMAL
    assert info["iters"] == g["iters"] and info["restarts"] == g["restarts"] and info["checks"] == g["checks"]
    rows = g["restart_log"]["rows"]
    got = [(e["iter"], e["omega"], e["r"]) for e in log if e["restart"]]
    assert [t for t, _, _ in got] == [int(t) for t, _, _ in rows]
    w_err = max(abs(a[1] - b[1]) / b[1] for a, b in zip(got, rows))
    r_err = max(abs(a[2] - b[2]) / b[2] for a, b in zip(got, rows))
    o = np_out(out)
    k = oracle.kkt(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, o["x"], o["y"])
    p_err = abs(k["pobj"] - g["info"]["pobj"]) / (1 + abs(g["info"]["pobj"]))
    print(f"c2: {info['iters']} iterations, {info['restarts']} restarts; omega err {w_err:.1e}, "
          f"r err {r_err:.1e}, pobj err {p_err:.1e}, oracle KKT of the GPU point {k['rel_kkt']:.3e}")
    assert w_err <= 1e-8 and r_err <= 1e-6
    assert k["rel_kkt"] <= 1e-8 * (1 + 1e-6)
    assert p_err <= 1e-10
    _match_summary(o["x"], g["x"], 1e-6, "c2 x")
    _match_summary(o["y"], g["y"], 1e-6, "c2 y")


@pytest.mark.timeout(900)
def test_c3b_scaling_stepsize_and_first_100_iterations_match_oracle():
    """The large skewed LP at full size (m=2e6, n=5e6, 29.6M nonzeros) in the
    bench's layout: scaling and power iteration against the stored oracle
    values; then 100 iterations with the oracle's stepsize against the oracle
    run here, with the artificial restart and PID update at iteration 64 and
    the final check at 100 inside the window."""
    g = _golden("c3b_setup.json")
    lp = lpgen.config("c3b", seed=1)
    assert g["workload"] == f"c3b: m={lp.m} n={lp.n} nnz={lp.nnz}"
    announce(f"c3b full size nnz={lp.nnz}: setup vs stored oracle values")
    prob = problem(lp)
    assert prob.panels()[0] == 40 and prob.dense()[1] > 0
    dr, dc, eta, passes = prob.scaling()
    prob.close()
    _match_summary(dr.cpu().numpy(), g["d_r"], 1e-12, "c3b d_r")
    _match_summary(dc.cpu().numpy(), g["d_c"], 1e-12, "c3b d_c")
    print(f"c3b eta {eta!r} vs oracle {g['eta']!r}; power passes {passes} vs {g['power_passes']}")
    assert eta == pytest.approx(g["eta"], rel=1e-9)
    assert abs(passes - g["power_passes"]) <= 1

    T = 100
    at = (1, 2, 3, 32, 63, 64, 65, 99, 100)
    announce("c3b: 100 iterations, GPU and oracle")
    prob = problem(lp, eta=g["eta"])
    out = prob.solve(tol=0.0, max_iter=T, trace_iters=T, want_r=False)
    gtr = {t: [out["trace"][k][t - 1].cpu().numpy() for k in ("xh", "yh", "x", "y")] for t in at}
    glog = out["log"]
    gx, gy = out["x"].cpu().numpy(), out["y"].cpu().numpy()
    prob.close()
    del out
    ref = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv,
                       Params(tol=0.0, max_iter=T, eta_override=g["eta"], trace_at=at))
    worst = 0.0
    for t in at:
        for key, a, b in zip(("xh", "yh", "x", "y"), gtr[t], ref.trace["at"][t]):
            e = rel(a, b)
            worst = max(worst, e)
            assert e <= 1e-10, (t, key, e)
    _compare_logs(glog, ref.log, 1e-9, 1e-12)
    assert [e["iter"] for e in glog if e["restart"]] == [64]
    assert rel(gx, ref.x) <= 1e-10 and rel(gy, ref.y) <= 1e-10
    print(f"c3b: worst trajectory error over {len(at)} sampled iterations {worst:.1e}; "
          f"checks {[(e['iter'], e['restart']) for e in glog]}")


@pytest.mark.timeout(600)
def test_c3a_scaling_stepsize_and_first_iterations_match_oracle():
    """The largest LP (m=2e6, n=5e6, 692M nonzeros, int32 offsets near 7e8)
    in the bench's layout (wide and narrow panels, the split transpose):
    scaling diagonals, stepsize and the first iterates against the oracle's
    stored values (sampled entries and norms)."""
    g = _golden("c3a_setup.json")
    lp = lpgen.config("c3a", seed=1)
    assert g["workload"] == f"c3a: m={lp.m} n={lp.n} nnz={lp.nnz}"
    announce(f"c3a full size nnz={lp.nnz}: setup vs stored oracle values")
    prob = problem(lp)
    assert prob.panels()[0] == 40 and prob.dense()[1] > 0
    dr, dc, eta, passes = prob.scaling()
    prob.close()
    _match_summary(dr.cpu().numpy(), g["d_r"], 1e-12, "c3a d_r")
    _match_summary(dc.cpu().numpy(), g["d_c"], 1e-12, "c3a d_c")
    print(f"c3a eta {eta!r} vs oracle {g['eta']!r}; power passes {passes} vs {g['power_passes']}")
    assert eta == pytest.approx(g["eta"], rel=1e-9)
    assert abs(passes - g["power_passes"]) <= 1
    T = g["iters"]
    prob = problem(lp, eta=g["eta"])
    out = prob.solve(tol=0.0, max_iter=T, trace_iters=T, want_r=False)
    for t in range(T):
        for key in ("xh", "yh", "x", "y"):
            _match_summary(out["trace"][key][t].cpu().numpy(), g["trajectory"][t][key], 1e-10, f"c3a {key} t={t + 1}")
    print(f"c3a relative KKT after {T} iterations {out['info']['rel_kkt']!r} vs oracle {g['final_rel_kkt']!r}")
    assert out["info"]["rel_kkt"] == pytest.approx(g["final_rel_kkt"], rel=1e-8)
    prob.close()


@pytest.mark.timeout(900)
def test_mixed_c3b_first_100_iterations_match_fp32_oracle():
    """The FP32 path on the large skewed LP at full size (wide and narrow
    panels, the split transpose, FP32 partial sums) against the oracle's FP32
    iteration (oracle/mixed.py) with the oracle's stepsize, over the first
    100 iterations, with the artificial restart and its re-centring at 64.
    Both sides sum FP32 products in FP32 but in different orders (panel and
    slice order here, row order in the oracle), so each row sum differs by
    rounding of about u * sqrt(L) relative for a row of L terms (u = 6e-8):
    up to about 1.3e-5 for the 50,000-nonzero rows, about 2e-7 for the short
    rows that make up most of the vector; over 100 nonexpansive steps the
    bar is 1e-4 relative in the 2-norm per compared iteration (the medium
    LP's bar 1e-5 scaled by the longest rows)."""
    from oracle.mixed import solve_mixed
    from paper_2507_14051_amd import MIXED
    g = _golden("c3b_setup.json")
    lp = lpgen.config("c3b", seed=1)
    T = 100
    at = (1, 2, 3, 32, 63, 64, 65, 99, 100)
    announce(f"mixed c3b full size nnz={lp.nnz}: 100 iterations, GPU and oracle/mixed.py")
    prob = problem(lp, eta=g["eta"], precision=MIXED)
    assert prob.panels()[0] == 40 and prob.dense()[1] > 0
    out = prob.solve(tol=0.0, max_iter=T, trace_iters=T, want_r=False)
    gtr = {t: [out["trace"][k][t - 1].cpu().numpy() for k in ("xh", "yh")] for t in at}
    glog = out["log"]
    prob.close()
    del out
    ref = solve_mixed(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv,
                      Params(tol=0.0, max_iter=T, eta_override=g["eta"], trace_at=at))
    worst = 0.0
    for t in at:
        for key, a, b in zip(("xh", "yh"), gtr[t], ref["trace"]["at"][t]):
            e = rel(a, b)
            worst = max(worst, e)
            assert e <= 1e-4, (t, key, e)
    assert [e["iter"] for e in glog] == [e["t"] for e in ref["log"]]
    assert [e["iter"] for e in glog if e["restart"]] == [64]
    for gl, rl in zip(glog, ref["log"]):
        assert abs(gl["rel_kkt"] - rl["rel_kkt"]) <= 1e-3 * rl["rel_kkt"], (gl["iter"], gl["rel_kkt"], rl["rel_kkt"])
    print(f"mixed c3b: worst relative error over {len(at)} sampled iterations vs oracle/mixed.py {worst:.2e}; "
          f"rel_kkt at the checks {[(e['iter'], e['rel_kkt']) for e in glog]} vs "
          f"{[(e['t'], e['rel_kkt']) for e in ref['log']]}")
