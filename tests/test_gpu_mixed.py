"""GPU mixed precision (FP32 iteration, FP64 checks and refinement at every
restart) against the oracle.  FP32 summation order differs between the GPU
and NumPy, so the trajectory is compared at FP32 accuracy (1e-5 relative over
the first iterations); the end result must meet the FP64 tolerance by the
oracle's own KKT routine, and its error against the FP64 solution is
reported."""
import numpy as np
import pytest

import lpgen
import oracle
from oracle.mixed import solve_mixed
from oracle.pdhg import Params
from tests._gpu import announce, np_out, oracle_eta, problem, rel

pytestmark = pytest.mark.gpu


def test_mixed_c1_matches_oracle_and_tolerance():
    from paper_2507_14051_amd import MIXED
    lp = lpgen.config("c1", seed=1)
    announce("mixed c1")
    eta = oracle_eta(lp)
    prob = problem(lp, eta=eta, precision=MIXED)
    T = 20
    out = prob.solve(tol=1e-8, trace_iters=T)
    tr = {k: v.cpu().numpy() for k, v in out["trace"].items()}
    ref = solve_mixed(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, Params(tol=1e-8, eta_override=eta), trace_iters=T)
    for t in range(T):
        assert rel(tr["xh"][t], ref["trace"]["xh"][t]) <= 1e-5
        assert rel(tr["yh"][t], ref["trace"]["yh"][t]) <= 1e-5
    o = np_out(out)
    info = o["info"]
    k = oracle.kkt(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, o["x"], o["y"])
    assert info["status"] == oracle.pdhg.OPTIMAL
    assert k["rel_kkt"] <= 1e-8 * (1 + 1e-6)
    f64 = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, Params(tol=1e-8, eta_override=eta))
    print(f"mixed iters {info['iters']} oracle-mixed iters {ref['iters']} fp64 iters {f64.iters}; "
          f"obj err {abs(k['pobj'] - f64.info['pobj']) / (1 + abs(f64.info['pobj'])):.2e}")
    assert abs(k["pobj"] - f64.info["pobj"]) <= 1e-7 * (1 + abs(f64.info["pobj"]))
    prob.close()


def test_mixed_c2_reaches_1e8():
    from paper_2507_14051_amd import MIXED
    lp = lpgen.config("c2", seed=1)
    announce(f"mixed c2 m={lp.m} n={lp.n}")
    pm = problem(lp, precision=MIXED)
    om = np_out(pm.solve(tol=1e-8))
    pm.close()
    pf = problem(lp)
    of = np_out(pf.solve(tol=1e-8))
    pf.close()
    k = oracle.kkt(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, om["x"], om["y"])
    assert om["info"]["status"] == oracle.pdhg.OPTIMAL
    assert k["rel_kkt"] <= 1e-8 * (1 + 1e-6)
    kf = oracle.kkt(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, of["x"], of["y"])
    assert of["info"]["status"] == oracle.pdhg.OPTIMAL
    assert kf["rel_kkt"] <= 1e-8 * (1 + 1e-6)
    xe = np.abs(om["x"] - of["x"]).max() / (1 + np.abs(of["x"]).max())
    ye = np.abs(om["y"] - of["y"]).max() / (1 + np.abs(of["y"]).max())
    oe = abs(om["info"]["pobj"] - of["info"]["pobj"]) / (1 + abs(of["info"]["pobj"]))
    print(f"mixed c2: iters {om['info']['iters']} vs fp64 {of['info']['iters']}; "
          f"x err {xe:.2e} y err {ye:.2e} obj err {oe:.2e}")
    assert oe <= 1e-7


def test_mixed_c2_first_100_iterations_match_oracle_and_errors_vs_fp64_oracle():
    """The FP32 path on the medium LP against the oracle's FP32 iteration
    (oracle/mixed.py) over the first 100 iterations, at FP32 accuracy: the
    two sum in different orders, so each rounding differs by about one FP32
    ulp and the iterates may drift apart by a few hundred ulps over 100
    nonexpansive steps (bar 1e-5 relative).  Then the full solve's result
    against the FP64 oracle's solution to 1e-8 (stored by
    tests/golden/make_goldens.py): errors of the objective and of x, y at the
    sampled indices, reported per result."""
    import json
    import os
    from paper_2507_14051_amd import MIXED
    lp = lpgen.config("c2", seed=1)
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_solve.json")))
    announce("mixed c2 first 100 iterations vs oracle/mixed.py")
    eta = g["eta"]
    prob = problem(lp, eta=eta, precision=MIXED)
    T = 100
    out = prob.solve(tol=0.0, max_iter=T, trace_iters=T, want_r=False)
    tr = {k: out["trace"][k].cpu().numpy() for k in ("xh", "yh")}
    ref = solve_mixed(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, Params(tol=0.0, max_iter=T, eta_override=eta),
                      trace_iters=T)
    worst = 0.0
    for t in range(T):
        for key in ("xh", "yh"):
            e = rel(tr[key][t], ref["trace"][key][t])
            worst = max(worst, e)
            assert e <= 1e-5, (key, t, e)
    assert [e["iter"] for e in out["log"]] == [e["t"] for e in ref["log"]]
    print(f"mixed c2: worst relative error over 100 iterations vs oracle/mixed.py {worst:.2e}")
    full = np_out(prob.solve(tol=1e-8))
    prob.close()
    info = full["info"]
    assert info["status"] == oracle.pdhg.OPTIMAL
    k = oracle.kkt(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, full["x"], full["y"])
    assert k["rel_kkt"] <= 1e-8 * (1 + 1e-6)
    from tests.test_gpu_fullsize import _sample_index
    errs = {}
    for key in ("x", "y"):
        s = g[key]
        vals = np.asarray(s["values"])
        got = full[key][_sample_index(s["size"], s["index_seed"])]
        errs[key] = float(np.abs(got - vals).max() / (1 + np.abs(vals).max()))
    errs["pobj"] = abs(k["pobj"] - g["info"]["pobj"]) / (1 + abs(g["info"]["pobj"]))
    print(f"mixed c2 vs FP64 oracle solution: objective {errs['pobj']:.2e}, x {errs['x']:.2e}, y {errs['y']:.2e} "
          f"(max-norm at sampled indices relative to 1 + max|.|); {info['iters']} iterations vs {g['iters']}")
    assert errs["pobj"] <= 1e-7


def test_mixed_long_and_dense_rows_solve_to_1e8():
    """The FP32 path with wide and narrow panels on a Zipf LP (long and dense
    rows): a solve to 1e-8 checked by the oracle's KKT routine, and the check
    quantities of its first runs (iterations, restart decisions, relative KKT,
    residual) equal to the unsplit FP32 path's at FP32 accuracy."""
    from paper_2507_14051_amd import MIXED
    lp = lpgen.gen(3000, 20000, zipf_alpha=1.3, cap=9000, eq_frac=0.3, free_frac=0.2, values="normal", seed=7)
    announce(f"mixed panels solve to 1e-8 nnz={lp.nnz}")
    eta = oracle_eta(lp)
    pp = problem(lp, eta=eta, precision=MIXED, column_panels=16, panel_row_min=8, dense_row_min=512)
    assert pp.panels()[0] == 16 and pp.panels()[1] > 0 and pp.dense()[1] > 0
    short = pp.solve(tol=0.0, max_iter=640, want_r=False)["log"]
    o = np_out(pp.solve(tol=1e-8, max_iter=400000))
    pp.close()
    plain = problem(lp, eta=eta, precision=MIXED, column_panels=0)
    ref = plain.solve(tol=0.0, max_iter=640, want_r=False)["log"]
    plain.close()
    assert [e["iter"] for e in short] == [e["iter"] for e in ref]
    assert [e["restart"] for e in short] == [e["restart"] for e in ref]
    for a, b in zip(short, ref):
        assert abs(a["rel_kkt"] - b["rel_kkt"]) <= 1e-4 * b["rel_kkt"], (a["iter"], a["rel_kkt"], b["rel_kkt"])
        assert abs(a["r"] - b["r"]) <= 1e-4 * b["r"], (a["iter"], a["r"], b["r"])
    k = oracle.kkt(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, o["x"], o["y"])
    print(f"mixed panels: {o['info']['iters']} iterations, GPU rel_kkt {o['info']['rel_kkt']:.2e}, "
          f"oracle KKT {k['rel_kkt']:.2e}")
    assert o["info"]["status"] == oracle.pdhg.OPTIMAL and k["rel_kkt"] <= 1e-8 * (1 + 1e-6)
