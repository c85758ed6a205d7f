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
    from paper_2507_14051_amd import FP64, MIXED
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
    xe = np.abs(om["x"] - of["x"]).max() / (1 + np.abs(of["x"]).max())
    ye = np.abs(om["y"] - of["y"]).max() / (1 + np.abs(of["y"]).max())
    oe = abs(om["info"]["pobj"] - of["info"]["pobj"]) / (1 + abs(of["info"]["pobj"]))
    print(f"mixed c2: iters {om['info']['iters']} vs fp64 {of['info']['iters']}; "
          f"x err {xe:.2e} y err {ye:.2e} obj err {oe:.2e}")
    assert oe <= 1e-7
