"""Write the oracle's reference values for the full-size parity tests.

    python tests/golden/make_goldens.py c2     # solve of the medium LP to 1e-8
    python tests/golden/make_goldens.py c3b    # scaling and stepsize of the skewed LP (~3e7 nonzeros)
    python tests/golden/make_goldens.py c3a    # scaling, stepsize, first iterations (~6.9e8 nonzeros)
    python tests/golden/make_goldens.py c3b_small  # the primal-weight switches on the c3b recipe at 1/500 size

Every number written here comes from the FP64 CPU oracle (``oracle/``) on the
seeded inputs of ``lpgen``; nothing is read from the GPU library.  The
outputs are small JSON files beside this script.  Vectors too long to store
are summarised by their 2-norm and by their entries at fixed sampled indices
(drawn from a seeded generator of their own).

c2 runs the oracle to 1e-8 (about 10 minutes on one core); c3b needs the
oracle's power iteration on a 3e7-nonzero matrix (minutes); c3a needs about
40 GB of memory and an hour on one core.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import lpgen  # noqa: E402
import oracle  # noqa: E402
from oracle.pdhg import Params, power_norm, rescale  # noqa: E402

SAMPLES = 4096


def sample_index(size, seed):
    """Fixed sampled indices of a vector of the given size (sorted, distinct)."""
    rng = np.random.default_rng(seed)
    k = min(SAMPLES, size)
    return np.sort(rng.choice(size, size=k, replace=False))


def summary(v, seed):
    v = np.asarray(v, dtype=np.float64)
    idx = sample_index(v.size, seed)
    return {"norm2": float(np.linalg.norm(v)), "index_seed": seed, "size": int(v.size),
            "values": [float(t) for t in v[idx]]}


def log(msg):
    print(msg, flush=True)


def write(name, data):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    log(f"wrote {path}")


def stepsize(lp):
    t0 = time.perf_counter()
    At, dr, dc = rescale(lp.A, 10, 1)
    t1 = time.perf_counter()
    nrm, passes = power_norm(At, 5000, 1e-8)
    log(f"scaling {t1 - t0:.1f} s, power iteration {time.perf_counter() - t1:.1f} s ({passes} passes)")
    return At, dr, dc, 0.998 / nrm, passes


def make_c2():
    lp = lpgen.config("c2", seed=1)
    _, _, _, eta, passes = stepsize(lp)
    t0 = time.perf_counter()
    res = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, Params(tol=1e-8, eta_override=eta))
    log(f"solve {time.perf_counter() - t0:.1f} s: status {res.status}, {res.iters} iterations, "
        f"{res.restarts} restarts, rel_kkt {res.info['rel_kkt']:.3e}")
    restarts = [[e["t"], e["omega"], e["r"]] for e in res.log if e["restart"]]
    write("c2_solve.json", {
        "source": "FP64 CPU oracle: the medium LP (lpgen config c2, seed 1) solved to 1e-8 relative KKT "
                  "from the all-zero start with the paper's settings; eta from the oracle's own scaling and "
                  "power iteration.",
        "workload": f"c2: m={lp.m} n={lp.n} nnz={lp.nnz}", "eta": eta, "power_passes": passes,
        "status": res.status, "iters": res.iters, "restarts": res.restarts, "omega": res.omega,
        "checks": len(res.log), "info": res.info,
        "restart_log": {"columns": ["iter", "omega_before_update", "r"], "rows": restarts},
        "x": summary(res.x, 101), "y": summary(res.y, 102)})


def make_c3b():
    lp = lpgen.config("c3b", seed=1)
    At, dr, dc, eta, passes = stepsize(lp)
    write("c3b_setup.json", {
        "source": "FP64 CPU oracle: scaling (10 Ruiz passes, one Pock-Chambolle pass) and stepsize "
                  "eta = 0.998 / ||A~||_2 by power iteration (tol 1e-8, at most 5000 passes) of the skewed "
                  "LP lpgen config c3b, seed 1.",
        "workload": f"c3b: m={lp.m} n={lp.n} nnz={lp.nnz}", "eta": eta, "power_passes": passes,
        "d_r": summary(dr, 201), "d_c": summary(dc, 202)})


def make_c3a(iters=3):
    t0 = time.perf_counter()
    lp = lpgen.config("c3a", seed=1)
    log(f"generated c3a in {time.perf_counter() - t0:.1f} s: nnz {lp.nnz}")
    At, dr, dc = rescale(lp.A, 10, 1)
    write_c3a = {"source": "FP64 CPU oracle on the skewed LP lpgen config c3a, seed 1: scaling (10 Ruiz "
                           "passes, one Pock-Chambolle pass), stepsize by power iteration, and the iterates "
                           f"of its first {iters} iterations from the all-zero start.",
                 "workload": f"c3a: m={lp.m} n={lp.n} nnz={lp.nnz}",
                 "d_r": summary(dr, 301), "d_c": summary(dc, 302)}
    write("c3a_setup.json", write_c3a)
    t1 = time.perf_counter()
    nrm, passes = power_norm(At, 5000, 1e-8)
    eta = 0.998 / nrm
    del At
    log(f"power iteration {time.perf_counter() - t1:.1f} s ({passes} passes)")
    write_c3a.update(eta=eta, power_passes=passes)
    write("c3a_setup.json", write_c3a)
    res = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv,
                       Params(tol=0.0, max_iter=iters, eta_override=eta, trace_iters=iters))
    traj = []
    for t in range(iters):
        traj.append({key: summary(res.trace[key][t], 310 + i) for i, key in enumerate(("xh", "yh", "x", "y"))})
    write_c3a.update(iters=iters, trajectory=traj, final_rel_kkt=res.info["rel_kkt"])
    write("c3a_setup.json", write_c3a)


SWITCHES = {
    "paper_default": {},
    "omega_ratio": dict(kp=1.0, ki=0.0, kd=0.0),
    "omega_smoothed": dict(kp=0.5, ki=0.0, kd=0.0),
    "omega_fixed": dict(kp=0.0, ki=0.0, kd=0.0),
    "halpern_gamma0": dict(gamma=0.0),
}


def make_c3b_small(iters=60000):
    """How far each primal-weight rule gets on the skewed family: the c3b
    recipe at 1/500 of its size, FP64 oracle, from the all-zero start."""
    lp = lpgen.config("c3b", seed=1, scale=0.002)
    _, _, _, eta, passes = stepsize(lp)
    out = {"source": "FP64 CPU oracle on lpgen config c3b, seed 1, scale 0.002 (Zipf(1.882) rows, values "
                     f"sign*10^U[-3,3]), {iters} iterations (or to 1e-8) under each primal-weight switch, eta from "
                     "the oracle's scaling and power iteration; every 20th check kept.",
           "workload": f"c3b at 1/500: m={lp.m} n={lp.n} nnz={lp.nnz}", "eta": eta, "power_passes": passes,
           "columns": ["iter", "rel_kkt", "rel_gap", "rel_primal", "rel_dual", "omega", "restart"], "by_switch": {}}
    for name, kw in SWITCHES.items():
        t0 = time.perf_counter()
        res = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv,
                           Params(tol=1e-8, max_iter=iters, eta_override=eta, **kw))
        rows = [[e["t"], e["rel_kkt"], e["rel_gap"], e["rel_primal"], e["rel_dual"], e["omega"], int(e["restart"])]
                for e in res.log[19::20]]
        out["by_switch"][name] = {"params": kw, "status": res.status, "iters": res.iters,
                                  "restarts": res.restarts, "final": {k: res.info[k] for k in (
                                      "rel_kkt", "rel_gap", "rel_primal", "rel_dual")},
                                  "omega": res.omega, "log": rows}
        log(f"{name}: {time.perf_counter() - t0:.0f} s, status {res.status}, {res.iters} iterations, "
            f"rel_kkt {res.info['rel_kkt']:.3e}, omega {res.omega:.3g}")
    write("c3b_small_switches.json", out)


if __name__ == "__main__":
    what = sys.argv[1:] or ["c2", "c3b"]
    for w in what:
        {"c2": make_c2, "c3b": make_c3b, "c3a": make_c3a, "c3b_small": make_c3b_small}[w]()
