"""Benchmark: restarted reflected Halpern PDHG on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (one "step"): one full solve of the medium synthetic LP
(m=100,000, n=200,000, 8 nonzeros per row at uniform random columns, N(0,1)
values, 30% equality rows, 20% of the columns free above) to 1e-8 relative KKT
error in FP64, inputs resident in HBM and the handle set up (transpose,
rescaling, power iteration) before the timed region.  ``value`` is PDHG
iterations per second over the timed steps.  The same run also reports the
setup time, the FP32 + refinement solve of the same LP to 1e-8, the dominant
kernel against the HBM roofline (HIP events on the library's stream), the
HBM-bound skewed LP (m=2e6, n=5e6, Zipf row lengths, ~3e7 nonzeros) and the
FP64 CPU oracle on a bounded sample of the medium LP.  Prints ONE JSON line.

    python bench.py --kernels-only

runs only the per-kernel timing of the medium LP and a 256 MiB copy of known
size (used to calibrate hardware counters); it is the command profiled with
rocprofv3 --pmc.
"""
import os

# The CPU baseline is the single-threaded oracle; pin the BLAS/OpenMP pools to
# one thread before numpy loads so "cores" is what actually runs.
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import argparse
import hashlib
import json
import math
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "c2"
KERNEL_SOURCES = ("paper_2507_14051_amd/csrc/kernels_iter.hip", "paper_2507_14051_amd/csrc/device.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_primal_c2.md")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(m, n, nnz, fp=8):
    """Bytes one kernel must move (each array once, gathered vectors once).

    primal half-step: col_ptr 4(n+1), row idx 4 nnz, values fp nnz, y gathered fp m,
                      x, x0, c, lv, uv read (5 fp n), xbar and x written (2 fp n)
    dual half-step:   row_ptr 4(m+1), col idx 4 nnz, values fp nnz, xbar gathered fp n,
                      y, y0, lc, uc read (4 fp m), y written (fp m)"""
    primal = 4 * (n + 1) + (4 + fp) * nnz + fp * m + 7 * fp * n
    dual = 4 * (m + 1) + (4 + fp) * nnz + fp * n + 5 * fp * m
    return primal, dual


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM bytes per launch of the FP64 primal half-step from the committed
    rocprofv3 --pmc summary, if it was taken on the current kernel sources."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d


HBM_WORKLOADS = {
    "c3b": "c3b: m=2000000 n=5000000 nnz={nnz} Zipf(1.882) rows capped at 50,000, values +-10^U[-3,3]",
    "c3a": "c3a: m=2000000 n=5000000 nnz={nnz} Zipf(1.5) rows capped at 50,000, values +-10^U[-3,3]",
}


def measure_hbm(dev, name="c3b", iters=640):
    """Iteration rate and per-kernel GB/s on a large skewed LP (rows of
    Zipf-distributed length) whose two matrices exceed the 256 MB Infinity
    Cache: the HBM-bound case."""
    import torch

    import lpgen
    from paper_2507_14051_amd import MIXED, Problem

    t0 = time.perf_counter()
    lp3 = lpgen.config(name, seed=1, progress=lambda k, n: log(f"# {name}: rows chunk {k}/{n}") if k % 8 == 0 else None)
    gen_s = time.perf_counter() - t0
    m3, n3, nnz3 = lp3.m, lp3.n, lp3.nnz
    log(f"# hbm-bound {name}: m={m3} n={n3} nnz={nnz3} max_row={lp3.meta['max_row']} "
        f"rows_at_cap={lp3.meta['rows_at_cap']} (generated in {gen_s:.0f} s)")
    t0 = time.perf_counter()
    p3 = Problem(lp3.A, lp3.c, lp3.lc, lp3.uc, lp3.lv, lp3.uv, device=dev)
    torch.cuda.synchronize()
    s3 = time.perf_counter() - t0
    panels = p3.panels()
    dense = p3.dense()
    _, _, _, power_iters = p3.scaling()
    log(f"# {name}: setup {s3:.2f} s (power iterations {power_iters}), panels {panels}, dense {dense}")
    p3.solve(max_iter=64, tol=0.0, want_r=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p3.solve(max_iter=iters, tol=0.0, want_r=False)
    torch.cuda.synchronize()
    it_s = iters / (time.perf_counter() - t0)
    pr3 = p3.profile(iters=min(100, iters))
    pb3, db3 = algorithmic_bytes(m3, n3, nnz3)
    hbm = {"workload": HBM_WORKLOADS[name].format(nnz=nnz3), "setup_s": round(s3, 3),
           "power_iters": power_iters, "column_panels": panels[0], "long_rows": panels[1],
           "narrow_panels": dense[0], "dense_rows": dense[1],
           "iters_per_s": round(it_s, 1),
           "primal_us": round(pr3["primal_ms"] * 1e3, 2), "dual_us": round(pr3["dual_ms"] * 1e3, 2),
           "primal_gbs": round(pb3 / (pr3["primal_ms"] * 1e-3) / 1e9, 1),
           "dual_gbs": round(db3 / (pr3["dual_ms"] * 1e-3) / 1e9, 1),
           "iter_gbs": round((pb3 + db3) / (pr3["iter_ms"] * 1e-3) / 1e9, 1)}
    hbm["iter_frac_of_peak"] = round(hbm["iter_gbs"] / HBM_PEAK_GBS, 4)
    eta3 = p3.scaling()[2]
    p3.close()
    # the same plain iterations in FP32 (mixed precision: FP32 matrix copies
    # and iterates, FP64 refinement at restarts), same stepsize
    pm = Problem(lp3.A, lp3.c, lp3.lc, lp3.uc, lp3.lv, lp3.uv, device=dev, precision=MIXED, eta_override=eta3)
    del lp3
    pm.solve(max_iter=64, tol=0.0, want_r=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pm.solve(max_iter=iters, tol=0.0, want_r=False)
    torch.cuda.synchronize()
    itm = iters / (time.perf_counter() - t0)
    prm = pm.profile(iters=min(100, iters))
    pm.close()
    hbm["fp32"] = {"iters_per_s": round(itm, 1), "speedup_vs_fp64": round(itm / it_s, 3),
                   "primal_us": round(prm["primal_ms"] * 1e3, 2), "dual_us": round(prm["dual_ms"] * 1e3, 2)}
    log(f"# hbm: {hbm}")
    return hbm


def measure_adjoint(dev, K=2000, ckpt=100, reps=3):
    """The differentiation workload (c5: m=50,000, n=100,000, 8 nnz/row): K
    unrolled iterations with a checkpoint every ckpt (hlp_unrolled_forward),
    then the reverse pass (hlp_unrolled_backward) for the loss
    ||x - x_target||^2 + c^T x; times of both and their ratio."""
    import torch

    import lpgen
    from paper_2507_14051_amd import Problem
    from paper_2507_14051_amd.hlp import hlp_tape_bytes, hlp_unrolled_backward, hlp_unrolled_forward

    lp = lpgen.config("c5", seed=1)
    prob = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device=dev)
    f64 = dict(dtype=torch.float64, device=dev)
    p = prob.params_for()
    tape = torch.empty(hlp_tape_bytes(prob.handle, K, ckpt), dtype=torch.uint8, device=dev)
    x = torch.empty(prob.n, **f64)
    y = torch.empty(prob.m, **f64)
    c = torch.as_tensor(lp.c, **f64)
    xt = torch.as_tensor(lpgen.x_target(lp.n, seed=1), **f64)
    g = [torch.empty(k, **f64) for k in (prob.n, prob.m, prob.m, prob.n, prob.n)]
    fw, bw = [], []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hlp_unrolled_forward(prob.handle, p, K, ckpt, 0, None, None, x, y, tape)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gx = 2.0 * (x - xt) + c
        gy = torch.zeros_like(y)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        hlp_unrolled_backward(prob.handle, tape, gx, gy, *g)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if r:
            fw.append(t1 - t0)
            bw.append(t3 - t2)
    prob.close()
    f, b = min(fw), min(bw)
    out = {"workload": f"c5: m={lp.m} n={lp.n} nnz={lp.nnz}, K={K} unrolled iterations, checkpoint every {ckpt}",
           "forward_ms": round(f * 1e3, 2), "backward_ms": round(b * 1e3, 2),
           "backward_over_forward": round(b / f, 2), "forward_iter_us": round(f / K * 1e6, 2),
           "tape_mb": round(tape.numel() / 1e6, 1)}
    log(f"# adjoint: {out}")
    return out


# Switches of the method the paper argues for (Sec. 3).  PID gains (theta, 0, 0)
# are the exponentially smoothed distance-ratio primal-weight update the paper
# attributes to cuPDLP, theta = 1 its unsmoothed form; zero gains keep the
# weight fixed.  A beta of -1 turns a decay test off, 1e18 the artificial one.
ABLATIONS = {
    "paper_default": {},
    "halpern_gamma0": dict(gamma=0.0),
    "gamma_half": dict(gamma=0.5),
    "omega_ratio": dict(kp=1.0, ki=0.0, kd=0.0),
    "omega_smoothed": dict(kp=0.5, ki=0.0, kd=0.0),
    "omega_fixed": dict(kp=0.0, ki=0.0, kd=0.0),
    "no_sufficient": dict(beta_sufficient=-1.0),
    "no_necessary": dict(beta_necessary=-1.0),
    "no_artificial": dict(beta_artificial=1e18),
    "no_restarts": dict(beta_sufficient=-1.0, beta_necessary=-1.0, beta_artificial=1e18),
}


def measure_ablation(dev, max_iter=600000, c1_seeds=8):
    """Iterations to 1e-8 relative KKT under each switch: the medium LP (seed
    1) and the geometric mean over c1_seeds small LPs, relative to the
    paper's settings.  One handle per LP, so every variant takes the same
    scaling and stepsize."""
    import torch

    import lpgen
    from paper_2507_14051_amd import Problem

    def run(lp, tag):
        prob = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device=dev)
        res = {}
        for name, kw in ABLATIONS.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = prob.solve(tol=1e-8, max_iter=max_iter, want_r=False, **kw)["info"]
            torch.cuda.synchronize()
            res[name] = {"iters": info["iters"], "restarts": info["restarts"], "status": info["status"],
                         "rel_kkt": info["rel_kkt"], "time_s": round(time.perf_counter() - t0, 3)}
            log(f"# ablation {tag} {name}: {res[name]}")
        prob.close()
        return res

    med = run(lpgen.config("c2", seed=1), "c2")
    base = med["paper_default"]["iters"]
    for r in med.values():
        r["iters_vs_default"] = round(r["iters"] / base, 3)
    small = [run(lpgen.config("c1", seed=s), f"c1 seed {s}") for s in range(1, c1_seeds + 1)]
    geo = {}
    for name in ABLATIONS:
        ratios = [r[name]["iters"] / r["paper_default"]["iters"] for r in small]
        geo[name] = {"geomean_iters_vs_default": round(math.exp(sum(map(math.log, ratios)) / len(ratios)), 3),
                     "solved": sum(r[name]["status"] == 0 for r in small), "of": len(small)}
    return {"tol": 1e-8, "max_iter": max_iter, "c2_seed1": med, f"c1_seeds_1_to_{c1_seeds}": geo}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiation workload")
    ap.add_argument("--no-hbm", action="store_true", help="skip the HBM-bound skewed LPs (c3b, c3a)")
    ap.add_argument("--profile-iters", type=int, default=400)
    ap.add_argument("--kernels-only", action="store_true",
                    help="only time the half-steps of --kernels-workload and a 256 MiB copy (for counter runs)")
    ap.add_argument("--kernels-workload", default=WORKLOAD, choices=("c2", "c3b", "c3a"))
    ap.add_argument("--hbm-only", action="store_true", help="only the skewed-LP measurement (for profiling it)")
    ap.add_argument("--hbm-workload", default="c3b", choices=("c3b", "c3a"),
                    help="LP of --hbm-only (c3a: ~6.9e8 nonzeros, minutes to generate)")
    ap.add_argument("--ablation", action="store_true",
                    help="only the iterations-to-tolerance of the method's switches (reflection, primal weight, "
                         "restart tests)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import lpgen
    from paper_2507_14051_amd import MIXED, OPTIMAL, Problem

    dev = torch.device("cuda:0")
    if args.ablation:
        print(json.dumps({"ablation": measure_ablation(dev)}), flush=True)
        return
    if args.hbm_only:
        iters = 640 if args.hbm_workload == "c3b" else 128
        print(json.dumps({"hbm_only": True, "hbm_bound": measure_hbm(dev, args.hbm_workload, iters)}), flush=True)
        return
    wl = args.kernels_workload if args.kernels_only else WORKLOAD
    lp = lpgen.config(wl, seed=1)
    tol = lpgen.tolerance(wl)
    m, n, nnz = lp.m, lp.n, lp.nnz
    pb, db = algorithmic_bytes(m, n, nnz)
    log(f"# workload {wl}: m={m} n={n} nnz={nnz} max_row={lp.meta['max_row']}")

    t0 = time.perf_counter()
    prob = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device=dev)
    torch.cuda.synchronize()
    setup_wall = time.perf_counter() - t0
    _, _, eta, power_iters = prob.scaling()

    if args.kernels_only:
        prof = prob.profile(iters=args.profile_iters)
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)   # 256 MiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"kernels_only": True, "workload": wl, "primal_us": prof["primal_ms"] * 1e3,
                          "dual_us": prof["dual_ms"] * 1e3, "iters": prof["iters"],
                          "primal_bytes": pb, "dual_bytes": db, "copy_bytes": 2 * a.numel() * 8,
                          "kernel_source_hash": kernel_source_hash()}), flush=True)
        prob.close()
        return

    for _ in range(args.warmup):
        prob.solve(tol=tol, want_r=False)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(prob.solve(tol=tol, want_r=False)["info"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    iters = sum(i["iters"] for i in infos)
    ok = all(i["status"] == OPTIMAL for i in infos)
    ms_per_step = 1e3 * elapsed / args.steps
    log(f"# fp64: {infos[-1]['iters']} iters, {ms_per_step:.1f} ms/solve, rel_kkt {infos[-1]['rel_kkt']:.2e}")

    # dominant kernel against the roofline: HIP events around every launch
    prof = prob.profile(iters=args.profile_iters)
    kern = "primal" if prof["primal_ms"] >= prof["dual_ms"] else "dual"
    kms = prof["primal_ms"] if kern == "primal" else prof["dual_ms"]
    kbytes = pb if kern == "primal" else db
    achieved = kbytes / (kms * 1e-3) / 1e9
    tr = load_traffic() if kern == "primal" else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": (tr["traffic_bytes_per_launch"] if tr else None),
                "kernel": f"k_{kern} (fused {'transpose ' if kern == 'primal' else ''}SpMV + update), FP64",
                "bytes_per_launch": kbytes, "avg_launch_us": round(kms * 1e3, 3),
                "primal_avg_launch_us": round(prof["primal_ms"] * 1e3, 3),
                "dual_avg_launch_us": round(prof["dual_ms"] * 1e3, 3),
                "iter_us_with_events": round(prof["iter_ms"] * 1e3, 3),
                "solve_iter_us": round(1e6 * elapsed / iters, 3)}
    prob.close()

    mixed = None
    if not args.no_mixed:
        probm = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device=dev, precision=MIXED)
        probm.solve(tol=tol, want_r=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mi = [probm.solve(tol=tol, want_r=False)["info"] for _ in range(args.steps)]
        torch.cuda.synchronize()
        mt = (time.perf_counter() - t0) / args.steps
        profm = probm.profile(iters=args.profile_iters)
        pb32, db32 = algorithmic_bytes(m, n, nnz, fp=4)
        mixed = {"time_to_tol_s": round(mt, 4), "iters": mi[-1]["iters"], "status": mi[-1]["status"],
                 "rel_kkt": mi[-1]["rel_kkt"], "iters_per_s": round(mi[-1]["iters"] / mt, 1),
                 "speedup_vs_fp64_time": round((elapsed / args.steps) / mt, 3),
                 "primal_us": round(profm["primal_ms"] * 1e3, 3), "dual_us": round(profm["dual_ms"] * 1e3, 3),
                 "primal_gbs": round(pb32 / (profm["primal_ms"] * 1e-3) / 1e9, 1)}
        probm.close()
        log(f"# mixed: {mixed}")

    hbm = hbm_a = None
    if not args.no_hbm:
        hbm = measure_hbm(dev, "c3b", 640)
        hbm_a = measure_hbm(dev, "c3a", 128)

    adjoint = None if args.no_adjoint else measure_adjoint(dev)

    cpu = None
    if not args.no_cpu:
        import oracle
        K = 2000
        res = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, oracle.Params(tol=tol, max_iter=K))
        cpu = {"value": round(K / res.info["iter_s"], 3), "unit": "iter/s", "cores": 1, "kind": "oracle",
               "sample": f"{K} oracle iterations of the same LP (its own scaling and power iteration, "
                         f"{res.info['setup_s']:.1f} s, not counted), NumPy/SciPy FP64 single thread; "
                         f"host nproc={os.cpu_count()}"}
        log(f"# cpu: {cpu}")

    line = {
        "metric": "PDHG iterations/s, FP64 solve to 1e-8 relative KKT (time-to-tolerance and HBM roofline alongside)",
        "value": round(iters / elapsed, 1), "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{WORKLOAD}: m={m} n={n} nnz={nnz} (8/row uniform columns, N(0,1) values, "
                               f"30% equality rows, 20% free columns), tol {tol:g}",
                   "seed": 1, "global_batch": 1, "parallelism": "single GPU"},
        "time_to_tol_s": round(elapsed / args.steps, 4), "iters_per_solve": infos[-1]["iters"],
        "restarts": infos[-1]["restarts"], "rel_kkt": infos[-1]["rel_kkt"], "all_optimal": ok,
        "setup_s": round(setup_wall, 4), "power_iters": power_iters,
        "mixed": mixed, "hbm_bound": hbm, "hbm_bound_c3a": hbm_a, "adjoint": adjoint, "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
