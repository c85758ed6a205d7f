"""Benchmark: restarted reflected Halpern PDHG on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Headline workload: the largest configuration, the skewed LP with the literal
row-length law (m=2,000,000, n=5,000,000, Zipf(1.5) row lengths capped at
50,000 -- 692M nonzeros, 7,007 rows at the cap -- values sign * 10^U[-3,3],
30% equality rows, 20% of the columns free above), in FP64, inputs resident
in HBM and the handle set up (transpose, rescaling, power iteration) before
the timed region.  One step is one FP64 solve from the all-zero start with
the paper's settings and tolerance 1e-8, capped at --step-iters PDHG
iterations (every 64 iterations a check: fixed-point residual, relative KKT,
restart tests, PID update).  ``value`` is PDHG iterations per second over the
timed steps.

The same run reports, for the headline LP, one solve under a time limit in
FP64 and in FP32 with refinement (status, relative KKT reached and its course
over time: 1e-8 is out of reach in a benchmark's time on this LP family), the
dominant half-step against the HBM roofline (HIP events on the library's
stream) and a measured device-copy bandwidth; the same for the skewed LP of
the stated size (~3e7 nonzeros); the medium LP (cache-resident) solved to
1e-8 in FP64 and FP32; the differentiation workload; and the FP64 CPU oracle
on a bounded sample of the headline LP.  Prints ONE JSON line.

    python bench.py --kernels-only --kernels-workload c3a

runs only the per-half-step timing of an LP and a 256 MiB copy of known size
(used to calibrate hardware counters); it is the command profiled with
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
HEADLINE = "c3a"
KERNEL_SOURCES = ("paper_2507_14051_amd/csrc/kernels_iter.hip", "paper_2507_14051_amd/csrc/device.h",
                  "paper_2507_14051_amd/csrc/abi.cpp")  # the kernels and the layout rules
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_half_steps.md")
C3B_GOLDEN = os.path.join(ROOT, "tests", "golden", "c3b_setup.json")

WORKLOADS = {
    "c2": "c2: m={m} n={n} nnz={nnz} (8 nonzeros per row at uniform columns, N(0,1) values, 30% equality rows, "
          "20% free columns)",
    "c3a": "c3a: m={m} n={n} nnz={nnz} (Zipf(1.5) row lengths capped at 50,000, {cap} rows at the cap, values "
           "sign*10^U[-3,3], 30% equality rows, 20% free columns)",
    "c3b": "c3b: m={m} n={n} nnz={nnz} (Zipf(1.882) row lengths capped at 50,000, {cap} rows at the cap, values "
           "sign*10^U[-3,3], 30% equality rows, 20% free columns)",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def describe(name, lp):
    return WORKLOADS[name].format(m=lp.m, n=lp.n, nnz=lp.nnz, cap=lp.meta.get("rows_at_cap", 0))


def algorithmic_bytes(m, n, nnz, fp=8):
    """Bytes one half-step must move (each array once, gathered vectors once).

    primal half-step: col_ptr 4(n+1), row idx 4 nnz, values fp nnz, y gathered fp m,
                      x, x0, c, lv, uv read (5 fp n), xbar and x written (2 fp n)
    dual half-step:   row_ptr 4(m+1), col idx 4 nnz, values fp nnz, xbar gathered fp n,
                      y, y0, lc, uc read (4 fp m), y written (fp m)"""
    primal = 4 * (n + 1) + (4 + fp) * nnz + fp * m + 7 * fp * n
    dual = 4 * (m + 1) + (4 + fp) * nnz + fp * n + 5 * fp * m
    return primal, dual


def kernel_source_hash():
    """Hash of the kernel and layout sources with comments and blank space
    removed, so that an edit of a comment keeps a traffic record valid and an
    edit of the code does not."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(workload, half):
    """HBM bytes per launch of an FP64 half-step ("primal" or "dual") from the
    committed rocprofv3 --pmc summary, if it was taken on the current kernel
    sources."""
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
    return d.get(workload, {}).get(half)


def reserve_device_memory(dev, lp):
    """One device allocation up front, returned at once to torch's caching
    allocator, large enough for the biggest workspace of the run (the FP32
    path's) and the inputs: the later Problems, FP64 and FP32, are carved from
    it and so sit on the same device memory.  (Without it the FP32 problem gets
    a fresh allocation after the FP64 one was freed; such a second allocation
    has run the 692M-nonzero LP's primal half-step up to 5% slower than the
    first, with identical results; with the memory reused it does not.)"""
    import torch
    from paper_2507_14051_amd import MIXED
    from paper_2507_14051_amd.hlp import hlp_params_default, hlp_workspace_bytes
    ws = max(hlp_workspace_bytes(lp.m, lp.n, lp.nnz, hlp_params_default()),
             hlp_workspace_bytes(lp.m, lp.n, lp.nnz, hlp_params_default(precision=MIXED)))
    inputs = 12 * lp.nnz + 4 * (lp.m + 1) + 8 * (3 * lp.n + 2 * lp.m)
    try:
        r = torch.empty(ws + inputs + (1 << 30), dtype=torch.uint8, device=dev)
    except torch.cuda.OutOfMemoryError:
        log(f"# could not reserve {(ws + inputs) / 1e9:.1f} GB up front; each problem allocates its own")
        return
    del r
    log(f"# reserved {(ws + inputs) / 1e9:.1f} GB of device memory for the run")


def copy_bandwidth(dev, nbytes=4 << 30, reps=10):
    """Device-to-device copy of nbytes (read + write) timed with HIP events:
    the bandwidth a plain streaming kernel reaches on this GPU."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (s.elapsed_time(e) * 1e-3) / 1e9
    del a, b
    return round(gbs, 1)


def kkt_course(log_, marks=(1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8), points=12):
    """From a solve's check log: the first time each relative KKT level was
    reached, and a dozen (seconds, iterations, rel_kkt) samples."""
    first = {}
    for e in log_:
        for mk in marks:
            if mk not in first and e["rel_kkt"] <= mk:
                first[mk] = [round(e["seconds"], 3), e["iter"]]
    step = max(1, len(log_) // points)
    samples = [[round(e["seconds"], 3), e["iter"], float(f"{e['rel_kkt']:.4g}")] for e in log_[step - 1::step]]
    if log_ and (not samples or samples[-1][1] != log_[-1]["iter"]):
        e = log_[-1]
        samples.append([round(e["seconds"], 3), e["iter"], float(f"{e['rel_kkt']:.4g}")])
    return {"first_reached_s_iter": {f"{mk:g}": v for mk, v in first.items()},
            "samples_s_iter_relkkt": samples}


def timed_solve(prob, time_limit, **kw):
    """One solve to 1e-8 under a time limit; status, KKT reached and its course."""
    import torch
    from paper_2507_14051_amd import STATUS_NAMES
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = prob.solve(tol=1e-8, time_limit_s=time_limit, want_r=False, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = out["info"]
    res = {"time_limit_s": time_limit, "status": STATUS_NAMES[info["status"]], "wall_s": round(wall, 3),
           "iters": info["iters"], "restarts": info["restarts"], "iters_per_s": round(info["iters"] / wall, 1),
           "rel_kkt": info["rel_kkt"], "rel_gap": info["rel_gap"], "rel_primal": info["rel_primal"],
           "rel_dual": info["rel_dual"], "omega": info["omega"],
           "time_to_tol_s": round(wall, 3) if info["status"] == 0 else None}
    res.update(kkt_course(out["log"]))
    return res, out["log"]


def half_step_roofline(prob, m, n, nnz, workload, profile_iters):
    """The dominant FP64 half-step of an LP against the HBM roofline.  A
    half-step is one launch unit: the transpose SpMV fused with the primal
    update (primal), or the SpMV fused with the dual update (dual), each of
    one or more kernels; its duration runs from the first kernel's start to
    the last kernel's end (HIP events taking the kernels' own timestamps on
    the library's stream, hlp_profile_iterations)."""
    prof = prob.profile(iters=profile_iters)
    pb, db = algorithmic_bytes(m, n, nnz)
    half = "primal" if prof["primal_ms"] >= prof["dual_ms"] else "dual"
    kms = prof[f"{half}_ms"]
    kbytes = pb if half == "primal" else db
    achieved = kbytes / (kms * 1e-3) / 1e9
    tr = load_traffic(workload, half)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (tr["traffic_bytes_per_launch"] if tr else None),
            "kernel": f"FP64 {half} half-step of {workload} "
                      f"({'transpose SpMV fused with the primal update' if half == 'primal' else 'SpMV fused with the dual update'})",
            "bytes_per_launch": kbytes, "avg_launch_us": round(kms * 1e3, 2),
            "primal_avg_us": round(prof["primal_ms"] * 1e3, 2), "dual_avg_us": round(prof["dual_ms"] * 1e3, 2),
            "primal_gbs": round(pb / (prof["primal_ms"] * 1e-3) / 1e9, 1),
            "dual_gbs": round(db / (prof["dual_ms"] * 1e-3) / 1e9, 1),
            "iteration_us": round(prof["iter_ms"] * 1e3, 2),
            "iteration_gbs": round((pb + db) / (prof["iter_ms"] * 1e-3) / 1e9, 1),
            "iteration_frac": round((pb + db) / (prof["iter_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "profiled_iterations": prof["iters"]}


def gen(name):
    import lpgen
    t0 = time.perf_counter()
    lp = lpgen.config(name, seed=1,
                      progress=lambda k, n: log(f"# {name}: rows chunk {k}/{n}") if k % 16 == 0 else None)
    log(f"# {name}: m={lp.m} n={lp.n} nnz={lp.nnz} max_row={lp.meta['max_row']} "
        f"rows_at_cap={lp.meta['rows_at_cap']} (generated in {time.perf_counter() - t0:.0f} s)")
    return lp


def measure_skewed(dev, lp, name, rate_iters, time_limit, profile_iters):
    """Iteration rate, half-step rooflines and a time-limited solve of a large
    skewed LP, in FP64 and in FP32 with refinement (same stepsize)."""
    import torch
    from paper_2507_14051_amd import MIXED, Problem
    t0 = time.perf_counter()
    p = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device=dev)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    _, _, eta, power_iters = p.scaling()
    out = {"workload": describe(name, lp), "setup_s": round(setup, 3), "power_iters": power_iters,
           "workspace_gb": round(p.workspace.numel() / 1e9, 2), "workspace_layout": p.layout,
           "column_panels": p.panels()[0], "long_rows": p.panels()[1], "narrow_panels": p.dense()[0],
           "dense_rows": p.dense()[1]}
    p.solve(max_iter=64, tol=1e-8, want_r=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.solve(max_iter=rate_iters, tol=1e-8, want_r=False)
    torch.cuda.synchronize()
    out["iters_per_s"] = round(rate_iters / (time.perf_counter() - t0), 1)
    out["roofline"] = half_step_roofline(p, lp.m, lp.n, lp.nnz, name, profile_iters)
    out["fp64_time_limited"], _ = timed_solve(p, time_limit)
    log(f"# {name} fp64: {out['iters_per_s']} iter/s; {out['fp64_time_limited']['status']} "
        f"rel_kkt {out['fp64_time_limited']['rel_kkt']:.3e}")
    p.close()
    del p
    pm = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device=dev, precision=MIXED, eta_override=eta)
    pm.solve(max_iter=64, tol=1e-8, want_r=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pm.solve(max_iter=rate_iters, tol=1e-8, want_r=False)
    torch.cuda.synchronize()
    itm = rate_iters / (time.perf_counter() - t0)
    prm = pm.profile(iters=profile_iters)
    tl, tlog = timed_solve(pm, time_limit)
    pm.close()
    del pm
    f64 = out["fp64_time_limited"]
    reach = next((e["seconds"] for e in tlog if e["rel_kkt"] <= f64["rel_kkt"]), None)
    out["fp32_refined"] = {"iters_per_s": round(itm, 1), "rate_vs_fp64": round(itm / out["iters_per_s"], 3),
                           "primal_us": round(prm["primal_ms"] * 1e3, 2), "dual_us": round(prm["dual_ms"] * 1e3, 2),
                           "time_limited": tl,
                           "time_to_fp64_final_kkt_s": round(reach, 3) if reach is not None else None}
    log(f"# {name} fp32: {itm:.1f} iter/s; {tl['status']} rel_kkt {tl['rel_kkt']:.3e}")
    return out


def measure_c2(dev, steps, profile_iters, with_cpu=True, cpu_iters=50):
    """The medium LP, whose ~38 MB working set stays in the 256 MB Infinity
    Cache: FP64 and FP32 solves to 1e-8 and the FP64 half-steps' rates
    (cache-resident, not HBM-bound); with_cpu: the oracle's time per
    iteration on the same LP (cpu_iters iterations after its own scaling, a
    fixed stepsize, one thread) and the time to 1e-8 it implies at the GPU's
    iteration count (extrapolated, not run)."""
    import torch
    import lpgen
    from paper_2507_14051_amd import MIXED, OPTIMAL, Problem
    lp = lpgen.config("c2", seed=1)
    p = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device=dev)
    p.solve(tol=1e-8, want_r=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [p.solve(tol=1e-8, want_r=False)["info"] for _ in range(steps)]
    torch.cuda.synchronize()
    t64 = (time.perf_counter() - t0) / steps
    rf = half_step_roofline(p, lp.m, lp.n, lp.nnz, "c2", profile_iters)
    rf["bound"] = "cache-resident (38 MB per iteration, inside the 256 MB Infinity Cache): latency and L2 requests"
    p.close()
    pm = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device=dev, precision=MIXED)
    pm.solve(tol=1e-8, want_r=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mi = [pm.solve(tol=1e-8, want_r=False)["info"] for _ in range(steps)]
    torch.cuda.synchronize()
    t32 = (time.perf_counter() - t0) / steps
    pm.close()
    out = {"workload": describe("c2", lp) + ", tol 1e-8",
           "fp64": {"time_to_tol_s": round(t64, 4), "iters": infos[-1]["iters"], "restarts": infos[-1]["restarts"],
                    "all_optimal": all(i["status"] == OPTIMAL for i in infos), "rel_kkt": infos[-1]["rel_kkt"],
                    "iters_per_s": round(infos[-1]["iters"] / t64, 1)},
           "fp32_refined": {"time_to_tol_s": round(t32, 4), "iters": mi[-1]["iters"],
                            "all_optimal": all(i["status"] == OPTIMAL for i in mi), "rel_kkt": mi[-1]["rel_kkt"],
                            "iters_per_s": round(mi[-1]["iters"] / t32, 1),
                            "time_to_tol_vs_fp64": round(t64 / t32, 3)},
           "half_steps": rf}
    if with_cpu:
        import oracle
        res = oracle.solve(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv,
                           oracle.Params(tol=0.0, max_iter=cpu_iters, eta_override=0.5))
        per_iter = res.info["iter_s"] / cpu_iters
        out["cpu_oracle"] = {"iter_ms": round(per_iter * 1e3, 3), "cores": 1, "kind": "oracle",
                             "time_to_tol_s_extrapolated": round(per_iter * infos[-1]["iters"], 1),
                             "gpu_fp64_speedup_to_tol": round(per_iter * infos[-1]["iters"] / t64, 1),
                             "sample": f"{cpu_iters} oracle iterations (NumPy/SciPy FP64, one thread) on the whole "
                                       f"LP after its own scaling ({res.info['setup_s']:.1f} s, not counted), "
                                       f"fixed stepsize; time to 1e-8 = time per iteration x the "
                                       f"{infos[-1]['iters']} iterations of the solve (not run)"}
    log(f"# c2: {out['fp64']} {out['fp32_refined']} {out.get('cpu_oracle')}")
    return out


def cpu_baseline(lp, name, rows_div=32, iters=32):
    """The FP64 CPU oracle as it stands on a bounded sample of the headline LP:
    the LP restricted to its first m/rows_div rows (rows are drawn
    independently, so the sample keeps the row-length law; all columns and
    their bounds kept), its own scaling (not timed), a fixed stepsize in place
    of its power iteration (hours at this size; the stepsize does not change
    the work per iteration), then `iters` iterations; the time per iteration
    is scaled to the full LP by the ratio of the algorithmic bytes per
    iteration (24 nnz + 68 n + 52 m)."""
    import oracle
    import lpgen
    r = lp.m // rows_div
    A = lp.A[:r]
    sub = lpgen.LP(A=A, c=lp.c, lc=lp.lc[:r], uc=lp.uc[:r], lv=lp.lv, uv=lp.uv)
    res = oracle.solve(sub.A, sub.c, sub.lc, sub.uc, sub.lv, sub.uv,
                       oracle.Params(tol=0.0, max_iter=iters, eta_override=0.5))
    per_iter = res.info["iter_s"] / iters
    full = 24 * lp.nnz + 68 * lp.n + 52 * lp.m
    part = 24 * A.nnz + 68 * lp.n + 52 * r
    value = 1.0 / (per_iter * full / part)
    return {"value": round(value, 4), "unit": "iter/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} oracle iterations (NumPy/SciPy FP64, one thread) on the first {r} rows of the "
                      f"{name} LP ({A.nnz} nonzeros, all {lp.n} columns) after its own scaling "
                      f"({res.info['setup_s']:.1f} s, not counted) with a fixed stepsize; "
                      f"{per_iter:.3f} s per iteration scaled by the algorithmic bytes ratio {full / part:.2f} "
                      f"to the full LP; host nproc={os.cpu_count()}"}


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


def measure_ablation(dev, max_iter=600000, c1_seeds=8, c3b_time_limit=30.0):
    """Iterations to 1e-8 relative KKT under each switch: the medium LP (seed
    1) and the geometric mean over c1_seeds small LPs, relative to the
    paper's settings; and on the skewed LP of ~3e7 nonzeros, which none of
    the switches solves to 1e-8 in minutes, the relative KKT reached in
    c3b_time_limit seconds.  One handle per LP, so every variant takes the
    same scaling and stepsize."""
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
    lp = gen("c3b")
    prob = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device=dev)
    big = {}
    for name, kw in ABLATIONS.items():
        res, _ = timed_solve(prob, c3b_time_limit, **kw)
        big[name] = {k: res[k] for k in ("status", "iters", "restarts", "rel_kkt", "rel_gap", "rel_primal",
                                         "rel_dual", "omega", "first_reached_s_iter")}
        log(f"# ablation c3b {name}: {big[name]}")
    prob.close()
    return {"tol": 1e-8, "max_iter": max_iter, "c2_seed1": med, f"c1_seeds_1_to_{c1_seeds}": geo,
            f"c3b_full_size_{c3b_time_limit:g}s": {"workload": describe("c3b", lp), "by_switch": big}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--step-iters", type=int, default=256,
                    help="PDHG iterations per step (one capped FP64 solve of the headline LP)")
    ap.add_argument("--time-limit", type=float, default=45.0,
                    help="seconds of the time-limited headline solves (FP64 and FP32 with refinement)")
    ap.add_argument("--time-limit-c3b", type=float, default=30.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline LP (no c3b, c2, adjoint)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiation workload")
    ap.add_argument("--profile-iters", type=int, default=50)
    ap.add_argument("--kernels-only", action="store_true",
                    help="only time the half-steps of --kernels-workload and a 256 MiB copy (for counter runs)")
    ap.add_argument("--kernels-workload", default=HEADLINE, choices=("c2", "c3b", "c3a"))
    ap.add_argument("--ablation", action="store_true",
                    help="only the iterations-to-tolerance of the method's switches (reflection, primal weight, "
                         "restart tests)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the build targets a single MI355X); "
                                   "--gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2507_14051_amd import MIXED, Problem

    dev = torch.device("cuda:0")
    if args.ablation:
        print(json.dumps({"ablation": measure_ablation(dev)}), flush=True)
        return
    if args.kernels_only:
        lp = gen(args.kernels_workload)
        prob = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device=dev)
        prof = prob.profile(iters=args.profile_iters)
        pb, db = algorithmic_bytes(lp.m, lp.n, lp.nnz)
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)   # 256 MiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"kernels_only": True, "workload": args.kernels_workload,
                          "primal_us": prof["primal_ms"] * 1e3, "dual_us": prof["dual_ms"] * 1e3,
                          "iters": prof["iters"], "primal_bytes": pb, "dual_bytes": db,
                          "copy_bytes": 2 * a.numel() * 8, "kernel_source_hash": kernel_source_hash()}), flush=True)
        prob.close()
        return

    # ---------------------------------------------------------------- headline
    lp = gen(HEADLINE)
    reserve_device_memory(dev, lp)
    m, n, nnz = lp.m, lp.n, lp.nnz
    workload = describe(HEADLINE, lp)
    t0 = time.perf_counter()
    prob = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device=dev)
    torch.cuda.synchronize()
    setup_wall = time.perf_counter() - t0
    _, _, eta, power_iters = prob.scaling()
    workspace_gb = round(prob.workspace.numel() / 1e9, 2)
    log(f"# {HEADLINE}: setup {setup_wall:.2f} s (power iterations {power_iters}), panels {prob.panels()}, "
        f"dense {prob.dense()}, workspace {workspace_gb} GB ({prob.layout} layout)")
    for _ in range(args.warmup):
        prob.solve(tol=1e-8, max_iter=args.step_iters, want_r=False)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(prob.solve(tol=1e-8, max_iter=args.step_iters, want_r=False)["info"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    iters = sum(i["iters"] for i in infos)
    ms_per_step = 1e3 * elapsed / args.steps
    log(f"# {HEADLINE} steps: {iters / elapsed:.1f} iter/s, {ms_per_step:.1f} ms per step")
    prob_layout = prob.layout
    roofline = half_step_roofline(prob, m, n, nnz, HEADLINE, args.profile_iters)
    fp64_tl, _ = timed_solve(prob, args.time_limit)
    log(f"# {HEADLINE} fp64 time-limited: {fp64_tl['status']} rel_kkt {fp64_tl['rel_kkt']:.3e}")
    prob.close()
    del prob
    pm = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device=dev, precision=MIXED, eta_override=eta)
    pm.solve(max_iter=64, tol=1e-8, want_r=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pm.solve(max_iter=args.step_iters, tol=1e-8, want_r=False)
    torch.cuda.synchronize()
    rate32 = args.step_iters / (time.perf_counter() - t0)
    fp32_tl, f32log = timed_solve(pm, args.time_limit)
    pm.close()
    del pm
    reach = next((e["seconds"] for e in f32log if e["rel_kkt"] <= fp64_tl["rel_kkt"]), None)
    mixed = {"iters_per_s": round(rate32, 1), "rate_vs_fp64": round(rate32 / (iters / elapsed), 3),
             "time_limited": fp32_tl,
             "time_to_fp64_final_kkt_s": round(reach, 3) if reach is not None else None}
    log(f"# {HEADLINE} fp32 time-limited: {fp32_tl['status']} rel_kkt {fp32_tl['rel_kkt']:.3e}")
    copy_gbs = copy_bandwidth(dev)
    roofline["copy_peak_gbs"] = copy_gbs
    roofline["frac_of_copy_peak"] = round(roofline["achieved"] / copy_gbs, 4)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(lp, HEADLINE)
        log(f"# cpu: {cpu}")
    del lp

    extra = {}
    if not args.no_extra:
        extra["c3b"] = measure_skewed(dev, gen("c3b"), "c3b", 640, args.time_limit_c3b, args.profile_iters)
        extra["c2_cache_resident"] = measure_c2(dev, 2, 400, with_cpu=not args.no_cpu)
        if not args.no_adjoint:
            extra["adjoint"] = measure_adjoint(dev)

    line = {
        "metric": "PDHG iterations/s of FP64 restarted Halpern PDHG (time to 1e-8 relative KKT, FP32-vs-FP64 and "
                  "the HBM roofline alongside)",
        "value": round(iters / elapsed, 2), "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": workload,
                   "step": f"one FP64 solve from the all-zero start, paper settings, tol 1e-8, capped at "
                           f"{args.step_iters} iterations (a check every 64)",
                   "seed": 1, "global_batch": 1, "parallelism": "single GPU"},
        "setup_s": round(setup_wall, 3), "power_iters": power_iters, "eta": eta, "workspace_gb": workspace_gb,
        "workspace_layout": prob_layout,
        "time_to_tol_s": fp64_tl["time_to_tol_s"], "fp64_time_limited": fp64_tl, "mixed": mixed,
        "roofline": roofline, "cpu_baseline": cpu, **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
