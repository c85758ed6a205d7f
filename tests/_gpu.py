"""Helpers for the GPU parity tests: run the HIP library and the oracle on the
same seeded inputs and compare."""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def problem(lp, **setup):
    from paper_2507_14051_amd import Problem
    return Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device="cuda:0", **setup)


def np_out(out):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items() if k != "trace"}


def announce(msg):
    print(msg, flush=True)
