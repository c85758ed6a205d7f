"""Helpers for the GPU parity tests: run the HIP library and the oracle on the
same seeded inputs and compare."""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def oracle_eta(lp, ruiz_iters=10, pock_chambolle=1):
    """eta = 0.998 / ||A~||_2 from the oracle's own scaling and power iteration.

    Comparisons of iterates feed this one stepsize to both sides (the GPU takes
    it as eta_override), so they do not depend on where each power iteration
    stops; the GPU's power iteration is compared with the oracle's separately."""
    key = ("_oracle_eta", ruiz_iters, pock_chambolle)
    cached = getattr(lp, "_eta_cache", {})
    if key not in cached:
        from oracle.pdhg import power_norm, rescale
        At, _, _ = rescale(lp.A, ruiz_iters, pock_chambolle)
        nrm, _ = power_norm(At, 5000, 1e-8)
        cached[key] = 0.998 / nrm if nrm > 0 else 1.0
        lp._eta_cache = cached
    return cached[key]


def problem(lp, eta=None, layout="auto", **setup):
    """The GPU handle for lp; eta (if given) replaces the GPU's power iteration."""
    from paper_2507_14051_amd import Problem
    if eta is not None:
        setup["eta_override"] = eta
    return Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device="cuda:0", layout=layout, **setup)


def np_out(out):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items() if k != "trace"}


def announce(msg):
    print(msg, flush=True)
