"""Restarted reflected Halpern PDHG for LP on one AMD MI355X (gfx950).

The solver is the C-ABI library libhlp.so (HIP kernels + host controller);
this package only marshals arguments.  PyTorch provides device memory and the
stream.  See include/hlp.h for the contract of every entry point.

    from paper_2507_14051_amd import Problem
    prob = Problem(A_csr, c, lc, uc, lv, uv)          # setup on the GPU
    out = prob.solve(tol=1e-8)                         # dict: x, y, r (torch), info
"""
from __future__ import annotations

import numpy as np

from .hlp import (FP64, MIXED, HLP_OK, ITER_LIMIT, NUMERICAL, OPTIMAL, STATUS_NAMES, SYMBOLS, TIME_LIMIT,
                  HlpCheck, HlpError, HlpInfo, HlpParams, hlp_check_log, hlp_last_error, hlp_lp_create, hlp_lp_destroy,
                  hlp_lp_panels, hlp_lp_scaling, hlp_lp_transpose, hlp_lp_update_vectors, hlp_params_default,
                  hlp_profile_iterations, hlp_solve, hlp_tape_bytes, hlp_unrolled_backward,
                  hlp_unrolled_forward, hlp_workspace_bytes, hlp_workspace_bytes_csr, lib)

__all__ = ["Problem", "solve", "HlpError", "FP64", "MIXED", "OPTIMAL", "ITER_LIMIT", "TIME_LIMIT",
           "NUMERICAL", "STATUS_NAMES", "hlp_params_default"]

SETUP_FIELDS = ("precision", "eta_override", "ruiz_iters", "pock_chambolle", "power_max_iter", "power_tol",
                "stream_matrix", "column_panels", "panel_row_min", "dense_row_min")


def _dev_tensor(a, dtype, device):
    import torch
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


def _aligned_bytes(nbytes, device, align=256):
    import torch
    buf = torch.empty(nbytes + align, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % align
    return buf, buf[off:off + nbytes]


class Problem:
    """An LP held on the GPU: CSR and vectors as torch tensors, the library
    workspace and the handle built by hlp_lp_create (setup runs here)."""

    def __init__(self, A, c, lc, uc, lv, uv, device="cuda", stream=None, layout="auto", **setup):
        import torch
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the solver runs on the GPU only")
        self.stream = stream
        if hasattr(A, "indptr"):
            A = A.tocsr()
            m, n = A.shape
            rp, ci, va = A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64)
        else:
            (rp, ci, va), (m, n) = A
        self.m, self.n = int(m), int(n)
        self.row_ptr = _dev_tensor(rp, torch.int64, self.device)
        self.col_idx = _dev_tensor(ci, torch.int32, self.device)
        self.val = _dev_tensor(va, torch.float64, self.device)
        self.nnz = int(self.col_idx.numel())
        self.vectors = [_dev_tensor(v, torch.float64, self.device) for v in (c, lc, uc, lv, uv)]
        bad = set(setup) - set(SETUP_FIELDS)
        if bad:
            raise TypeError(f"not setup parameters: {sorted(bad)}")
        self.setup = dict(setup)
        self.params = hlp_params_default(**self.setup)
        self.precision = self.params.precision
        # layout: "rows" sizes the column-panel layout for this matrix's rows
        # (hlp_workspace_bytes_csr), "worst" for any rows of its size
        # (hlp_workspace_bytes); "auto" takes the worst-case layout when it
        # fits in three quarters of the free device memory, counting what
        # torch's cache holds unused (on the 692M-nonzero LP it runs the primal
        # half-step 6-7% faster, measured), else the row-sized one.
        worst = hlp_workspace_bytes(self.m, self.n, self.nnz, self.params)
        if layout not in ("auto", "rows", "worst"):
            raise ValueError("layout must be 'auto', 'rows' or 'worst'")
        if layout == "auto":
            free, _ = torch.cuda.mem_get_info(self.device)
            # memory torch holds in its cache but does not use is free for us too
            free += torch.cuda.memory_reserved(self.device) - torch.cuda.memory_allocated(self.device)
            layout = "worst" if worst <= 0.75 * free else "rows"
        if layout == "rows":
            rp_host = rp.cpu().numpy() if hasattr(rp, "cpu") else np.asarray(rp)
            nbytes = hlp_workspace_bytes_csr(self.m, self.n, self.nnz, rp_host, self.params)
        else:
            nbytes = worst
        self.layout = layout
        self._ws_base, self.workspace = _aligned_bytes(nbytes, self.device)
        self.handle = hlp_lp_create(self.m, self.n, self.nnz, self.row_ptr, self.col_idx, self.val,
                                    *self.vectors, self.params, self.workspace, stream)

    def close(self):
        if getattr(self, "handle", None) is not None:
            hlp_lp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params_for(self, **kw) -> HlpParams:
        return hlp_params_default(**{**self.setup, **kw})

    def update_vectors(self, c, lc, uc, lv, uv):
        import torch
        self.vectors = [_dev_tensor(v, torch.float64, self.device) for v in (c, lc, uc, lv, uv)]
        hlp_lp_update_vectors(self.handle, *self.vectors)

    def solve(self, x0=None, y0=None, trace_iters=0, want_r=True, **params):
        """Run hlp_solve; returns dict(x, y, r, info, log, trace): torch tensors, the
        info dict and the check log (hlp_check_log, a list of dicts)."""
        import torch
        p = self.params_for(trace_iters=trace_iters, **params)
        f64 = dict(dtype=torch.float64, device=self.device)
        x = torch.empty(self.n, **f64)
        y = torch.empty(self.m, **f64)
        r = torch.empty(self.n, **f64) if want_r else None
        trace = torch.empty(max(trace_iters, 0) * (2 * self.n + 2 * self.m), **f64) if trace_iters else None
        x0 = None if x0 is None else _dev_tensor(x0, torch.float64, self.device)
        y0 = None if y0 is None else _dev_tensor(y0, torch.float64, self.device)
        info = hlp_solve(self.handle, p, x0, y0, x, y, r, trace)
        out = dict(x=x, y=y, r=r, info=info.as_dict(), log=hlp_check_log(self.handle))
        if trace is not None:
            T = trace.view(trace_iters, 2 * self.n + 2 * self.m)
            n, m = self.n, self.m
            out["trace"] = dict(xh=T[:, :n], yh=T[:, n:n + m], x=T[:, n + m:2 * n + m], y=T[:, 2 * n + m:])
        return out

    def scaling(self):
        import torch
        dr = torch.empty(self.m, dtype=torch.float64, device=self.device)
        dc = torch.empty(self.n, dtype=torch.float64, device=self.device)
        eta, it = hlp_lp_scaling(self.handle, dr, dc)
        return dr, dc, eta, it

    def transpose(self):
        import torch
        cp = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        ri = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        tv = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        hlp_lp_transpose(self.handle, cp, ri, tv)
        return cp, ri, tv

    def panels(self):
        """(panel count, long rows) of the column-panel layout; (0, 0) if unused."""
        return hlp_lp_panels(self.handle)[:2]

    def dense(self):
        """(narrow panel count, dense rows) of the LDS-staged layout; (0, 0) if unused."""
        return hlp_lp_panels(self.handle)[2:]

    def profile(self, iters=200, **params):
        return hlp_profile_iterations(self.handle, self.params_for(**params), iters)


def solve(A, c, lc, uc, lv, uv, device="cuda", **params):
    """One-call convenience: copy to the GPU, set up, solve; numpy outputs."""
    setup = {k: params.pop(k) for k in list(params) if k in SETUP_FIELDS}
    prob = Problem(A, c, lc, uc, lv, uv, device=device, layout=params.pop("layout", "auto"), **setup)
    try:
        out = prob.solve(**params)
        return (out["x"].cpu().numpy(), out["y"].cpu().numpy(), out["r"].cpu().numpy(), out["info"])
    finally:
        prob.close()
