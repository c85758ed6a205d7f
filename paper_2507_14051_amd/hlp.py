"""ctypes binding of libhlp.so, one Python function per C entry point.

Argument marshalling only: torch tensors are passed as raw device pointers
and the torch stream as a hipStream_t.  Every step of the solver runs in the
HIP library; this module raises if the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhlp.so")

HLP_OK, HLP_EINVAL, HLP_ENOMEM, HLP_EHIP, HLP_EUNSUPPORTED = 0, -1, -2, -3, -4
OPTIMAL, ITER_LIMIT, TIME_LIMIT, NUMERICAL = 0, 1, 2, 3
FP64, MIXED = 0, 1
STATUS_NAMES = {OPTIMAL: "OPTIMAL", ITER_LIMIT: "ITER_LIMIT", TIME_LIMIT: "TIME_LIMIT", NUMERICAL: "NUMERICAL"}

# The exported symbols, in the order of include/hlp.h.
SYMBOLS = ("hlp_params_default", "hlp_workspace_bytes", "hlp_workspace_bytes_csr", "hlp_lp_create",
           "hlp_lp_update_vectors", "hlp_solve", "hlp_check_log", "hlp_lp_scaling", "hlp_lp_transpose",
           "hlp_lp_panels", "hlp_tape_bytes", "hlp_unrolled_forward", "hlp_unrolled_backward",
           "hlp_profile_iterations", "hlp_solve_static", "hlp_lp_destroy", "hlp_last_error")


class HlpParams(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("max_iter", C.c_int64), ("time_limit_s", C.c_double),
        ("eval_freq", C.c_int32), ("precision", C.c_int32),
        ("gamma", C.c_double), ("beta_sufficient", C.c_double), ("beta_necessary", C.c_double),
        ("beta_artificial", C.c_double), ("kp", C.c_double), ("ki", C.c_double), ("kd", C.c_double),
        ("omega0", C.c_double), ("eta_override", C.c_double),
        ("ruiz_iters", C.c_int32), ("pock_chambolle", C.c_int32), ("power_max_iter", C.c_int32),
        ("restart_to_current", C.c_int32), ("power_tol", C.c_double), ("pid_min_norm", C.c_double),
        ("trace_iters", C.c_int32), ("debug_poison_iter", C.c_int32), ("graphs", C.c_int32),
        ("stream_matrix", C.c_int32), ("column_panels", C.c_int32), ("panel_row_min", C.c_int32),
        ("dense_row_min", C.c_int32),
    ]


class HlpInfo(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("power_iters", C.c_int32), ("iters", C.c_int64), ("restarts", C.c_int64),
        ("checks", C.c_int64), ("rel_kkt", C.c_double), ("rel_gap", C.c_double),
        ("rel_primal", C.c_double), ("rel_dual", C.c_double), ("pobj", C.c_double), ("dobj", C.c_double),
        ("omega", C.c_double), ("eta", C.c_double), ("setup_s", C.c_double), ("solve_s", C.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class HlpCheck(C.Structure):
    _fields_ = [
        ("iter", C.c_int64), ("k", C.c_int64), ("r", C.c_double), ("r0", C.c_double),
        ("rel_kkt", C.c_double), ("rel_gap", C.c_double), ("rel_primal", C.c_double), ("rel_dual", C.c_double),
        ("omega", C.c_double), ("seconds", C.c_double), ("restart", C.c_int32), ("reserved", C.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class HlpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hlp error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libhlp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python -m paper_2507_14051_amd.build")
        L = C.CDLL(LIB_PATH)
        P, I64, I32, SZ = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
        L.hlp_params_default.argtypes = [C.POINTER(HlpParams)]
        L.hlp_workspace_bytes.argtypes = [I32, I32, I64, C.POINTER(HlpParams), C.POINTER(SZ)]
        L.hlp_workspace_bytes_csr.argtypes = [I32, I32, I64, P, C.POINTER(HlpParams), C.POINTER(SZ)]
        L.hlp_lp_create.argtypes = [I32, I32, I64] + [P] * 8 + [C.POINTER(HlpParams), P, SZ, P, C.POINTER(P)]
        L.hlp_lp_update_vectors.argtypes = [P] * 6
        L.hlp_solve.argtypes = [P, C.POINTER(HlpParams), P, P, P, P, P, C.POINTER(HlpInfo), P]
        L.hlp_check_log.argtypes = [P, C.POINTER(HlpCheck), I64, C.POINTER(I64)]
        L.hlp_lp_scaling.argtypes = [P, P, P, C.POINTER(C.c_double), C.POINTER(I32)]
        L.hlp_lp_transpose.argtypes = [P, P, P, P]
        L.hlp_lp_panels.argtypes = [P] + [C.POINTER(I32)] * 4
        L.hlp_tape_bytes.argtypes = [P, I32, I32, C.POINTER(SZ)]
        L.hlp_unrolled_forward.argtypes = [P, C.POINTER(HlpParams), I32, I32, I32, P, P, P, P, P, SZ]
        L.hlp_unrolled_backward.argtypes = [P, P, SZ] + [P] * 7
        L.hlp_profile_iterations.argtypes = [P, C.POINTER(HlpParams), I32, C.POINTER(C.c_double)]
        L.hlp_solve_static.argtypes = [I32, I32, I64] + [P] * 8 + [C.POINTER(HlpParams), P, P, P, P,
                                                                   C.POINTER(HlpInfo)]
        L.hlp_lp_destroy.argtypes = [P]
        L.hlp_lp_destroy.restype = None
        L.hlp_last_error.argtypes = []
        L.hlp_last_error.restype = C.c_char_p
        for name in SYMBOLS[:-2]:
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(code):
    if code != HLP_OK:
        raise HlpError(code, lib().hlp_last_error().decode())


def _ptr(t):
    """Raw device pointer of a torch tensor (or None -> NULL)."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# --------------------------------------------------------------------------- entry points
def hlp_params_default(**overrides) -> HlpParams:
    p = HlpParams()
    _check(lib().hlp_params_default(C.byref(p)))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def hlp_workspace_bytes(m, n, nnz, params=None) -> int:
    out = C.c_size_t(0)
    _check(lib().hlp_workspace_bytes(m, n, nnz, C.byref(params) if params is not None else None, C.byref(out)))
    return out.value


def hlp_workspace_bytes_csr(m, n, nnz, row_ptr, params=None) -> int:
    """Workspace for this matrix (row_ptr: host int64 array of m + 1 row pointers)."""
    import numpy as np
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    if rp.size != m + 1:
        raise ValueError("row_ptr must hold m + 1 entries")
    out = C.c_size_t(0)
    _check(lib().hlp_workspace_bytes_csr(m, n, nnz, rp.ctypes.data_as(C.c_void_p),
                                         C.byref(params) if params is not None else None, C.byref(out)))
    return out.value


def hlp_lp_create(m, n, nnz, row_ptr, col_idx, val, c, lc, uc, lv, uv, params, workspace, stream=None):
    h = C.c_void_p()
    _check(lib().hlp_lp_create(m, n, nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(val), _ptr(c), _ptr(lc),
                               _ptr(uc), _ptr(lv), _ptr(uv), C.byref(params) if params is not None else None,
                               _ptr(workspace), workspace.numel() * workspace.element_size(),
                               _stream(stream), C.byref(h)))
    return h


def hlp_lp_update_vectors(lp, c, lc, uc, lv, uv):
    _check(lib().hlp_lp_update_vectors(lp, _ptr(c), _ptr(lc), _ptr(uc), _ptr(lv), _ptr(uv)))


def hlp_solve(lp, params, x0=None, y0=None, x=None, y=None, r=None, trace=None) -> HlpInfo:
    info = HlpInfo()
    _check(lib().hlp_solve(lp, C.byref(params) if params is not None else None, _ptr(x0), _ptr(y0), _ptr(x),
                           _ptr(y), _ptr(r), C.byref(info), _ptr(trace)))
    return info


def hlp_check_log(lp) -> list:
    """The check log of the last hlp_solve on lp, as a list of dicts."""
    count = C.c_int64(0)
    _check(lib().hlp_check_log(lp, None, 0, C.byref(count)))
    buf = (HlpCheck * max(count.value, 1))()
    _check(lib().hlp_check_log(lp, buf, count.value, C.byref(count)))
    return [buf[i].as_dict() for i in range(count.value)]


def hlp_lp_scaling(lp, d_r=None, d_c=None):
    eta = C.c_double(0.0)
    it = C.c_int32(0)
    _check(lib().hlp_lp_scaling(lp, _ptr(d_r), _ptr(d_c), C.byref(eta), C.byref(it)))
    return eta.value, it.value


def hlp_lp_panels(lp):
    """(panels, long rows, dense panels, dense rows)."""
    v = [C.c_int32(0) for _ in range(4)]
    _check(lib().hlp_lp_panels(lp, *[C.byref(x) for x in v]))
    return tuple(x.value for x in v)


def hlp_lp_transpose(lp, col_ptr=None, row_idx=None, val=None):
    _check(lib().hlp_lp_transpose(lp, _ptr(col_ptr), _ptr(row_idx), _ptr(val)))


def hlp_tape_bytes(lp, K, ckpt_every) -> int:
    out = C.c_size_t(0)
    _check(lib().hlp_tape_bytes(lp, K, ckpt_every, C.byref(out)))
    return out.value


def hlp_unrolled_forward(lp, params, K, ckpt_every, replay, x0, y0, x, y, tape):
    _check(lib().hlp_unrolled_forward(lp, C.byref(params) if params is not None else None, K, ckpt_every,
                                      int(replay), _ptr(x0), _ptr(y0), _ptr(x), _ptr(y), _ptr(tape),
                                      tape.numel() * tape.element_size()))


def hlp_unrolled_backward(lp, tape, gx, gy, gc, glc, guc, glv, guv):
    _check(lib().hlp_unrolled_backward(lp, _ptr(tape), tape.numel() * tape.element_size(), _ptr(gx), _ptr(gy),
                                       _ptr(gc), _ptr(glc), _ptr(guc), _ptr(glv), _ptr(guv)))


def hlp_profile_iterations(lp, params, iters):
    out = (C.c_double * 4)()
    _check(lib().hlp_profile_iterations(lp, C.byref(params) if params is not None else None, iters, out))
    return dict(primal_ms=out[0], dual_ms=out[1], iter_ms=out[2], iters=int(out[3]))


def hlp_solve_static(m, n, nnz, row_ptr, col_idx, val, c, lc, uc, lv, uv, params=None, stream=None,
                     x=None, y=None, r=None) -> HlpInfo:
    """Setup and solve in one call on the library's static device scratch
    (no device allocation inside; see include/hlp.h)."""
    info = HlpInfo()
    _check(lib().hlp_solve_static(m, n, nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(val), _ptr(c), _ptr(lc),
                                  _ptr(uc), _ptr(lv), _ptr(uv), C.byref(params) if params is not None else None,
                                  _stream(stream), _ptr(x), _ptr(y), _ptr(r), C.byref(info)))
    return info


def hlp_lp_destroy(lp):
    lib().hlp_lp_destroy(lp)


def hlp_last_error() -> str:
    return lib().hlp_last_error().decode()
