"""hlp_solve_static (setup + solve on the library's static device scratch, for
callers that cannot allocate) against hlp_lp_create + hlp_solve on a
caller-provided workspace: bitwise the same outputs, on two calls in a row,
the second on a smaller LP (the scratch keeps the first call's contents), and
a clean HLP_ENOMEM for an LP that does not fit."""
import numpy as np
import pytest

import lpgen
import oracle
from tests._gpu import announce

pytestmark = pytest.mark.gpu


def _device_inputs(lp):
    import torch
    dev = "cuda:0"
    A = lp.A.tocsr()
    f64 = dict(dtype=torch.float64, device=dev)
    return dict(row_ptr=torch.as_tensor(A.indptr.astype(np.int64), device=dev),
                col_idx=torch.as_tensor(A.indices.astype(np.int32), device=dev),
                val=torch.as_tensor(A.data, **f64),
                vecs=[torch.as_tensor(v, **f64) for v in (lp.c, lp.lc, lp.uc, lp.lv, lp.uv)])


def _static(lp, **kw):
    import torch
    from paper_2507_14051_amd.hlp import hlp_params_default, hlp_solve_static
    d = _device_inputs(lp)
    f64 = dict(dtype=torch.float64, device="cuda:0")
    x, y, r = torch.empty(lp.n, **f64), torch.empty(lp.m, **f64), torch.empty(lp.n, **f64)
    info = hlp_solve_static(lp.m, lp.n, lp.nnz, d["row_ptr"], d["col_idx"], d["val"], *d["vecs"],
                            params=hlp_params_default(**kw), x=x, y=y, r=r)
    torch.cuda.synchronize()
    return x.cpu().numpy(), y.cpu().numpy(), r.cpu().numpy(), info.as_dict()


def _handle(lp, **kw):
    from paper_2507_14051_amd import SETUP_FIELDS, Problem
    setup = {k: v for k, v in kw.items() if k in SETUP_FIELDS}
    solve = {k: v for k, v in kw.items() if k not in SETUP_FIELDS}
    prob = Problem(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, device="cuda:0", **setup)
    out = prob.solve(graphs=0, **solve)
    prob.close()
    return out["x"].cpu().numpy(), out["y"].cpu().numpy(), out["r"].cpu().numpy(), out["info"]


@pytest.mark.parametrize("layout", ["plain", "panels"])
def test_static_solve_matches_handle_solve_twice_second_smaller(layout):
    kw = dict(tol=1e-8)
    if layout == "panels":
        kw.update(column_panels=8, panel_row_min=3, dense_row_min=5)
    for tag, lp in (("c1 seed 1", lpgen.config("c1", seed=1)), ("c1 seed 2 scaled 0.3", lpgen.config("c1", seed=2, scale=0.3))):
        announce(f"static solve {layout} {tag} m={lp.m} n={lp.n} nnz={lp.nnz}")
        xs, ys, rs, si = _static(lp, **kw)
        xh, yh, rh, hi = _handle(lp, **kw)
        assert np.array_equal(xs, xh) and np.array_equal(ys, yh) and np.array_equal(rs, rh), tag
        for key in ("status", "iters", "restarts", "checks", "rel_kkt", "pobj", "dobj", "omega", "eta"):
            assert si[key] == hi[key], (tag, key, si[key], hi[key])
        assert si["status"] == oracle.pdhg.OPTIMAL
        k = oracle.kkt(lp.A, lp.c, lp.lc, lp.uc, lp.lv, lp.uv, xs, ys)
        assert k["rel_kkt"] <= 1e-8 * (1 + 1e-6)


def test_static_solve_rejects_an_lp_beyond_the_scratch():
    from paper_2507_14051_amd.hlp import HLP_ENOMEM, HlpError, hlp_params_default, hlp_solve_static
    announce("static solve: LP beyond the scratch")
    # the size check runs before any pointer is used or any device work is issued
    with pytest.raises(HlpError) as e:
        hlp_solve_static(2_000_000, 5_000_000, 30_000_000, None, None, None, None, None, None, None, None,
                         params=hlp_params_default())
    assert e.value.code == HLP_ENOMEM and "static scratch" in str(e.value)
